"""Successive fixing around the LP solver (Section IV): Round, the logic-driven
Fixing-Strategy of Algorithm 1, a minimal LP presolve, and the batch of reduced LPs that
successive-fixing rounds hand to the solver.

Host-side support code: it decides which binaries are fixed and rewrites the LP; it holds
none of the LP iteration's arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import scuc
from .scuc import LP, U, V, W


def round_tau(s, tau: float):
    """Round(s, tau) of Section IV-A: 1 if s >= 1 - tau, 0 if 0 <= s <= tau, else -1."""
    s = np.asarray(s, dtype=float)
    out = np.full(s.shape, -1, dtype=np.int8)
    out[(s >= 0.0) & (s <= tau)] = 0
    out[s >= 1.0 - tau] = 1
    return out


def fixing_strategy(u, v, w, tau: float):
    """Algorithm 1 for relaxed values u, v, w of shape [G, T] (hours 0-based).

    Per generator: round every hour; then for t = 2..T (1-based) stop at the first hour where
    one of Round(u_t), Round(u_{t-1}), Round(v_t), Round(w_t) is -1 or where the rounded
    values break u_t - u_{t-1} = v_t - w_t or v_t + w_t <= 1; every hour before that stop is
    fixed to its rounded (u, v, w). Hour 1 is never fixed (the loop starts at t = 2).
    Returns (fixed [G, T] bool, ur, vr, wr rounded values as int8).
    """
    ur, vr, wr = round_tau(u, tau), round_tau(v, tau), round_tau(w, tau)
    G, T = ur.shape
    fixed = np.zeros((G, T), dtype=bool)
    for g in range(G):
        for t in range(1, T):
            if ur[g, t] < 0 or ur[g, t - 1] < 0 or vr[g, t] < 0 or wr[g, t] < 0:
                break
            if ur[g, t] - ur[g, t - 1] == vr[g, t] - wr[g, t] and vr[g, t] + wr[g, t] <= 1:
                fixed[g, t] = True
            else:
                break
    return fixed, ur, vr, wr


def gather_binaries(x, G: int, T: int):
    """(u, v, w) of shape [G, T] from an LP point with the hour-major column order."""
    t = np.arange(T)[None, :]
    g = np.arange(G)[:, None]
    return (x[scuc.col_index(G, t, U, g)], x[scuc.col_index(G, t, V, g)], x[scuc.col_index(G, t, W, g)])


def fix_bounds(lp: LP, G: int, T: int, fixed, ur, vr, wr):
    """Fix(M, S, s): column bounds with the fixed (u, v, w) set to their rounded values."""
    lo, hi = lp.col_lo.copy(), lp.col_hi.copy()
    gg, tt = np.nonzero(fixed)
    for var, vals in ((U, ur), (V, vr), (W, wr)):
        cols = scuc.col_index(G, tt, var, gg)
        lo[cols] = vals[gg, tt]
        hi[cols] = vals[gg, tt]
    return lo, hi


@dataclass
class Presolved:
    lp: LP                 # the reduced LP
    cols: np.ndarray       # kept original columns
    rows: np.ndarray       # kept original rows
    x_fixed: np.ndarray    # values of the removed columns (original indexing, NaN where kept)
    feasible: bool         # no removed empty row violates its bounds


def presolve_fixed(lp: LP, tol: float = 1e-9) -> Presolved:
    """LP presolve of fixed columns: every column with equal bounds is substituted out
    (its contribution moves to the row bounds and the objective offset), and rows left
    without entries are dropped after checking that 0 lies within their shifted bounds."""
    fixed = lp.col_lo == lp.col_hi
    A = lp.to_scipy()
    xf = np.where(fixed, lp.col_lo, 0.0)
    shift = A @ xf
    keep_c = np.nonzero(~fixed)[0]
    Ak = A[:, keep_c].tocsr()
    lo = lp.row_lo - shift
    hi = lp.row_hi - shift
    nz = np.diff(Ak.indptr) > 0
    empty = ~nz
    ok = bool(np.all(lo[empty] <= tol * (1 + np.abs(lo[empty]))) and np.all(hi[empty] >= -tol * (1 + np.abs(hi[empty]))))
    keep_r = np.nonzero(nz)[0]
    Ak = Ak[keep_r].tocsr()
    Ak.sort_indices()
    red = LP(len(keep_r), len(keep_c), Ak.indptr.astype(np.int64), Ak.indices.astype(np.int32),
             Ak.data.astype(np.float64), lo[keep_r], hi[keep_r], lp.col_lo[keep_c], lp.col_hi[keep_c],
             lp.c[keep_c], float(lp.obj_offset + lp.c @ xf), dict(lp.meta))
    x_fixed = np.where(fixed, lp.col_lo, np.nan)
    return Presolved(red, keep_c, keep_r, x_fixed, ok)


def lift(pre: Presolved, x_red):
    """Original-space point from a reduced solution."""
    x = pre.x_fixed.copy()
    x[pre.cols] = x_red
    return x


# ----------------------------------------------------------------------------- the reduced batch

# Parent instances of the batch cycle through five sizes (buses, lines, units, hours,
# monitored lines, outages per line).
BATCH_PARENTS = [
    scuc.SCUCConfig(30, 41, 10, 24, None, 0, 0.0, "batch-30bus"),
    scuc.SCUCConfig(100, 150, 25, 24, 40, 3, 1e-3, "batch-100bus"),
    scuc.SCUCConfig(300, 450, 75, 36, 60, 4, 1e-3, "batch-300bus"),
    scuc.SCUCConfig(600, 900, 150, 48, 100, 5, 1e-3, "batch-600bus"),
    scuc.SCUCConfig(1000, 1500, 250, 48, 150, 6, 1e-3, "batch-1000bus"),
]


def synthetic_relaxation(G: int, T: int, target: float, rng: np.random.Generator):
    """Relaxed (u, v, w) standing in for a round's LP solution: every unit is confidently on
    (u = 1, v = w = 0) up to a seeded hour s_g and fractional from there on, with s_g drawn
    around 1 + target * T. Algorithm 1 then fixes hours 2..s_g of each unit on, so about
    `target` of the u variables end up fixed; fixing units on keeps the reduced LP feasible
    (the all-on dispatch the line limits are built from stays available)."""
    s = np.clip(np.round(1 + target * T + rng.normal(0.0, 0.15 * T, G)), 1, T).astype(int)
    t = np.arange(T)[None, :]
    frac = t >= s[:, None]
    u = np.where(frac, rng.uniform(0.2, 0.8, (G, T)), 1.0)
    v = np.where(frac, rng.uniform(0.15, 0.45, (G, T)), 0.0)
    w = np.where(frac, rng.uniform(0.15, 0.45, (G, T)), 0.0)
    return u, v, w


def reduced_lp(parent: scuc.SCUCConfig, seed: int, target: float, tau: float = 0.1):
    """One reduced LP of a successive-fixing round: Algorithm 1 (tau = 0.1) applied to the
    parent's relaxed binaries, the fixings written as equal column bounds, then presolved."""
    data, lp = scuc.make_instance(parent, seed)
    G, T = parent.n_gen, parent.T
    rng = np.random.default_rng(seed + 7919)
    u, v, w = synthetic_relaxation(G, T, target, rng)
    fixed, ur, vr, wr = fixing_strategy(u, v, w, tau)
    lo, hi = fix_bounds(lp, G, T, fixed, ur, vr, wr)
    pre = presolve_fixed(lp.replace(col_lo=lo, col_hi=hi))
    pre.lp.meta.update(parent=parent.name, seed=seed, fixed_u=float(fixed.sum()) / (G * T), target=target,
                       data=data, fixed=fixed, u_fixed=np.where(fixed, ur, 0).astype(np.int8),
                       cols=pre.cols, rows=pre.rows)
    return pre


def _batch_member(args):
    parent, seed, target = args
    return reduced_lp(parent, seed, target)


def make_reduced_batch(count: int = 64, seed0: int = 100, classes: int | None = None,
                       parent: scuc.SCUCConfig | None = None, workers: int = 1, log=None):
    """`count` reduced LPs: LP i has parent seed seed0 + i and about 0.2 + 0.7 i / (count - 1)
    of its u variables fixed. Its parent is `parent` when given (e.g. the 2,000-bus preset),
    else size class i mod (number of classes) of the mixed parent list."""
    k = classes or len(BATCH_PARENTS)
    jobs = [(parent if parent is not None else BATCH_PARENTS[i % k], seed0 + i,
             0.2 + 0.7 * i / max(count - 1, 1)) for i in range(count)]
    if workers <= 1:
        out = []
        for j in jobs:
            out.append(_batch_member(j))
            if log is not None:
                log(f"reduced LP {len(out)}/{count}: parent {j[0].name} seed {j[1]} nnz {out[-1].lp.nnz}")
        return out
    import multiprocessing as mp
    # fresh interpreters: the caller may already hold a GPU context, which a forked child
    # would inherit
    with mp.get_context("spawn").Pool(workers) as pool:
        out = []
        for r in pool.imap(_batch_member, jobs):
            out.append(r)
            if log is not None:
                log(f"reduced LP {len(out)}/{count}: parent {r.lp.meta['parent']} seed {r.lp.meta['seed']} "
                    f"nnz {r.lp.nnz}")
        return out
