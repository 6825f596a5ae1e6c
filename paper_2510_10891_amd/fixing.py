"""Successive fixing around the LP solver (Section IV): Round, the logic-driven
Fixing-Strategy of Algorithm 1, a minimal LP presolve (fixed columns, implied-free column
singletons), and the batch of reduced LPs that successive-fixing rounds hand to the solver
(built from stored fixings of solved relaxations, or from synthetic relaxations).

Host-side support code: it decides which binaries are fixed and rewrites the LP; it holds
none of the LP iteration's arithmetic.
"""
from __future__ import annotations

import base64
import json
import zlib
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


@dataclass
class Substituted:
    lp: LP                 # the reduced LP
    cols: np.ndarray       # kept original columns
    rows: np.ndarray       # kept original rows
    sub_c: np.ndarray      # substituted columns j ...
    sub_r: np.ndarray      # ... each defined by its equality row i
    orig: LP               # the LP before the substitution


def presolve_free_singletons(lp: LP, tol: float = 1e-9) -> Substituted:
    """LP presolve of implied-free column singletons: a column j whose only entry a_ij lies in
    an equality row i (sum_k a_ik x_k = b_i), and whose bounds are implied by that row and the
    bounds of the row's other columns, is substituted out, x_j = (b_i - sum_{k != j} a_ik x_k) / a_ij:
    its cost moves onto the row's other columns (c_k -= c_j a_ik / a_ij, offset += c_j b_i / a_ij)
    and row i and column j are dropped. At most one column per row. On SCUC models this removes
    cost variables defined by an equality (c_gt = sum_h C_gh p_gth), through which alone the
    objective would otherwise reach the segment outputs."""
    A = lp.to_scipy()
    cols = A.indices
    eq = (lp.row_lo == lp.row_hi) & np.isfinite(lp.row_lo)
    # singleton columns (one stored entry) in equality rows, the first one per row
    cnt = np.bincount(cols, minlength=lp.n)
    pos = np.nonzero(cnt[cols] == 1)[0]
    i_s = np.searchsorted(A.indptr, pos, side="right") - 1
    single, a_s = cols[pos], A.data[pos]
    ok = eq[i_s] & (a_s != 0.0)
    pos, i_s, single, a_s = pos[ok], i_s[ok], single[ok], a_s[ok]
    _, first = np.unique(i_s, return_index=True)
    pos, i_s, single, a_s = pos[first], i_s[first], single[first], a_s[first]
    # range of sum_{k != j} a_ik x_k over the column bounds (infinite where a term is unbounded)
    rest_lo, rest_hi = np.empty(len(i_s)), np.empty(len(i_s))
    for q, i in enumerate(i_s):
        seg = slice(A.indptr[i], A.indptr[i + 1])
        v, cc = A.data[seg], cols[seg]
        own = np.arange(seg.start, seg.stop) == pos[q]
        v, cc = v[~own], cc[~own]
        with np.errstate(invalid="ignore"):
            lo_t = np.where(v > 0, v * lp.col_lo[cc], v * lp.col_hi[cc])
            hi_t = np.where(v > 0, v * lp.col_hi[cc], v * lp.col_lo[cc])
        rest_lo[q] = -np.inf if np.any(~np.isfinite(lo_t)) else lo_t.sum()
        rest_hi[q] = np.inf if np.any(~np.isfinite(hi_t)) else hi_t.sum()
    b = lp.row_lo[i_s]
    with np.errstate(invalid="ignore", divide="ignore"):
        lo_j = np.where(a_s > 0, (b - rest_hi) / a_s, (b - rest_lo) / a_s)
        hi_j = np.where(a_s > 0, (b - rest_lo) / a_s, (b - rest_hi) / a_s)
    l, u = lp.col_lo[single], lp.col_hi[single]
    ok_lo = ~np.isfinite(l) | (lo_j >= l - tol * (1 + np.abs(l)))
    ok_hi = ~np.isfinite(u) | (hi_j <= u + tol * (1 + np.abs(u)))
    take = ok_lo & ok_hi
    sub_c, sub_r, a_sub = single[take].astype(np.int64), i_s[take].astype(np.int64), a_s[take]
    order = np.argsort(sub_c)
    sub_c, sub_r, a_sub = sub_c[order], sub_r[order], a_sub[order]
    if len(sub_c):
        f = lp.c[sub_c] / a_sub              # y_i of each dropped row
        c = lp.c - A[sub_r].T @ f
        offset = float(lp.obj_offset + f @ lp.row_lo[sub_r])
    else:
        c, offset = lp.c.copy(), float(lp.obj_offset)
    keep_c = np.setdiff1d(np.arange(lp.n), sub_c)
    keep_r = np.setdiff1d(np.arange(lp.m), sub_r)
    Ak = A[keep_r][:, keep_c].tocsr()
    Ak.sort_indices()
    red = LP(len(keep_r), len(keep_c), Ak.indptr.astype(np.int64), Ak.indices.astype(np.int32),
             Ak.data.astype(np.float64), lp.row_lo[keep_r], lp.row_hi[keep_r], lp.col_lo[keep_c],
             lp.col_hi[keep_c], c[keep_c], offset, dict(lp.meta))
    return Substituted(red, keep_c, keep_r, sub_c, sub_r, lp)


def postsolve_free_singletons(s: Substituted, x_red, y_red, z_red):
    """(x, y, z) of the original LP from a reduced solution: x_j from its defining row,
    y_i = c_j / a_ij for the dropped row (column j's reduced cost is 0, it is free), the
    other multipliers and reduced costs as computed on the reduced LP."""
    lp = s.orig
    A = lp.to_scipy()
    x = np.zeros(lp.n)
    x[s.cols] = x_red
    y = np.zeros(lp.m)
    y[s.rows] = y_red
    z = np.zeros(lp.n)
    z[s.cols] = z_red
    if len(s.sub_c) == 0:
        return x, y, z
    a = np.asarray(A[s.sub_r, s.sub_c]).ravel()
    rest = A[s.sub_r] @ x            # x_j is still 0 and appears in no other dropped row
    x[s.sub_c] = (lp.row_lo[s.sub_r] - rest) / a
    y[s.sub_r] = lp.c[s.sub_c] / a
    return x, y, z


# ----------------------------------------------------------------------------- the reduced batch

# Parent instances of the mixed batch (defined with the generator).
BATCH_PARENTS = scuc.BATCH_PARENTS


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


def _plane(text: str, G: int, T: int) -> np.ndarray:
    bits = np.unpackbits(np.frombuffer(zlib.decompress(base64.b64decode(text)), np.uint8))
    return bits[:G * T].reshape(G, T).astype(bool)


def decode_fixing(rec: dict):
    """(fixed, ur, vr, wr) over [G][T] of a stored fixing: a record with G, T and four bit
    planes (zlib-compressed, base64-encoded, row-major [G][T]): the fixed unit-hours and the
    rounded u, v, w of the fixed ones."""
    G, T = int(rec["G"]), int(rec["T"])
    fixed = _plane(rec["fixed"], G, T)
    ur, vr, wr = (_plane(rec[k], G, T).astype(np.int8) for k in ("u", "v", "w"))
    return fixed, ur, vr, wr


def load_fixings(path: str) -> list:
    """The member records of a stored batch of fixings (a JSON file with a "members" list)."""
    with open(path) as f:
        return json.load(f)["members"]


def reduced_lp(parent: scuc.SCUCConfig, seed: int, target: float, tau: float = 0.1, fixing: dict | None = None):
    """One reduced LP of a successive-fixing round: the parent's binaries fixed by Algorithm 1,
    the fixings written as equal column bounds, then presolved. With `fixing` (a stored record
    for this parent and seed: Algorithm 1 on the solved relaxation, see decode_fixing) that
    fixing is applied; otherwise Algorithm 1 (tau) runs on a synthetic relaxation aimed at
    `target`."""
    data, lp = scuc.make_instance(parent, seed)
    G, T = parent.n_gen, parent.T
    if fixing is not None:
        if fixing["parent"] != parent.name or int(fixing["seed"]) != seed:
            raise ValueError(f"stored fixing is for {fixing['parent']} seed {fixing['seed']}, "
                             f"not {parent.name} seed {seed}")
        fixed, ur, vr, wr = decode_fixing(fixing)
        source = f"solved relaxation, tau {fixing['tau']}"
    else:
        rng = np.random.default_rng(seed + 7919)
        u, v, w = synthetic_relaxation(G, T, target, rng)
        fixed, ur, vr, wr = fixing_strategy(u, v, w, tau)
        source = "synthetic relaxation"
    return apply_fixing(parent, seed, target, data, lp, fixed, ur, vr, wr, source)


def apply_fixing(parent: scuc.SCUCConfig, seed: int, target: float, data, lp: LP, fixed, ur, vr, wr,
                 source: str):
    """Fix(M, S, s) for the given fixing of the parent LP, then presolve; the result's LP
    carries the parent, seed, fixing and the kept columns and rows in its meta."""
    G, T = parent.n_gen, parent.T
    lo, hi = fix_bounds(lp, G, T, fixed, ur, vr, wr)
    pre = presolve_fixed(lp.replace(col_lo=lo, col_hi=hi))
    pre.lp.meta.update(parent=parent.name, seed=seed, fixed_u=float(fixed.sum()) / (G * T), target=target,
                       data=data, fixed=fixed, u_fixed=np.where(fixed, ur, 0).astype(np.int8),
                       cols=pre.cols, rows=pre.rows, fixing_source=source)
    return pre


def _batch_member(args):
    parent, seed, target, fixing = args
    return reduced_lp(parent, seed, target, fixing=fixing)


def make_reduced_batch(count: int = 64, seed0: int = 100, classes: int | None = None,
                       parent: scuc.SCUCConfig | None = None, workers: int = 1, log=None,
                       fixings: list | None = None):
    """`count` reduced LPs: LP i has parent seed seed0 + i and about 0.2 + 0.7 i / (count - 1)
    of its u variables fixed. Its parent is `parent` when given (e.g. the 2,000-bus preset),
    else size class i mod (number of classes) of the mixed parent list. `fixings` (optional):
    stored fixings, record i for LP i (see reduced_lp)."""
    k = classes or len(BATCH_PARENTS)
    jobs = [(parent if parent is not None else BATCH_PARENTS[i % k], seed0 + i,
             0.2 + 0.7 * i / max(count - 1, 1), fixings[i] if fixings is not None else None)
            for i in range(count)]
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
