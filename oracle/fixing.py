"""CPU reference of the successive-fixing loop around the LP solver (Section IV).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): the GPU fixing kernel and the product's
successive-fixing driver are checked against these functions; the product never imports them.

* round_value: the Round operator of Section IV-A.
* algorithm1: the Fixing-Strategy of Algorithm 1, unit by unit and hour by hour, with plain
  Python loops (hours are 0-based here: the paper's hour t is index t - 1, so its loop over
  t = 2..T is the index range 1..T-1 and hour 1 is never fixed).
* presolve_fixed: the LP-Presolve step this build takes for Algorithm 2 (columns with equal
  bounds substituted out, rows left empty dropped after checking that 0 fits their bounds).
* successive: Algorithm 2 without its MILP steps, driven by the oracle's solver.

Inputs name the binaries through `cols` [G][T][3], the LP column of (u, v, w) of unit g at
hour t.
"""
from __future__ import annotations

import numpy as np


def round_value(s: float, tau: float) -> int:
    """Round(s, tau): 1 if s >= 1 - tau, 0 if 0 <= s <= tau, -1 otherwise."""
    if s >= 1.0 - tau:
        return 1
    if 0.0 <= s <= tau:
        return 0
    return -1


def algorithm1(x, cols, tau: float):
    """Fixing-Strategy for the relaxed point x (original space).

    Returns (fixed [G][T] of 0/1, rounded [G][T][3] of -1/0/1)."""
    G, T = len(cols), len(cols[0])
    rounded = np.zeros((G, T, 3), np.int8)
    fixed = np.zeros((G, T), np.int8)
    for g in range(G):
        for t in range(T):
            for k in range(3):
                rounded[g, t, k] = round_value(float(x[cols[g][t][k]]), tau)
        for t in range(1, T):
            u, u_prev = int(rounded[g, t, 0]), int(rounded[g, t - 1, 0])
            v, w = int(rounded[g, t, 1]), int(rounded[g, t, 2])
            if u == -1 or u_prev == -1 or v == -1 or w == -1:
                break
            if u - u_prev == v - w and v + w <= 1:
                fixed[g, t] = 1
            else:
                break
    return fixed, rounded


def presolve_fixed(lp, tol: float = 1e-9):
    """Substitute every column with col_lo == col_hi into the rows and the objective.

    Returns (reduced LP, kept columns, kept rows, feasible): a row whose entries were all in
    fixed columns is dropped when 0 lies within its shifted bounds (up to tol), else the
    reduced problem is reported infeasible."""
    from paper_2510_10891_amd.scuc import LP   # the LP container of the input generator

    m, n = lp.m, lp.n
    fixed = np.asarray(lp.col_lo) == np.asarray(lp.col_hi)
    keep_c = [j for j in range(n) if not fixed[j]]
    new_index = {j: q for q, j in enumerate(keep_c)}
    lo = np.array(lp.row_lo, float)
    hi = np.array(lp.row_hi, float)
    offset = float(lp.obj_offset) + float(sum(lp.c[j] * lp.col_lo[j] for j in range(n) if fixed[j]))
    rows_idx, rows_val = [], []
    feasible = True
    keep_r = []
    for i in range(m):
        shift = 0.0
        idx, val = [], []
        for k in range(lp.row_ptr[i], lp.row_ptr[i + 1]):
            j = int(lp.col_idx[k])
            if fixed[j]:
                shift += lp.val[k] * lp.col_lo[j]
            else:
                idx.append(new_index[j])
                val.append(float(lp.val[k]))
        lo[i] -= shift
        hi[i] -= shift
        if idx:
            order = np.argsort(idx)
            rows_idx.append(np.asarray(idx, np.int32)[order])
            rows_val.append(np.asarray(val, float)[order])
            keep_r.append(i)
        elif lo[i] > tol * (1 + abs(lo[i])) or hi[i] < -tol * (1 + abs(hi[i])):
            feasible = False
    ptr = np.zeros(len(keep_r) + 1, np.int64)
    for q, r in enumerate(rows_idx):
        ptr[q + 1] = ptr[q] + len(r)
    keep_c = np.asarray(keep_c, np.int64)
    keep_r = np.asarray(keep_r, np.int64)
    red = LP(len(keep_r), len(keep_c), ptr,
             np.concatenate(rows_idx).astype(np.int32) if rows_idx else np.zeros(0, np.int32),
             np.concatenate(rows_val) if rows_val else np.zeros(0),
             lo[keep_r], hi[keep_r], np.asarray(lp.col_lo, float)[keep_c], np.asarray(lp.col_hi, float)[keep_c],
             np.asarray(lp.c, float)[keep_c], offset)
    return red, keep_c, keep_r, feasible


def successive(lp, cols, rounds: int, tau: float, opts, presolve: bool = True, warm: bool = True):
    """Algorithm 2 without the MILP steps on the oracle's solver: each round solves the
    current LP (the original LP with the fixings so far written as equal bounds, presolved
    when `presolve`), runs Algorithm 1 on the relaxed binaries of the original problem and
    fixes them. A round starts from the previous round's solution when `warm`. Stops after a
    round whose LP is not solved.

    Returns a list of per-round dicts (term, iters, objective, fixed [G][T], rounded)."""
    import oracle

    lo, hi = np.array(lp.col_lo, float), np.array(lp.col_hi, float)
    G, T = len(cols), len(cols[0])
    fixed_all = np.zeros((G, T), np.int8)
    out = []
    x_full = y_full = None
    for _ in range(rounds):
        cur = lp.replace(col_lo=lo.copy(), col_hi=hi.copy())
        if presolve:
            red, kc, kr, feasible = presolve_fixed(cur)
            if not feasible:
                out.append(dict(term="primal_infeasible", iters=0, objective=np.nan, fixed=fixed_all.copy()))
                break
        else:
            red, kc, kr = cur, np.arange(lp.n), np.arange(lp.m)
        x0 = y0 = None
        if warm and x_full is not None:
            x0, y0 = x_full[kc], y_full[kr]
        r = oracle.solve(red, opts, x0=x0, y0=y0)
        x_full = np.where(lo == hi, lo, 0.0)
        x_full[kc] = r.x
        y_full = np.zeros(lp.m)
        y_full[kr] = r.y
        if r.term != "solved":
            out.append(dict(term=r.term, iters=r.iters, objective=r.pobj, fixed=fixed_all.copy()))
            break
        fixed, rounded = algorithm1(x_full, cols, tau)
        new = (fixed == 1) & (fixed_all == 0)
        for g, t in zip(*np.nonzero(new)):
            for k in range(3):
                j = cols[g][t][k]
                lo[j] = hi[j] = float(rounded[g, t, k])
        fixed_all |= fixed
        out.append(dict(term=r.term, iters=r.iters, objective=r.pobj, fixed=fixed_all.copy(), rounded=rounded))
    return out
