"""Successive fixing (Algorithm 2) around the GPU LP solver, without the MILP presolve and
the final MILP solve (both need a MILP solver).

Each round solves the current LP relaxation, runs Round and the Fixing-Strategy (Algorithm 1)
on the device over the relaxed binaries of the bar point the solve left in HBM
(hpr_fix_binaries), and applies Fix(M, S, s) by setting equal column bounds. With `presolve`
(Algorithm 2's LP-Presolve step, the default) the next round's LP is the fixed LP with its
fixed columns substituted out and emptied rows dropped, on a handle of its own; without it one
handle serves every round and only the bounds change. A round starts from the previous round's
solution (restricted to the columns and rows it keeps) when `warm`. A round whose FP32 solve
stalls above the tolerance is finished with FP64 storage from that point (mixed.py). A round
whose LP cannot be solved (or that presolve finds infeasible) stops the loop.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import fixing, hprlp, mixed, scuc


@dataclass
class Round:
    index: int
    term: str
    iters: int
    solve_s: float
    objective: float
    rel_kkt: float
    fixed_u: float          # fraction of all u fixed after this round
    newly_fixed: int
    setup_s: float = 0.0    # creation of the round's handle (presolved LP), 0 when it was reused
    n: int = 0              # columns, rows and stored entries of the LP the round solved
    m: int = 0
    nnz: int = 0
    fixed: np.ndarray | None = None   # [G][T] units-hours fixed after this round
    continued: bool = False # the FP32 solve stalled and the round's LP was finished in FP64


@dataclass
class Result:
    rounds: list = field(default_factory=list)
    col_lo: np.ndarray | None = None
    col_hi: np.ndarray | None = None
    x: np.ndarray | None = None


def binary_columns(G: int, T: int) -> np.ndarray:
    """[G][T][3] columns of (u, v, w) of the compact SCUC model."""
    t = np.arange(T)[None, :]
    g = np.arange(G)[:, None]
    return np.stack([scuc.col_index(G, t, var, g) for var in (scuc.U, scuc.V, scuc.W)], -1).astype(np.int32)


def run(data: scuc.SCUCData, lp: scuc.LP, rounds: int = 4, tau: float = 0.1,
        opts: hprlp.Options | None = None, warm: bool = True, presolve: bool = True, log=None) -> Result:
    """Up to `rounds` rounds of solve, Algorithm 1 (device) and Fix; `log` (optional)
    receives one line per round."""
    G, T = data.cfg.n_gen, data.cfg.T
    opts = opts or hprlp.Options(tol=1e-4, precision=hprlp.HPR_FP32)
    cols = binary_columns(G, T)
    res = Result()
    lo, hi = lp.col_lo.copy(), lp.col_hi.copy()
    fixed = np.zeros((G, T), bool)
    x_full = y_full = None
    h = hs = None   # the round's handle, and the FP64 continuation's when its FP32 solve stalled
    try:
        for i in range(1, rounds + 1):
            setup = 0.0
            if presolve:
                pre = fixing.presolve_fixed(lp.replace(col_lo=lo, col_hi=hi))
                if not pre.feasible:
                    res.rounds.append(Round(i, "primal_infeasible", 0, 0.0, np.nan, np.nan, float(fixed.mean()), 0,
                                            fixed=fixed.copy()))
                    break
                cur, kc, kr = pre.lp, pre.cols, pre.rows
                if h is not None:
                    hprlp.hpr_destroy(h)
                    h = hs = None
                t0 = time.perf_counter()
                h = hprlp.hpr_create(cur, opts)
                setup = time.perf_counter() - t0
            else:
                cur, kc, kr = lp.replace(col_lo=lo, col_hi=hi), np.arange(lp.n), np.arange(lp.m)
                if h is None:
                    t0 = time.perf_counter()
                    h = hprlp.hpr_create(cur, opts)
                    setup = time.perf_counter() - t0
                else:
                    hprlp.hpr_set_bounds(h, lo, hi)
            if warm and x_full is not None:
                hprlp.hpr_set_start(h, x_full[kc], y_full[kr])
            hs = h
            t0 = time.perf_counter()
            info = hprlp.hpr_solve(h)
            if info.term == "stalled":  # FP32 plateau above tol: go on in FP64 from this point
                x, y, _ = hprlp.hpr_get_solution(h)
                hs = hprlp.hpr_create(cur, mixed.fp64_options(opts, info.iters))
                hprlp.hpr_set_start(hs, x, y)
                offset = time.perf_counter() - t0
                info = mixed.merge(info, hprlp.hpr_solve(hs), offset)
            dt = time.perf_counter() - t0
            x, y, _ = hprlp.hpr_get_solution(hs)
            x_full = np.where(lo == hi, lo, 0.0)
            x_full[kc] = x
            y_full = np.zeros(lp.m)
            y_full[kr] = y
            shape = dict(setup_s=setup, n=cur.n, m=cur.m, nnz=cur.nnz)
            continued = hs is not h
            if info.term != "solved":
                res.rounds.append(Round(i, info.term, info.iters, dt, info.pobj, info.rel_kkt,
                                        float(fixed.mean()), 0, fixed=fixed.copy(), continued=continued,
                                        **shape))
                break
            # Round and Algorithm 1 over the bar point in HBM: columns of the solved LP, and the
            # values of the binaries presolve removed
            pos = np.full(lp.n, -1, np.int64)
            pos[kc] = np.arange(len(kc))
            new, rounded = hprlp.hpr_fix_binaries(hs, pos[cols].astype(np.int32), tau, fixval=lo[cols])
            if continued:
                hprlp.hpr_destroy(hs)
                hs = h
            add = new & ~fixed
            gg, tt = np.nonzero(add)
            for k in range(3):
                c = cols[gg, tt, k]
                lo[c] = rounded[gg, tt, k]
                hi[c] = rounded[gg, tt, k]
            fixed |= new
            res.rounds.append(Round(i, info.term, info.iters, dt, info.pobj, info.rel_kkt,
                                    float(fixed.mean()), int(add.sum()), fixed=fixed.copy(), continued=continued,
                                    **shape))
            if log is not None:
                log(f"round {i}: {info.term}, {info.iters} iterations, {dt:.2f} s solve, {setup:.2f} s setup, "
                    f"n {cur.n}, {fixed.mean():.3f} of u fixed")
    finally:
        if hs is not None and hs is not h:
            hprlp.hpr_destroy(hs)
        if h is not None:
            hprlp.hpr_destroy(h)
    res.col_lo, res.col_hi, res.x = lo, hi, x_full
    return res


def solved_fixing(data: scuc.SCUCData, lp: scuc.LP, target: float, taus, opts: hprlp.Options | None = None):
    """Algorithm 1 on the solved relaxation of `lp`, at the tau of `taus` whose share of fixed
    unit-hours is nearest `target` (the smaller tau on a tie): the first round of the loop,
    with tau picked to reach a given share. Returns (fixed, ur, vr, wr, tau, info) with
    fixed [G][T] bool and the rounded u, v, w as int8, or None when the solve did not succeed."""
    G, T = data.cfg.n_gen, data.cfg.T
    opts = opts or hprlp.Options(tol=1e-4, precision=hprlp.HPR_FP32)
    cols = binary_columns(G, T)
    h = hprlp.hpr_create(lp, opts)
    try:
        info = hprlp.hpr_solve(h)
        if info.term != "solved":
            return None
        best = None
        for tau in taus:
            fixed, rounded = hprlp.hpr_fix_binaries(h, cols, tau)
            share = float(fixed.mean())
            if best is None or abs(share - target) < abs(best[1] - target):
                best = (tau, share, fixed, rounded)
    finally:
        hprlp.hpr_destroy(h)
    tau, _, fixed, rounded = best
    r = rounded.astype(np.int8)
    on = fixed.astype(bool)
    return on, np.where(on, r[:, :, 0], 0), np.where(on, r[:, :, 1], 0), np.where(on, r[:, :, 2], 0), tau, info

