"""Successive fixing (Algorithm 2) around the GPU LP solver, without the MILP presolve and
the final MILP solve (both need a MILP solver).

Each round solves the current LP relaxation, runs the Fixing-Strategy (Algorithm 1) on the
relaxed binaries and applies Fix(M, S, s) by setting equal column bounds. One solver handle
serves every round: the matrix, its scaling and lambda stay on the GPU, only the bounds
change, and each round starts from the previous round's solution (projected onto the new
bounds), so the re-solves are cheap. Rounds whose LP cannot be solved stop the loop.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import fixing, hprlp, scuc


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


@dataclass
class Result:
    rounds: list = field(default_factory=list)
    col_lo: np.ndarray | None = None
    col_hi: np.ndarray | None = None
    x: np.ndarray | None = None


def run(data: scuc.SCUCData, lp: scuc.LP, rounds: int = 4, tau: float = 0.1,
        opts: hprlp.Options | None = None, warm: bool = True, log=None) -> Result:
    """Up to `rounds` rounds of solve, Algorithm 1 and Fix on one handle; `log` (optional)
    receives one line per round."""
    G, T = data.cfg.n_gen, data.cfg.T
    opts = opts or hprlp.Options(tol=1e-4, precision=hprlp.HPR_FP32)
    h = hprlp.hpr_create(lp, opts)
    res = Result()
    lo, hi = lp.col_lo.copy(), lp.col_hi.copy()
    fixed = np.zeros((G, T), bool)
    x = y = None
    try:
        for i in range(1, rounds + 1):
            if warm and x is not None:
                hprlp.hpr_set_start(h, x, y)
            t0 = time.perf_counter()
            info = hprlp.hpr_solve(h)
            dt = time.perf_counter() - t0
            x, y, _ = hprlp.hpr_get_solution(h)
            if info.term != "solved":
                res.rounds.append(Round(i, info.term, info.iters, dt, info.pobj, info.rel_kkt,
                                        float(fixed.mean()), 0))
                break
            u, v, w = fixing.gather_binaries(x, G, T)
            new, ur, vr, wr = fixing.fixing_strategy(u, v, w, tau)
            add = new & ~fixed
            lo, hi = fixing.fix_bounds(lp.replace(col_lo=lo, col_hi=hi), G, T, add, ur, vr, wr)
            fixed |= new
            hprlp.hpr_set_bounds(h, lo, hi)
            res.rounds.append(Round(i, info.term, info.iters, dt, info.pobj, info.rel_kkt,
                                    float(fixed.mean()), int(add.sum())))
            if log is not None:
                log(f"round {i}: {info.term}, {info.iters} iterations, {dt:.2f} s, "
                    f"{fixed.mean():.3f} of u fixed")
    finally:
        hprlp.hpr_destroy(h)
    res.col_lo, res.col_hi, res.x = lo, hi, x
    return res
