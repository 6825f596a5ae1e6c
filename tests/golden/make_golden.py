"""Writes the stored expected values under tests/golden/ without the GPU path.

Usage: python tests/golden/make_golden.py [medium]
For the 2,000-bus instance (generator preset "medium", seed 0) the optimal objective is
computed by scipy's HiGHS interior-point solver (with crossover), an LP solver independent
of both the oracle and the GPU library; the record names the instance and the solver.
"""
import json
import os
import sys
import time

import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2510_10891_amd import scuc  # noqa: E402


def highs_objective(lp):
    A = lp.to_scipy()
    eq = lp.row_lo == lp.row_hi
    ub = np.isfinite(lp.row_hi) & ~eq
    lb = np.isfinite(lp.row_lo) & ~eq
    res = linprog(lp.c, A_ub=sp.vstack([A[ub], -A[lb]]).tocsr(), b_ub=np.r_[lp.row_hi[ub], -lp.row_lo[lb]],
                  A_eq=A[eq], b_eq=lp.row_lo[eq], bounds=np.c_[lp.col_lo, lp.col_hi], method="highs-ipm")
    return res


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "medium"
    _, lp = scuc.make_instance(which, 0)
    t = time.time()
    res = highs_objective(lp)
    rec = dict(preset=which, seed=0, m=lp.m, n=lp.n, nnz=lp.nnz, status=int(res.status), message=res.message,
               objective=float(res.fun + lp.obj_offset), seconds=round(time.time() - t, 1),
               source="scipy.optimize.linprog(method='highs-ipm') on the generated LP")
    with open(os.path.join(HERE, f"highs_{which}_seed0.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))
