"""Shared test helpers: an independent LP solve by HiGHS (scipy) and tiny-LP builders."""
import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog

from paper_2510_10891_amd.scuc import LP


def highs(lp: LP):
    """Solve the row-bounded LP with scipy's HiGHS; returns (objective, x, y) in our sign convention.

    y follows the convention c = A^T y + z: y_i > 0 on an active lower side, < 0 on an
    active upper side.
    """
    A = lp.to_scipy()
    eq = lp.row_lo == lp.row_hi
    ub = np.isfinite(lp.row_hi) & ~eq
    lb = np.isfinite(lp.row_lo) & ~eq
    A_ub = sp.vstack([A[ub], -A[lb]]).tocsr() if (ub.any() or lb.any()) else None
    b_ub = np.r_[lp.row_hi[ub], -lp.row_lo[lb]] if A_ub is not None else None
    A_eq = A[eq] if eq.any() else None
    b_eq = lp.row_lo[eq] if eq.any() else None
    res = linprog(lp.c, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=b_eq,
                  bounds=np.c_[lp.col_lo, lp.col_hi], method="highs")
    assert res.status == 0, res.message
    y = np.zeros(lp.m)
    if eq.any():
        y[eq] = res.eqlin.marginals
    if A_ub is not None:
        mu = res.ineqlin.marginals
        y[ub] += mu[: ub.sum()]
        y[lb] -= mu[ub.sum():]
    return res.fun + lp.obj_offset, res.x, y


def dense_lp(A, lo, hi, l, u, c, off=0.0) -> LP:
    A = sp.csr_matrix(np.asarray(A, float))
    A.sort_indices()
    m, n = A.shape
    return LP(m, n, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(float),
              np.asarray(lo, float), np.asarray(hi, float), np.asarray(l, float),
              np.asarray(u, float), np.asarray(c, float), off)


def rel(a, b):
    return abs(a - b) / max(1.0, abs(b))
