"""Pins of the oracle's dual infeasibility test (CPU): LPs with no finite optimum.

An LP whose cost keeps falling along a direction its rows and bounds admit must end as
"dual_infeasible", with an independent LP solver (HiGHS) agreeing that it is unbounded; LPs
with unbounded columns but a finite optimum must still be solved to HiGHS's optimum and never
end that way.
"""
import numpy as np
import pytest
from scipy.optimize import linprog

import oracle
from tests.helpers import dense_lp, highs, rel

INF = np.inf


def highs_status(lp):
    """scipy's HiGHS status on the row-bounded LP: 0 optimal, 2 infeasible, 3 unbounded."""
    A = lp.to_scipy().toarray()
    eq = lp.row_lo == lp.row_hi
    ub = np.isfinite(lp.row_hi) & ~eq
    lb = np.isfinite(lp.row_lo) & ~eq
    A_ub = np.vstack([A[ub], -A[lb]]) if (ub.any() or lb.any()) else None
    b_ub = np.r_[lp.row_hi[ub], -lp.row_lo[lb]] if A_ub is not None else None
    res = linprog(lp.c, A_ub=A_ub, b_ub=b_ub, A_eq=A[eq] if eq.any() else None,
                  b_eq=lp.row_lo[eq] if eq.any() else None,
                  bounds=[(None if not np.isfinite(a) else a, None if not np.isfinite(b) else b)
                          for a, b in zip(lp.col_lo, lp.col_hi)], method="highs")
    return res.status


def nonneg_rays(seed, m=6, n=7):
    """min c^T x, A x >= b with A >= 0, x >= 0: columns in S unbounded above, the others boxed;
    some column of S costs < 0, so x_j -> inf lowers the cost while every row stays satisfied."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(0.1, 2.0, (m, n)) * (rng.random((m, n)) < 0.7)
    A[np.arange(m), rng.integers(0, n, m)] += 0.5
    b = A @ rng.uniform(0.2, 1.0, n)
    unb = rng.random(n) < 0.5
    unb[rng.integers(n)] = True
    c = rng.uniform(0.5, 3.0, n)
    j = rng.choice(np.nonzero(unb)[0])
    c[j] = -rng.uniform(0.5, 2.0)
    u = np.where(unb, INF, rng.uniform(1.0, 3.0, n))
    return dense_lp(A, b, np.full(m, INF), np.zeros(n), u, c)


UNBOUNDED = {
    "chain of equalities": dense_lp([[1, -1, 0], [0, 1, -1]], [0, 0], [0, 0], [0, 0, 0], [INF] * 3,
                                    [-1.0, 0.0, 0.0]),
    "free column": dense_lp([[1, 1]], [1], [INF], [-INF, 0], [INF, INF], [1.0, -1.0]),
    "ranged row, ray in its null space": dense_lp([[1, -1]], [-1], [1], [0, 0], [INF, INF], [-1.0, -1.0]),
    "ray below an upper bound": dense_lp([[1, 2], [1, 0]], [-INF, -INF], [4, 1], [-INF, -INF], [5, 2],
                                         [0.5, 1.0]),
}
for _s in range(6):
    UNBOUNDED[f"nonnegative rays seed {_s}"] = nonneg_rays(_s)

BOUNDED = {
    "covering with free growth": dense_lp([[1, 1]], [1], [INF], [0, 0], [INF, INF], [1.0, 1.0]),
    "growth capped by a row": dense_lp([[-1, 1], [1, 0]], [-INF, 0], [5, 3], [0, 0], [INF, INF], [1.0, -1.0]),
    "free column priced both ways": dense_lp([[1, -1], [1, 1]], [-1, 0], [1, INF], [-INF, 0], [INF, INF],
                                             [0.5, 1.0]),
}
for _s in range(4):
    _lp = nonneg_rays(100 + _s)
    BOUNDED[f"nonnegative rays, positive costs seed {_s}"] = _lp.replace(c=np.abs(_lp.c) + 0.1)


@pytest.mark.parametrize("name", sorted(UNBOUNDED))
def test_unbounded_lps_end_dual_infeasible(name):
    lp = UNBOUNDED[name]
    assert highs_status(lp) == 3, "HiGHS must call the LP unbounded"
    r = oracle.solve(lp, oracle.Options(tol=1e-8, max_iter=200000))
    assert r.term == "dual_infeasible", (r.term, r.iters)


@pytest.mark.parametrize("name", sorted(BOUNDED))
def test_bounded_lps_with_unbounded_columns_are_solved(name):
    lp = BOUNDED[name]
    assert highs_status(lp) == 0
    ref, _, _ = highs(lp)
    r = oracle.solve(lp, oracle.Options(tol=1e-9, max_iter=400000))
    assert r.term == "solved", (r.term, r.iters)
    assert rel(r.pobj, ref) < 1e-6


def test_boxed_lps_never_end_dual_infeasible(small_instances):
    # every SCUC column is boxed: no ray exists, whatever the iterates do
    _, lp = small_instances[0]
    r = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=2000))
    assert r.term == "iter_limit"
