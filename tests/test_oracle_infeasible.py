"""Pins of the oracle's primal infeasibility certificate (CPU).

Infeasible LPs must end as "primal_infeasible", with an independent LP solver (HiGHS)
agreeing that they are infeasible and the returned bar point y passing a Farkas check done
here with numpy on the original data: y sign-feasible, and
    h(y) = sum lo_i y_i+ - hi_i y_i- + sum l_j dz_j+ - u_j dz_j-  > 0,  dz = -A^T y,
which no feasible LP allows (h(y) <= y'Ax - y'Ax = 0 for every feasible x). Feasible LPs must
never end that way.
"""
import numpy as np
import pytest
from scipy.optimize import linprog

import oracle
from paper_2510_10891_amd import fixing, scuc
from tests.helpers import dense_lp, highs


def farkas(lp, y):
    """(h, magnitude, violation) of the certificate built from y on the original LP. y must
    be sign-feasible for the rows (None otherwise); dz = -A^T y should be for the column
    bounds, and `violation` = sum of |dz_j| on the wrong side of an infinite bound, relative
    to sum |y_i| (0 for an exact certificate; those terms are left out of h)."""
    A = lp.to_scipy()
    if np.any((y > 0) & ~np.isfinite(lp.row_lo)) or np.any((y < 0) & ~np.isfinite(lp.row_hi)):
        return None
    dz = -(A.T @ y)
    bad = ((dz > 0) & ~np.isfinite(lp.col_lo)) | ((dz < 0) & ~np.isfinite(lp.col_hi))
    viol = np.abs(dz[bad]).sum() / max(np.abs(y).sum(), 1e-300)
    dz = np.where(bad, 0.0, dz)
    yp, ym = np.maximum(y, 0), np.maximum(-y, 0)
    zp, zm = np.maximum(dz, 0), np.maximum(-dz, 0)
    lo, hi = np.where(yp > 0, lp.row_lo, 0.0), np.where(ym > 0, lp.row_hi, 0.0)
    l, u = np.where(zp > 0, lp.col_lo, 0.0), np.where(zm > 0, lp.col_hi, 0.0)
    h = lo @ yp - hi @ ym + l @ zp - u @ zm
    mag = np.abs(lo) @ yp + np.abs(hi) @ ym + np.abs(l) @ zp + np.abs(u) @ zm
    return h, mag, viol


def highs_infeasible(lp):
    with pytest.raises(AssertionError, match="nfeasible"):
        highs(lp)


def test_box_too_small_for_a_row():
    # x1 + x2 >= 3 with 0 <= x <= 1
    lp = dense_lp([[1.0, 1.0]], [3.0], [np.inf], [0, 0], [1, 1], [1.0, 2.0])
    highs_infeasible(lp)
    r = oracle.solve(lp, oracle.Options(tol=1e-6, max_iter=20000))
    assert r.term == "primal_infeasible"
    h, mag, viol = farkas(lp, r.y)
    assert h > 1e-6 * mag > 0 and viol == 0


def test_contradicting_rows_on_a_free_column():
    # x >= 1 and x <= 0 with x free: the certificate combines the two rows, dz = 0
    lp = dense_lp([[1.0], [1.0]], [1.0, -np.inf], [np.inf, 0.0], [-np.inf], [np.inf], [0.5])
    highs_infeasible(lp)
    r = oracle.solve(lp, oracle.Options(tol=1e-6, max_iter=20000))
    assert r.term == "primal_infeasible"
    h, mag, viol = farkas(lp, r.y)
    assert h > 1e-6 * mag > 0 and viol < 1e-5


@pytest.mark.parametrize("seed", range(6))
def test_random_lps_made_infeasible(seed):
    """A feasible random LP plus a row its box cannot satisfy."""
    rng = np.random.default_rng(seed)
    base = scuc.random_lp(rng, 6, 5)
    A = base.to_scipy().toarray()
    a = rng.standard_normal(5)
    reach = np.where(a > 0, a * base.col_hi, a * base.col_lo).sum()   # max of a'x over the box
    lp = dense_lp(np.vstack([A, a]), np.r_[base.row_lo, reach + 1.0], np.r_[base.row_hi, np.inf],
                  base.col_lo, base.col_hi, base.c)
    highs_infeasible(lp)
    r = oracle.solve(lp, oracle.Options(tol=1e-6, max_iter=200000))
    assert r.term == "primal_infeasible"
    h, mag, viol = farkas(lp, r.y)
    assert h > 1e-6 * mag > 0 and viol == 0


@pytest.mark.parametrize("seed", range(8))
def test_feasible_random_lps_are_never_declared_infeasible(seed):
    lp = scuc.random_lp(np.random.default_rng(100 + seed), 7, 5)
    r = oracle.solve(lp, oracle.Options(tol=1e-8, max_iter=200000))
    assert r.term == "solved"


def test_scuc_fixing_round_that_leaves_no_capacity():
    """The 30-bus seed-3 case: the first round of Algorithm 1 switches off units whose relaxed
    commitment is below tau for the whole horizon; the next LP is infeasible."""
    data, lp = scuc.make_instance("small", 3)
    G, T = data.cfg.n_gen, data.cfg.T
    r1 = oracle.solve(lp, oracle.Options(tol=1e-6, max_iter=200000))
    assert r1.term == "solved"
    u, v, w = fixing.gather_binaries(r1.x, G, T)
    fixed, ur, vr, wr = fixing.fixing_strategy(u, v, w, 0.1)
    lo, hi = fixing.fix_bounds(lp, G, T, fixed, ur, vr, wr)
    lp2 = lp.replace(col_lo=lo, col_hi=hi)
    highs_infeasible(lp2)
    r2 = oracle.solve(lp2, oracle.Options(tol=1e-6, max_iter=200000))
    assert r2.term == "primal_infeasible" and r2.iters < 200000
    h, mag, viol = farkas(lp2, r2.y)
    assert h > 1e-6 * mag > 0 and viol == 0
