"""Pins of the host-side LP presolve steps (CPU): the substituted LP has the optimum of the
original (HiGHS on both), and postsolved oracle solutions satisfy the original's KKT
conditions."""
import numpy as np
import scipy.sparse as sp

import oracle
from paper_2510_10891_amd import fixing, scuc
from tests.helpers import highs


def test_full_scuc_cost_variables_are_substituted():
    data, lp = scuc.make_instance("small", 0, formulation="full")
    s = fixing.presolve_free_singletons(lp)
    G, T, H = data.cfg.n_gen, data.cfg.T, lp.meta["segments"]
    ccols = scuc.full_col_index(G, H, np.arange(T)[:, None], H + 1, np.arange(G)[None, :], T).ravel()
    assert sorted(s.sub_c.tolist()) == sorted(ccols.tolist())
    assert np.all(lp.meta["row_kind"][s.sub_r] == lp.meta["row_kinds"]["cost_def"])
    assert np.array_equal(s.cols[: 4 * G * T], np.arange(4 * G * T))   # compact layout kept
    o1, o2 = highs(lp)[0], highs(s.lp)[0]
    assert abs(o1 - o2) <= 1e-9 * abs(o1)


def test_compact_scuc_has_nothing_to_substitute():
    _, lp = scuc.make_instance("small", 1)
    s = fixing.presolve_free_singletons(lp)
    assert len(s.sub_c) == 0 and s.lp.m == lp.m and s.lp.n == lp.n


def test_postsolved_oracle_solution_is_optimal_for_the_original():
    _, lp = scuc.make_instance("small", 3, formulation="full")
    s = fixing.presolve_free_singletons(lp)
    r = oracle.solve(s.lp, oracle.Options(tol=1e-8, max_iter=400000))
    assert r.term == "solved"
    x, y, z = fixing.postsolve_free_singletons(s, r.x, r.y, r.z)
    ev = oracle.kkt(lp, x, y, z)
    assert ev["rel_kkt"] <= 1e-7, ev
    assert abs(ev["pobj"] - r.pobj) <= 1e-9 * (1 + abs(r.pobj))


def _planted(seed):
    """A random feasible LP plus three singleton columns: j1 in an equality row with bounds
    implied by the row (substitutable), j2 in an equality row with bounds tighter than the
    row implies (kept), j3 in an inequality row (kept)."""
    rng = np.random.default_rng(seed)
    base = scuc.random_lp(rng, 6, 5)
    A = base.to_scipy().toarray()
    m, n = A.shape
    xf = base.meta["x_feasible"]
    lo, hi = base.row_lo.copy(), base.row_hi.copy()
    rows = []
    for kind in ("implied", "tight", "ineq"):
        a = rng.standard_normal(n)
        rows.append((kind, a))
    A2 = np.zeros((m + 3, n + 3))
    A2[:m, :n] = A
    col_lo = np.r_[base.col_lo, np.zeros(3)]
    col_hi = np.r_[base.col_hi, np.zeros(3)]
    row_lo, row_hi = np.r_[lo, np.zeros(3)], np.r_[hi, np.zeros(3)]
    for k, (kind, a) in enumerate(rows):
        r, j = m + k, n + k
        A2[r, :n] = a
        A2[r, j] = -1.0                      # x_j = a'x (row: a'x - x_j = 0)
        reach_lo = np.minimum(a * base.col_lo, a * base.col_hi).sum()
        reach_hi = np.maximum(a * base.col_lo, a * base.col_hi).sum()
        if kind == "tight":
            col_lo[j], col_hi[j] = 0.5 * reach_lo + 0.5 * (a @ xf), 0.5 * reach_hi + 0.5 * (a @ xf)
        else:
            col_lo[j], col_hi[j] = reach_lo - 1.0, reach_hi + 1.0
        if kind == "ineq":
            row_lo[r], row_hi[r] = -np.inf, 0.5
        else:
            row_lo[r] = row_hi[r] = 0.0
    c = np.r_[base.c, rng.standard_normal(3)]
    S = sp.csr_matrix(A2)
    S.sort_indices()
    lp = scuc.LP(m + 3, n + 3, S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data.copy(),
                 row_lo, row_hi, col_lo, col_hi, c, 0.5)
    return lp, n


def test_only_implied_free_equality_singletons_are_substituted():
    for seed in range(5):
        lp, n = _planted(seed)
        s = fixing.presolve_free_singletons(lp)
        assert s.sub_c.tolist() == [n], (seed, s.sub_c)
        o1, o2 = highs(lp)[0], highs(s.lp)[0]
        assert abs(o1 - o2) <= 1e-9 * (1 + abs(o1))
        r = oracle.solve(s.lp, oracle.Options(tol=1e-9, max_iter=400000))
        x, y, z = fixing.postsolve_free_singletons(s, r.x, r.y, r.z)
        assert oracle.kkt(lp, x, y, z)["rel_kkt"] <= 1e-8
