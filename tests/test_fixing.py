"""Algorithm 1 (Fixing-Strategy), the Round operator and the LP presolve of the
successive-fixing loop (Section IV), on hand-worked cases and invariants: the oracle's
reference (oracle/fixing.py) against the paper's text, the product's host versions (used to
build the reduced-LP batches) against the oracle, and the stored fixings of the mixed batch."""
import json
import os

import numpy as np
import pytest

from oracle import fixing as ofix
from paper_2510_10891_amd import fixing, scuc
from tests.helpers import highs, rel

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "algorithm1_cases.json")))


def test_round_operator_thresholds():
    tau = 0.1
    s = np.array([0.0, 0.1, 0.1000001, 0.5, 0.8999999, 0.9, 1.0, -1e-12])
    assert fixing.round_tau(s, tau).tolist() == [0, 0, -1, -1, -1, 1, 1, -1]


def test_oracle_round_operator_thresholds():
    tau = 0.1
    s = [0.0, 0.1, 0.1000001, 0.5, 0.8999999, 0.9, 1.0, -1e-12]
    assert [ofix.round_value(v, tau) for v in s] == [0, 0, -1, -1, -1, 1, 1, -1]


def cols_of(G, T):
    """[G][T][3] columns of (u, v, w) when unit g's hour t holds them at 3 (g T + t) + k."""
    return [[[3 * (g * T + t) + k for k in range(3)] for t in range(T)] for g in range(G)]


@pytest.mark.parametrize("case", GOLDEN["cases"], ids=[c["name"] for c in GOLDEN["cases"]])
def test_oracle_algorithm1_hand_worked(case):
    T = len(case["u"])
    x = np.zeros(3 * T)
    for t in range(T):
        x[3 * t:3 * t + 3] = case["u"][t], case["v"][t], case["w"][t]
    fixed, rounded = ofix.algorithm1(x, cols_of(1, T), case["tau"])
    hours = (np.nonzero(fixed[0])[0] + 1).tolist()
    assert hours == case["fixed"]
    assert [rounded[0, h - 1].tolist() for h in hours] == case["values"]


def test_product_algorithm1_matches_oracle_on_random_relaxations():
    rng = np.random.default_rng(3)
    G, T = 40, 24
    for tau in (0.05, 0.1, 0.3):
        u = np.clip(rng.choice([0, 1], (G, T)) + rng.normal(0, 0.1, (G, T)), 0, 1)
        v = np.clip(np.abs(rng.normal(0.0, 0.15, (G, T))), 0, 1)
        w = np.clip(np.abs(rng.normal(0.0, 0.15, (G, T))), 0, 1)
        x = np.stack([u, v, w], -1).reshape(-1)
        ofixed, orounded = ofix.algorithm1(x, cols_of(G, T), tau)
        fixed, ur, vr, wr = fixing.fixing_strategy(u, v, w, tau)
        assert np.array_equal(fixed, ofixed == 1)
        assert np.array_equal(np.stack([ur, vr, wr], -1), orounded)


def test_oracle_presolve_matches_the_products_and_keeps_the_optimum():
    data, lp = scuc.make_instance("small", 6)
    G, T = data.cfg.n_gen, data.cfg.T
    u, v, w = fixing.synthetic_relaxation(G, T, 0.5, np.random.default_rng(1))
    fixed, ur, vr, wr = fixing.fixing_strategy(u, v, w, 0.1)
    lo, hi = fixing.fix_bounds(lp, G, T, fixed, ur, vr, wr)
    full = lp.replace(col_lo=lo, col_hi=hi)
    red, kc, kr, feasible = ofix.presolve_fixed(full)
    pre = fixing.presolve_fixed(full)
    assert feasible and pre.feasible
    assert np.array_equal(kc, pre.cols) and np.array_equal(kr, pre.rows)
    assert np.array_equal(red.row_ptr, pre.lp.row_ptr) and np.array_equal(red.col_idx, pre.lp.col_idx)
    assert np.array_equal(red.val, pre.lp.val)
    for a, b in ((red.row_lo, pre.lp.row_lo), (red.row_hi, pre.lp.row_hi), (red.c, pre.lp.c)):
        fin = np.isfinite(b)
        assert np.array_equal(np.isfinite(a), fin) and np.allclose(a[fin], b[fin], rtol=1e-12, atol=1e-12)
    assert rel(red.obj_offset, pre.lp.obj_offset) < 1e-12
    a_obj, _, _ = highs(full)
    b_obj, _, _ = highs(red)
    assert rel(a_obj, b_obj) < 1e-9


def test_oracle_presolve_flags_a_violated_empty_row():
    from tests.helpers import dense_lp
    lp = dense_lp([[1.0, 0.0], [1.0, 1.0]], [2.0, 0.0], [np.inf, 5.0], [0, 0], [1, 1], [1.0, 1.0])
    fixed = lp.replace(col_lo=np.array([1.0, 0.0]), col_hi=np.array([1.0, 1.0]))
    assert not ofix.presolve_fixed(fixed)[3]


@pytest.mark.parametrize("case", GOLDEN["cases"], ids=[c["name"] for c in GOLDEN["cases"]])
def test_algorithm1_hand_worked(case):
    u, v, w = (np.array([case[k]], float) for k in ("u", "v", "w"))
    fixed, ur, vr, wr = fixing.fixing_strategy(u, v, w, case["tau"])
    hours = (np.nonzero(fixed[0])[0] + 1).tolist()
    assert hours == case["fixed"]
    vals = [[int(ur[0, h - 1]), int(vr[0, h - 1]), int(wr[0, h - 1])] for h in hours]
    assert vals == case["values"]


def test_algorithm1_invariants_on_random_relaxations():
    rng = np.random.default_rng(0)
    G, T = 50, 24
    u = np.clip(rng.choice([0, 1], (G, T)) + rng.normal(0, 0.08, (G, T)), 0, 1)
    v = np.clip(rng.normal(0.0, 0.08, (G, T)), 0, 1)
    w = np.clip(rng.normal(0.0, 0.08, (G, T)), 0, 1)
    for tau in (0.05, 0.1, 0.3):
        fixed, ur, vr, wr = fixing.fixing_strategy(u, v, w, tau)
        assert not fixed[:, 0].any()                      # hour 1 is never fixed
        for g in range(G):
            hrs = np.nonzero(fixed[g])[0]
            if len(hrs):                                  # a contiguous prefix from hour 2
                assert hrs.tolist() == list(range(1, 1 + len(hrs)))
            for t in hrs:                                 # the logic rows hold for fixed triples
                assert ur[g, t] - ur[g, t - 1] == vr[g, t] - wr[g, t]
                assert vr[g, t] + wr[g, t] <= 1 and min(ur[g, t], vr[g, t], wr[g, t]) >= 0


def test_presolve_keeps_the_optimum_of_the_fixed_lp():
    data, lp = scuc.make_instance("small", 6)
    G, T = data.cfg.n_gen, data.cfg.T
    rng = np.random.default_rng(1)
    u, v, w = fixing.synthetic_relaxation(G, T, 0.5, rng)
    fixed, ur, vr, wr = fixing.fixing_strategy(u, v, w, 0.1)
    assert fixed.any()
    lo, hi = fixing.fix_bounds(lp, G, T, fixed, ur, vr, wr)
    full = lp.replace(col_lo=lo, col_hi=hi)
    pre = fixing.presolve_fixed(full)
    assert pre.feasible
    assert pre.lp.n == lp.n - int((lo == hi).sum())
    a, xa, _ = highs(full)
    b, xb, _ = highs(pre.lp)
    assert rel(a, b) < 1e-9
    x = fixing.lift(pre, xb)
    assert abs(full.c @ x - a) <= 1e-7 * max(1, abs(a))
    ax = full.to_scipy() @ x
    assert np.all(ax >= full.row_lo - 1e-6) and np.all(ax <= full.row_hi + 1e-6)


def test_presolve_flags_a_violated_empty_row():
    from tests.helpers import dense_lp
    lp = dense_lp([[1.0, 0.0], [1.0, 1.0]], [2.0, 0.0], [np.inf, 5.0], [0, 0], [1, 1], [1.0, 1.0])
    fixed = lp.replace(col_lo=np.array([1.0, 0.0]), col_hi=np.array([1.0, 1.0]))
    pre = fixing.presolve_fixed(fixed)
    assert not pre.feasible                               # x0 = 1 cannot meet x0 >= 2


def test_reduced_batch_members_are_feasible_and_uneven():
    pres = fixing.make_reduced_batch(count=6, seed0=100, classes=2)
    assert all(p.feasible for p in pres)
    fracs = [p.lp.meta["fixed_u"] for p in pres]
    assert fracs[0] < fracs[-1]
    for p in pres[:2]:
        obj, _, _ = highs(p.lp)                           # every member has an optimum
        assert np.isfinite(obj)


def test_stored_fixings_are_algorithm1_outputs():
    """The stored fixings of the mixed batch (Algorithm 1 on oracle-solved relaxations): member
    i is parent class i mod 5 with seed 100 + i; per unit the fixed hours are one run starting
    at the second hour; on fixed hours the rounded binaries satisfy v + w <= 1 and, where the
    previous hour is fixed too, u_t - u_{t-1} = v_t - w_t; the share matches the record."""
    path = os.path.join(os.path.dirname(__file__), "golden", "fixing_masks_mixed.json")
    recs = fixing.load_fixings(path)
    assert len(recs) == 64
    shares = []
    for i, r in enumerate(recs):
        parent = fixing.BATCH_PARENTS[i % len(fixing.BATCH_PARENTS)]
        assert (r["parent"], r["seed"], r["G"], r["T"]) == (parent.name, 100 + i, parent.n_gen, parent.T)
        assert r["oracle_term"] == "solved" and r["oracle_rel_kkt"] <= 1e-4
        fixed, ur, vr, wr = fixing.decode_fixing(r)
        assert abs(fixed.mean() - r["fixed_u"]) < 1e-12
        assert not fixed[:, 0].any()
        run = np.cumprod(fixed[:, 1:], axis=1).astype(bool)      # the run from the second hour
        assert np.array_equal(run, fixed[:, 1:])
        assert np.all(vr[fixed] + wr[fixed] <= 1)
        both = fixed[:, 2:] & fixed[:, 1:-1]
        lhs = ur[:, 2:].astype(int) - ur[:, 1:-1]
        assert np.array_equal(lhs[both], (vr[:, 2:].astype(int) - wr[:, 2:])[both])
        assert not (ur[~fixed].any() or vr[~fixed].any() or wr[~fixed].any())
        shares.append(r["fixed_u"])
    assert min(shares) < 0.3 and max(shares) > 0.8


def test_stored_fixings_give_feasible_reduced_lps():
    path = os.path.join(os.path.dirname(__file__), "golden", "fixing_masks_mixed.json")
    recs = fixing.load_fixings(path)
    pres = fixing.make_reduced_batch(count=3, seed0=100, fixings=recs[:3])
    for p, r in zip(pres, recs):
        assert p.feasible and p.lp.meta["fixing_source"].startswith("solved relaxation")
        obj, _, _ = highs(p.lp)
        assert np.isfinite(obj)
    with pytest.raises(ValueError):                        # a record for another parent or seed
        fixing.reduced_lp(fixing.BATCH_PARENTS[1], 100, 0.5, fixing=recs[0])


def _highs_status(lp) -> int:
    import scipy.sparse as sp
    from scipy.optimize import linprog
    A = lp.to_scipy()
    eq = lp.row_lo == lp.row_hi
    ub = np.isfinite(lp.row_hi) & ~eq
    lb = np.isfinite(lp.row_lo) & ~eq
    res = linprog(lp.c, A_ub=sp.vstack([A[ub], -A[lb]]).tocsr(), b_ub=np.r_[lp.row_hi[ub], -lp.row_lo[lb]],
                  A_eq=A[eq], b_eq=lp.row_lo[eq], bounds=np.c_[lp.col_lo, lp.col_hi], method="highs")
    return int(res.status)


def test_some_stored_fixings_make_the_lp_infeasible():
    """Rounding and fixing a relaxed solution can leave no feasible dispatch (Section IV's
    intermediate models): HiGHS finds members 45, 55 and 60 of the mixed batch (30-bus
    parents, 73-81% of u fixed) infeasible and members 40 and 50 feasible."""
    path = os.path.join(os.path.dirname(__file__), "golden", "fixing_masks_mixed.json")
    recs = fixing.load_fixings(path)
    for i, status in ((40, 0), (45, 2), (50, 0), (55, 2), (60, 2)):
        parent = fixing.BATCH_PARENTS[i % len(fixing.BATCH_PARENTS)]
        pre = fixing.reduced_lp(parent, 100 + i, 0.0, fixing=recs[i])
        assert _highs_status(pre.lp) == status, i
