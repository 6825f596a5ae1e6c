"""Algorithm 1 (Fixing-Strategy), the Round operator and the LP presolve of the
successive-fixing loop (Section IV), on hand-worked cases and invariants."""
import json
import os

import numpy as np
import pytest

from paper_2510_10891_amd import fixing, scuc
from tests.helpers import highs, rel

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "algorithm1_cases.json")))


def test_round_operator_thresholds():
    tau = 0.1
    s = np.array([0.0, 0.1, 0.1000001, 0.5, 0.8999999, 0.9, 1.0, -1e-12])
    assert fixing.round_tau(s, tau).tolist() == [0, 0, -1, -1, -1, 1, 1, -1]


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
