"""Successive fixing (Algorithm 2 without the MILP steps) driving re-solves on one handle."""
import numpy as np
import pytest

from paper_2510_10891_amd import fixing, hprlp, scuc, successive
from tests.helpers import highs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed", [0, 3])
def test_rounds_fix_more_and_stay_consistent(seed):
    """Seed 0 stays feasible for 4 rounds. On seed 3 the first fixing switches off units whose
    relaxed commitment is below tau for the whole horizon, which leaves too little capacity
    behind the line limits: the logic check of Algorithm 1 keeps eq.(status) consistent, not
    the balance and security rows (Section IV-A claims better feasibility, not a guarantee).
    The solver must certify that round's LP infeasible, the loop must stop there, and an
    independent solver must agree."""
    data, lp = scuc.make_instance("small", seed)
    G, T = data.cfg.n_gen, data.cfg.T
    opts = hprlp.Options(tol=1e-6, max_iter=50000)
    res = successive.run(data, lp, rounds=4, tau=0.1, opts=opts)
    assert res.rounds[0].term == "solved"
    assert all(r.term == "solved" for r in res.rounds[:-1])
    if res.rounds[-1].term != "solved":
        assert res.rounds[-1].term == "primal_infeasible"
        with pytest.raises(AssertionError, match="nfeasible"):
            highs(lp.replace(col_lo=res.col_lo, col_hi=res.col_hi))
        res.rounds.pop()
    else:
        assert len(res.rounds) == 4
    fr = [r.fixed_u for r in res.rounds]
    assert all(b >= a for a, b in zip(fr, fr[1:])) and fr[-1] > 0
    objs = [r.objective for r in res.rounds]
    for a, b in zip(objs, objs[1:]):           # each round's LP restricts the previous one
        assert b >= a - 1e-4 * abs(a)
    fixed = res.col_lo == res.col_hi
    assert fixed.any()
    # the fixed triples satisfy the logic rows of eq.(status) with the rounded values
    u = res.col_lo[scuc.col_index(G, np.arange(T)[None, :], scuc.U, np.arange(G)[:, None])]
    v = res.col_lo[scuc.col_index(G, np.arange(T)[None, :], scuc.V, np.arange(G)[:, None])]
    w = res.col_lo[scuc.col_index(G, np.arange(T)[None, :], scuc.W, np.arange(G)[:, None])]
    fu = fixed[scuc.col_index(G, np.arange(T)[None, :], scuc.U, np.arange(G)[:, None])]
    assert not fu[:, 0].any()                 # Algorithm 1 never fixes hour 1
    for g, t in zip(*np.nonzero(fu)):
        if fu[g, t - 1]:
            assert u[g, t] - u[g, t - 1] == v[g, t] - w[g, t]
            assert v[g, t] + w[g, t] <= 1
    if len(res.rounds) == 4:   # the final restricted LP still has an optimum (independent LP solver)
        obj, _, _ = highs(lp.replace(col_lo=res.col_lo, col_hi=res.col_hi))
        assert np.isfinite(obj) and obj >= objs[0] - 1e-4 * abs(objs[0])


def test_warm_started_rounds_need_fewer_iterations():
    data, lp = scuc.make_instance("small", 1)
    opts = hprlp.Options(tol=1e-6, max_iter=200000, warm_fallback=0)
    warm = successive.run(data, lp, rounds=3, opts=opts, warm=True)
    cold = successive.run(data, lp, rounds=3, opts=opts, warm=False)
    assert [r.fixed_u for r in warm.rounds] and warm.rounds[0].iters == cold.rounds[0].iters
    assert sum(r.iters for r in warm.rounds[1:]) < sum(r.iters for r in cold.rounds[1:])
