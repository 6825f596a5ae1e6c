"""Pins of the full SCUC formulation (Section II with cost segments, no-load cost and
unserved demand): each checked against something other than the builder itself — the
compact form it must reduce to, an independent DC power flow, HiGHS, and identities of
the model."""
import numpy as np
import pytest

import oracle
from paper_2510_10891_amd import scuc
from tests.helpers import highs
from tests.test_scuc_generator import _flows_with_slack


def _pen_cols(data, lp):
    G, T, B, H = data.cfg.n_gen, data.cfg.T, data.cfg.n_bus, lp.meta["segments"]
    return scuc.pen_col_index(G, H, T, B, np.arange(T)[:, None], np.arange(B)[None, :]).ravel()


def _extra(data, lp, slot):
    G, T, H = data.cfg.n_gen, data.cfg.T, lp.meta["segments"]
    return scuc.full_col_index(G, H, np.arange(T)[None, :], slot, np.arange(G)[:, None], T)   # [G, T]


@pytest.mark.parametrize("seed", [0, 1, 3])
def test_one_segment_without_unserved_demand_is_the_compact_lp(seed):
    """With one segment priced at the unit's cost, C^L = cost * P^L and d^pen held at 0, the
    full model is the compact one after the change of variables p = p' + P^L u: same optimum."""
    _, compact = scuc.make_instance("small", seed)
    data, full = scuc.make_instance("small", seed, formulation="full", segments=1)
    hi = full.col_hi.copy()
    hi[_pen_cols(data, full)] = 0.0
    oc = highs(compact)[0] * compact.meta["eta_c"]
    of = highs(full.replace(col_hi=hi))[0] * full.meta["eta_c"]
    assert abs(of - oc) <= 1e-9 * abs(oc)


def test_instance_scaling_only_changes_units():
    """Section III-A: the scaled optimum times eta^C is the unscaled optimum."""
    _, scaled = scuc.make_instance("small", 2, formulation="full")
    _, plain = scuc.make_instance("small", 2, instance_scaling=False, formulation="full")
    assert scaled.meta["eta_c"] > 1.0 and plain.meta["eta_c"] == 1.0
    o1 = highs(scaled)[0] * scaled.meta["eta_c"]
    o2 = highs(plain)[0]
    assert abs(o1 - o2) <= 1e-8 * abs(o2)


def test_all_on_dispatch_is_feasible():
    for name, seed in (("small", 0), ("small", 5)):
        data, lp = scuc.make_instance(name, seed, formulation="full")
        x = scuc.feasible_point_full(data, lp)
        ax = lp.to_scipy() @ x
        tol = 1e-9 * (1 + np.abs(ax))
        assert np.all(ax >= lp.row_lo - tol) and np.all(ax <= lp.row_hi + tol)
        assert np.all(x >= lp.col_lo) and np.all(x <= lp.col_hi + 1e-12)


def test_security_rows_are_post_outage_flows_of_the_bus_injection():
    """Row activity minus the row's midpoint = flow on the monitored line after the outage,
    for injection sum_{g at b} p_g - D_b + d^pen_b: the bus-level coefficients (with d^pen) against
    flows re-solved on the network without the outaged line (no LODF)."""
    cfg = scuc.SCUCConfig(40, 60, 12, 4, 10, 3, 0.0, "t")
    data = scuc.make_scuc_data(cfg, 3, bus_rows=True)
    lp = scuc.build_full_lp(data, instance_scaling=False)
    rng = np.random.default_rng(3)          # the generator's own first draws: the network
    fr, to, x = scuc.random_network(rng, cfg.n_bus, cfg.n_line)
    net = scuc.DCNetwork(fr, to, x, cfg.n_bus)
    r = np.random.default_rng(11)
    xv = np.zeros(lp.n)
    G, T, B = cfg.n_gen, cfg.T, cfg.n_bus
    for t in range(T):
        xv[scuc.col_index(G, t, scuc.P, np.arange(G))] = r.uniform(0, 1, G) * data.p_max
    pen = _pen_cols(data, lp)
    xv[pen] = r.uniform(0, 1, len(pen)) * lp.col_hi[pen]
    act = lp.to_scipy() @ xv
    kinds = lp.meta["row_kind"]
    sec = np.nonzero(kinds == lp.meta["row_kinds"]["security"])[0]
    checked = 0
    for i in sec:
        t = int(lp.meta["row_hour"][i])
        s = int(lp.meta["row_sec"][i])
        mon, out = data.sec_label[s]
        p = xv[scuc.col_index(G, t, scuc.P, np.arange(G))]
        inj = np.bincount(data.gen_bus, weights=p, minlength=B) - data.demand[t] * data.bus_share
        inj += xv[scuc.pen_col_index(G, lp.meta["segments"], T, B, t, np.arange(B))]
        f = _flows_with_slack(net, inj, 0, None if out < 0 else int(out))
        mid = 0.5 * (lp.row_lo[i] + lp.row_hi[i])
        assert abs((act[i] - mid) - f[mon]) <= 1e-9 * (1 + np.abs(f).max()), (i, mon, out)
        checked += 1
    assert checked == len(sec) > 0


@pytest.mark.parametrize("seed", [0, 4])
def test_optimum_identities(seed):
    """At an optimal point: p = p' + P^L u, sum of segments = p', c = sum C_h p_h, the logic
    identity u_t - u_{t-1} = v_t - w_t, and segments filled cheapest first (only their sum
    enters the other rows and the costs increase)."""
    data, lp = scuc.make_instance("small", seed, formulation="full", instance_scaling=False)
    _, x, _ = highs(lp)
    G, T, H = data.cfg.n_gen, data.cfg.T, lp.meta["segments"]
    g, t = np.arange(G)[:, None], np.arange(T)[None, :]
    u = x[scuc.col_index(G, t, scuc.U, g)]
    v = x[scuc.col_index(G, t, scuc.V, g)]
    w = x[scuc.col_index(G, t, scuc.W, g)]
    p = x[scuc.col_index(G, t, scuc.P, g)]
    pa = x[_extra(data, lp, 0)]
    seg = np.stack([x[_extra(data, lp, 1 + h)] for h in range(H)], 0)   # [H, G, T]
    c = x[_extra(data, lp, H + 1)]
    width, cost, _ = scuc.segment_data(data, H)
    assert np.allclose(p, pa + data.p_min[:, None] * u, atol=1e-6)
    assert np.allclose(seg.sum(0), pa, atol=1e-6)
    assert np.allclose(c, np.einsum("hgt,gh->gt", seg, cost), rtol=1e-7, atol=1e-4)
    du = np.diff(np.concatenate([np.ones((G, 1)), u], 1), axis=1)
    assert np.allclose(du, v - w, atol=1e-7)
    assert np.all(np.diff(cost, axis=1) > 0)
    for h in range(1, H):
        # a dearer segment in use => every cheaper one at its limit width * u
        busy = seg[h] > 1e-6
        for k in range(h):
            assert np.all(seg[k][busy] >= width[:, k][:, None].repeat(T, 1)[busy] * u[busy] - 1e-6)


def test_unserved_demand_keeps_an_overloaded_system_feasible():
    """Demand above the total capacity: the compact model is infeasible, the full one serves
    what it can and leaves at least (demand - capacity) unserved in every hour."""
    data = scuc.make_scuc_data(scuc.SMALL, 1, bus_rows=True)
    cap = data.p_max.sum()
    data.demand = data.demand * (1.3 * cap / data.demand.min())
    with pytest.raises(AssertionError, match="nfeasible"):
        highs(scuc.build_lp(data, instance_scaling=False))
    lp = scuc.build_full_lp(data, instance_scaling=False)
    _, x, _ = highs(lp)
    G, T, B = data.cfg.n_gen, data.cfg.T, data.cfg.n_bus
    for t in range(T):
        d = x[scuc.pen_col_index(G, lp.meta["segments"], T, B, t, np.arange(B))].sum()
        assert d >= data.demand[t] - cap - 1e-6 * data.demand[t]


def test_oracle_solves_the_full_formulation():
    """The oracle's HPR iteration on the full model reaches 1e-6 relative KKT, and its
    objective agrees with HiGHS."""
    data, lp = scuc.make_instance("small", 0, formulation="full")
    ref = highs(lp)[0]
    r = oracle.solve(lp, oracle.Options(tol=1e-6, max_iter=400000))
    assert r.term == "solved", (r.term, r.iters, r.rel_kkt)
    assert abs(r.pobj - ref) <= 1e-5 * (1 + abs(ref))
    ev = oracle.kkt(lp, r.x, r.y, r.z)
    assert ev["rel_kkt"] <= 1e-6 * (1 + 1e-9)
