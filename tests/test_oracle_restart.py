"""Pins of the oracle's merit, restart rule and sigma update (Section III names adaptive
sigma updates and restart schemes without giving their rules; Theorem 1 fixes the metric
they rest on).

* The merit is the norm of the fixed-point residual w^k - wbar^{k+1} in the metric in which
  one step of eq.(hpr) is firmly nonexpansive. That metric is found here independently: of
  the two candidate cross-term signs, only M = [[I/sigma, A^T], [A, lambda sigma I]] makes
  random pairs of steps firmly nonexpansive; the oracle's merit is then compared with the
  densely assembled quadratic form at real checks of a solve.
* sigma* is compared with the numerical minimiser of ||dx||^2/sigma + lambda sigma ||dy||^2.
* The restart rule is driven through hand-worked merit sequences, and the trace of real
  solves is checked for the state it must keep (r0 reset at each restart, k counted from
  the last restart, sigma carried from one check to the next).
"""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import oracle
from paper_2510_10891_amd import scuc
from tests.helpers import dense_lp


def tiny(seed, m=5, n=4):
    return scuc.random_lp(np.random.default_rng(seed), m, n)


def metric(A, sigma, lam, sign=1.0):
    m, n = A.shape
    return np.block([[np.eye(n) / sigma, sign * A.T], [sign * A, lam * sigma * np.eye(m)]])


def scaled_problem(lp, opts=None):
    """The scaled LP the oracle iterates on, rebuilt from its scaling factors."""
    dr, dc, bb, bc, lam, _ = oracle.scaling(lp, opts)
    A = lp.to_scipy().toarray()
    As = dr[:, None] * A * dc[None, :]
    sp = dense_lp(As, dr * lp.row_lo / bb, dr * lp.row_hi / bb, lp.col_lo / (bb * dc),
                  lp.col_hi / (bb * dc), dc * lp.c / bc)
    return As, sp, lam


# ----------------------------------------------------------------------------- the metric

@pytest.mark.parametrize("seed", range(6))
def test_only_the_plus_metric_makes_the_step_firmly_nonexpansive(seed):
    """||Tw - Tw'||_M^2 <= <Tw - Tw', w - w'>_M for T = one step of eq.(hpr) (the bar point)."""
    lp = tiny(seed)
    A = lp.to_scipy().toarray()
    lam = 1.01 * np.linalg.eigvalsh(A @ A.T).max()
    rng = np.random.default_rng(100 + seed)
    worst = {1.0: -np.inf, -1.0: -np.inf}
    for sigma in (0.3, 1.0, 3.0):
        Mp, Mm = metric(A, sigma, lam, 1.0), metric(A, sigma, lam, -1.0)
        for _ in range(200):
            w = [rng.normal(0, 2, lp.n), rng.normal(0, 2, lp.m)]
            v = [rng.normal(0, 2, lp.n), rng.normal(0, 2, lp.m)]
            _, _, xb1, yb1, _ = oracle.hpr_step(lp, sigma, lam, 0, w[0], w[1], w[0], w[1])
            _, _, xb2, yb2, _ = oracle.hpr_step(lp, sigma, lam, 0, v[0], v[1], v[0], v[1])
            d = np.r_[xb1 - xb2, yb1 - yb2]
            e = np.r_[w[0] - v[0], w[1] - v[1]]
            for sign, M in ((1.0, Mp), (-1.0, Mm)):
                gap = d @ M @ d - d @ M @ e
                worst[sign] = max(worst[sign], gap / (1.0 + e @ e))
    assert worst[1.0] <= 1e-10
    assert worst[-1.0] > 1e-6          # the other sign is not a metric of the step


@pytest.mark.parametrize("which", [("small", 0), ("small", 1), ("tiny", 3)])
def test_merit_is_the_dense_m_norm_of_the_fixed_point_residual(which):
    lp = scuc.make_instance("small", which[1])[1] if which[0] == "small" else tiny(which[1], 6, 5)
    As, sp, lam = scaled_problem(lp)
    res, tr, _ = oracle.solve_trace(lp, oracle.Options(tol=0.0, max_iter=64 * 6 + 1))
    assert len(tr["it"]) >= 5
    for c in (1, 2, 4):
        _, tr2, v = oracle.solve_trace(lp, oracle.Options(tol=0.0, max_iter=64 * 6 + 1), vec_check=c)
        sigma = tr2["sigma"][c]
        # the vectors are the step's start and its bar point: one step from them reproduces it
        k = int(tr2["k"][c]) - 1
        _, _, xb, yb, _ = oracle.hpr_step(sp, sigma, res.lam, k, v["x0"], v["y0"], v["x"], v["y"])
        assert np.allclose(xb, v["xbar"], rtol=0, atol=1e-13) and np.allclose(yb, v["ybar"], rtol=0, atol=1e-13)
        d = np.r_[v["x"] - v["xbar"], v["y"] - v["ybar"]]
        r_dense = np.sqrt(max(d @ metric(As, sigma, res.lam) @ d, 0.0))
        assert abs(tr2["r"][c] - r_dense) <= 1e-10 * r_dense


# ----------------------------------------------------------------------------- sigma*

def numeric_sigma_star(ndx, ndy, lam):
    f = lambda ls: ndx ** 2 / np.exp(ls) + lam * np.exp(ls) * ndy ** 2
    r = minimize_scalar(f, bounds=(-30, 30), method="bounded", options=dict(xatol=1e-12))
    return float(np.exp(r.x))


@pytest.mark.parametrize("ndx,ndy,lam", [(1.0, 1.0, 1.0), (3.0, 0.2, 0.5), (0.01, 4.0, 0.98),
                                         (2.5, 0.7, 0.25), (1e-3, 1e-3, 1.0)])
def test_sigma_star_is_the_minimiser_of_the_diagonal_metric(ndx, ndy, lam):
    star = numeric_sigma_star(ndx, ndy, lam)
    assert abs(oracle.sigma_next(0.37, ndx, ndy, lam, 1.0) - star) <= 1e-6 * star
    # half weight: the geometric mean of the old sigma and sigma*
    assert abs(oracle.sigma_next(0.37, ndx, ndy, lam, 0.5) - np.sqrt(0.37 * star)) <= 1e-6 * star
    # a general weight interpolates in log space
    w = 0.3
    exp = np.exp(0.7 * np.log(0.37) + w * np.log(star))
    assert abs(oracle.sigma_next(0.37, ndx, ndy, lam, w) - exp) <= 1e-6 * exp


def test_sigma_update_is_clamped_and_skipped_on_tiny_moves():
    assert oracle.sigma_next(1.0, 1e6, 1e-6, 1.0, 1.0) == 1e4
    assert oracle.sigma_next(1.0, 1e-6, 1e6, 1.0, 1.0) == 1e-4
    assert oracle.sigma_next(0.5, 1e-13, 1.0, 1.0, 1.0) == 0.5
    assert oracle.sigma_next(0.5, 1.0, 1e-13, 1.0, 1.0) == 0.5


@pytest.mark.parametrize("warm", [False, True])
def test_sigma_at_real_restarts_minimises_the_anchor_move(warm, small_instances):
    _, lp = small_instances[0]
    x0 = y0 = None
    if warm:
        ref = oracle.solve(lp, oracle.Options(tol=1e-6, max_iter=100000))
        rng = np.random.default_rng(1)
        x0 = ref.x * (1 + 0.05 * rng.standard_normal(lp.n))
        y0 = ref.y * (1 + 0.3 * rng.standard_normal(lp.m))
    opts = oracle.Options(tol=0.0, max_iter=64 * 12 + 1)
    _, tr, _ = oracle.solve_trace(lp, opts, x0=x0, y0=y0)
    restarts = np.nonzero(tr["restart"])[0]
    assert len(restarts) >= 3
    for c in restarts[:3]:
        res2, tr2, v = oracle.solve_trace(lp, opts, x0=x0, y0=y0, vec_check=int(c))
        ndx = np.linalg.norm(v["xbar"] - v["x0"])
        ndy = np.linalg.norm(v["ybar"] - v["y0"])
        assert abs(ndx - tr2["ndx"][c]) <= 1e-12 * ndx and abs(ndy - tr2["ndy"][c]) <= 1e-12 * ndy
        star = np.clip(numeric_sigma_star(ndx, ndy, res2.lam), 1e-4, 1e4)
        expect = star if not warm else np.sqrt(tr2["sigma"][c] * star)
        assert abs(tr2["sigma_next"][c] - expect) <= 1e-6 * expect


# ----------------------------------------------------------------------------- restart rule

# (r, k, done, expected decision) at successive checks; worked out by hand from the rule:
# restart iff r <= 0.2 r0, or r <= 0.8 r0 and r > r_prev, or k >= 0.2 done; the first check
# only sets r0 = r_prev = r; a restart sets r0 = r.
SEQUENCES = {
    "sufficient decay": [(5.0, 1, 1, False), (4.5, 64, 1000, False), (0.99, 128, 1064, True),
                         (0.9, 64, 1128, False)],
    "sufficient decay at equality": [(5.0, 1, 1, False), (1.0, 64, 1000, True)],
    "necessary decay without progress": [(10.0, 1, 1, False), (7.9, 64, 1000, False),
                                         (7.95, 128, 1064, True)],
    "no progress above 0.8 r0": [(10.0, 1, 1, False), (8.5, 64, 1000, False),
                                 (9.0, 128, 1064, False)],
    "r0 is reset at a restart": [(10.0, 1, 1, False), (7.9, 64, 1000, False), (7.95, 128, 1064, True),
                                 (1.7, 64, 1128, False), (1.5, 128, 1192, True)],
    "r_prev follows every check": [(10.0, 1, 1, False), (7.5, 64, 1000, False),
                                   (7.6, 128, 1064, True)],
    "long run since the restart": [(3.0, 1, 1, False), (2.9, 59, 300, False), (2.95, 60, 300, True)],
    "first check never restarts": [(0.0, 1, 1, False), (1.0, 64, 65, True)],
}


@pytest.mark.parametrize("name", list(SEQUENCES))
def test_restart_rule_on_hand_worked_sequences(name):
    rule = oracle.RestartRule()
    for r, k, done, expect in SEQUENCES[name]:
        assert rule(r, k, done) == expect, (name, r, k, done)


def test_restart_rule_state_after_a_restart():
    rule = oracle.RestartRule()
    for r, k, done, _ in SEQUENCES["r0 is reset at a restart"][:3]:
        rule(r, k, done)
    assert rule.r0 == 7.95 and rule.r_prev == 7.95
    rule(1.7, 64, 1128)
    assert rule.r0 == 7.95 and rule.r_prev == 1.7


def test_restart_rule_disabled_never_restarts():
    rule = oracle.RestartRule(enabled=False)
    assert [rule(r, k, d) for r, k, d, _ in SEQUENCES["sufficient decay"]] == [False] * 4


@pytest.mark.parametrize("which", [0, 1, 2])
def test_trace_of_a_solve_keeps_the_rules_state(which, small_instances):
    _, lp = small_instances[which]
    res, tr, _ = oracle.solve_trace(lp, oracle.Options(tol=1e-6, max_iter=100000))
    n = len(tr["it"])
    assert n >= 5 and int(tr["restart"].sum()) == res.restarts
    it, k, r = tr["it"].astype(int), tr["k"].astype(int), tr["r"]
    last_restart_it, r_at_restart = None, r[0]
    for c in range(n):
        # k counts the steps since the last restart (from the start before the first one)
        expect_k = it[c] + 1 if last_restart_it is None else it[c] - last_restart_it
        assert k[c] == expect_k, c
        if c > 0:
            assert tr["r0"][c] == r_at_restart, c           # r0: the merit at the last restart
            assert tr["r_prev"][c] == r[c - 1], c            # r_prev: the previous check's merit
            assert tr["sigma"][c] == tr["sigma_next"][c - 1], c
        if tr["restart"][c]:
            last_restart_it, r_at_restart = it[c], r[c]
        else:
            assert tr["sigma_next"][c] == tr["sigma"][c]
    # the decisions are the rule's on the recorded merits
    rule = oracle.RestartRule()
    assert [rule(r[c], k[c], it[c] + 1) for c in range(n)] == tr["restart"].astype(bool).tolist()
