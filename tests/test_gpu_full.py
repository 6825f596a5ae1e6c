"""GPU parity on the full SCUC formulation (cost segments, no-load cost, unserved demand in
the balance and security rows): iterates element by element against the oracle, and solves
to 1e-4 judged by the FP64 KKT evaluator. At the 2,000-bus size its security rows hold the
bus terms of the unserved demand, span more than 65,536 columns and are read through 32-bit
indices, 1.9e8 stored entries in all."""
import numpy as np
import pytest

import oracle
from paper_2510_10891_amd import fixing, hprlp, scuc
from tests.helpers import highs, rel
from tests.test_gpu_parity import FP32_RTOL, FP64_RTOL, assert_close, assert_parity, run_both

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("K", [1, 65, 1000])
@pytest.mark.parametrize("seed", [0, 1])
def test_full_small_fp64_iterates_match_oracle(seed, K):
    _, lp = scuc.make_instance("small", seed, formulation="full")
    o, info, x, y, z = run_both(lp, K)
    assert_parity(o, info, x, y, z, FP64_RTOL)


def test_full_small_fp32_iterates_track_oracle():
    _, lp = scuc.make_instance("small", 2, formulation="full")
    o, info, x, y, z = run_both(lp, 2, precision=hprlp.HPR_FP32)
    assert info.iters == o.iters
    assert_close(x, o.x, FP32_RTOL * 20, "x")
    assert_close(y, o.y, FP32_RTOL * 20, "y")


@pytest.mark.parametrize("precision", [hprlp.HPR_FP64, hprlp.HPR_FP32])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_full_small_reaches_tolerance(seed, precision):
    _, lp = scuc.make_instance("small", seed, formulation="full")
    info, x, y, z = hprlp.solve(lp, hprlp.Options(tol=1e-4, precision=precision, max_iter=400000))
    assert info.term == "solved", info
    ev = oracle.kkt(lp, x, y, z)
    assert ev["rel_kkt"] <= 1e-4 * (1 + 1e-6), ev
    assert abs(ev["rel_kkt"] - info.rel_kkt) <= 1e-6 + 1e-3 * info.rel_kkt
    if precision == hprlp.HPR_FP64:
        o = oracle.solve(lp, oracle.Options(tol=1e-4, max_iter=400000))
        assert o.iters == info.iters and rel(info.pobj, o.pobj) < 1e-8


@pytest.mark.parametrize("seed", [0, 1])
def test_full_small_tight_tolerance_matches_highs(seed):
    """At 1e-4 relative KKT a point of the full model can still be ~1% off the optimal
    objective (its primal residual is measured against the large bounds of the cost and
    penalty columns); at 1e-8, on the presolved model, the postsolved point reaches the optimum
    an interior-point solver finds."""
    _, lp = scuc.make_instance("small", seed, formulation="full")
    sub = fixing.presolve_free_singletons(lp)
    info, xr, yr, zr = hprlp.solve(sub.lp, hprlp.Options(tol=1e-8, max_iter=1000000))
    assert info.term == "solved", info
    x, y, z = fixing.postsolve_free_singletons(sub, xr, yr, zr)
    ev = oracle.kkt(lp, x, y, z)
    assert ev["rel_kkt"] <= 2e-8, ev
    assert rel(ev["pobj"], highs(lp)[0]) < 1e-6


def test_full_medium_parity_and_tolerance():
    """2,000-bus full formulation: 65 iterations against the oracle (lambda = 1 on both sides,
    a valid bound after the Pock-Chambolle scaling); then, with the cost variables substituted
    out by the presolve, an FP32-storage solve to 1e-4 whose postsolved point is judged on the
    original LP. Postsolve keeps every residual; only the dual residual's normalisation changes
    with the moved costs, by (1 + |c_reduced|) / (1 + |c|)."""
    _, lp = scuc.make_instance("medium", 0, formulation="full")
    span = max(lp.col_idx[a:b].max() - lp.col_idx[a:b].min()
               for a, b in zip(lp.row_ptr[:-1:997], lp.row_ptr[1::997]) if b > a)
    assert span >= 65536     # wide rows present
    o, info, x, y, z = run_both(lp, 65, lambda_in=1.0)
    assert_parity(o, info, x, y, z, FP64_RTOL)
    sub = fixing.presolve_free_singletons(lp)
    assert len(sub.sub_c) == 500 * 48
    info, xr, yr, zr = hprlp.solve(sub.lp, hprlp.Options(tol=1e-4, precision=hprlp.HPR_FP32, max_iter=100000,
                                                         time_limit_s=100.0))
    ev_red = oracle.kkt(sub.lp, xr, yr, zr)
    assert abs(ev_red["rel_kkt"] - info.rel_kkt) <= 1e-6 + 1e-3 * info.rel_kkt
    assert info.term == "solved", info
    assert ev_red["rel_kkt"] <= 1e-4 * (1 + 1e-6), ev_red
    x, y, z = fixing.postsolve_free_singletons(sub, xr, yr, zr)
    ev = oracle.kkt(lp, x, y, z)
    factor = max(1.0, (1 + np.linalg.norm(sub.lp.c)) / (1 + np.linalg.norm(lp.c)))
    assert ev["rel_kkt"] <= 1e-4 * factor * (1 + 1e-6), (ev, factor)
    assert abs(ev["pobj"] - ev_red["pobj"]) <= 1e-9 * (1 + abs(ev_red["pobj"]))
