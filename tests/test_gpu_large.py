"""The 13,500-bus instance (4,000 units, 36 h, 1,000 monitored lines x (1 + 20 outages);
m = 1.82e6, n = 5.76e5, nnz = 2.84e8) at full size, in the launch configuration the bench
uses: short runs element by element against the oracle, and an FP32-storage solve judged
by the FP64 KKT evaluator.

lambda = 1 is given to both sides (a valid bound after the Pock-Chambolle scaling), so the
oracle's power method on 2.8e8 entries is not needed for the comparison."""
import numpy as np
import pytest

import oracle
from paper_2510_10891_amd import hprlp, scuc
from tests.test_gpu_parity import FP64_RTOL, assert_close, assert_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def large():
    return scuc.make_instance("large", 0)[1]


def test_large_fp64_and_fp32_iterates_match_oracle(large):
    lp = large
    o65 = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=65, lambda_in=1.0))
    info, x, y, z = hprlp.solve(lp, hprlp.Options(tol=0.0, max_iter=65, lambda_=1.0))
    assert_parity(o65, info, x, y, z, FP64_RTOL)
    info, x, y, z = hprlp.solve(lp, hprlp.Options(tol=0.0, max_iter=65, lambda_=1.0, precision=hprlp.HPR_FP32))
    assert info.iters == o65.iters
    assert_close(x, o65.x, 2e-4, "x")
    assert_close(y, o65.y, 2e-4, "y")


@pytest.fixture(scope="module")
def large_o65(large):
    return oracle.solve(large, oracle.Options(tol=0.0, max_iter=65, lambda_in=1.0))


@pytest.mark.parametrize("mode,precision", [(4, hprlp.HPR_FP64), (5, hprlp.HPR_FP64), (3, hprlp.HPR_FP32),
                                            (4, hprlp.HPR_FP32), (5, hprlp.HPR_FP32), (6, hprlp.HPR_FP64),
                                            (7, hprlp.HPR_FP32)])
def test_large_regrouped_sliced_windows_match_oracle(large, large_o65, mode, precision):
    """Sliced windows with the long rows regrouped to 16 (mode 4) or 8 (mode 5) lanes per row,
    every row capped at 16 or 8 lanes (modes 6, 7), and the sliced modes in FP32 storage
    (4,096-column windows): 65 iterations against the oracle (FP64 storage at the FP64
    tolerance, FP32 storage at the FP32 tolerance)."""
    lp, o65 = large, large_o65
    h = hprlp.hpr_create(lp, hprlp.Options(tol=0.0, max_iter=65, lambda_=1.0, lds_windows=mode, unroll=2,
                                           precision=precision))
    try:
        info = hprlp.hpr_solve(h)
        x, y, z = hprlp.hpr_get_solution(h)
        ks = hprlp.hpr_get_kernel_stats(h)
    finally:
        hprlp.hpr_destroy(h)
    assert ks["sliced_blocks_at"] > 0, ks
    if precision == hprlp.HPR_FP64:
        assert_parity(o65, info, x, y, z, FP64_RTOL)
    else:
        assert info.iters == o65.iters
        assert_close(x, o65.x, 2e-4, "x")
        assert_close(y, o65.y, 2e-4, "y")


def test_large_sliced_windows_match_oracle(large):
    """The primal step of this instance reads y through sliced LDS windows (a unit's output
    column meets the 21,000 security rows of its hour): 65 FP64 iterations with lds_windows = 3
    against the oracle."""
    lp = large
    o65 = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=65, lambda_in=1.0))
    h = hprlp.hpr_create(lp, hprlp.Options(tol=0.0, max_iter=65, lambda_=1.0, lds_windows=3, unroll=2))
    try:
        info = hprlp.hpr_solve(h)
        x, y, z = hprlp.hpr_get_solution(h)
        ks = hprlp.hpr_get_kernel_stats(h)
    finally:
        hprlp.hpr_destroy(h)
    assert ks["sliced_blocks_at"] > 0
    assert_parity(o65, info, x, y, z, FP64_RTOL)


def test_large_fp32_solve_reaches_tolerance(large):
    lp = large
    info, x, y, z = hprlp.solve(lp, hprlp.Options(tol=1e-4, precision=hprlp.HPR_FP32, max_iter=60000,
                                                  time_limit_s=150.0))
    ev = oracle.kkt(lp, x, y, z)
    assert abs(ev["rel_kkt"] - info.rel_kkt) <= 1e-6 + 1e-3 * info.rel_kkt
    if info.term == "solved":
        assert ev["rel_kkt"] <= 1e-4 * (1 + 1e-6)
    else:
        pytest.skip(f"not solved within the test's limits: {info.term} after {info.iters} iterations, "
                    f"rel_kkt {info.rel_kkt:.2e}")
