"""FP32 storage's floor: the stall test (HPR_STALLED) and the FP64 continuation from the
stalled point (mixed.py), against the oracle's FP64 solve."""
import numpy as np
import pytest

import oracle
from paper_2510_10891_amd import hprlp, mixed, scuc

pytestmark = pytest.mark.gpu

TIGHT = 1e-11   # below what FP32 storage reaches on these LPs (2^-24 rounding of A~ and iterates)


@pytest.mark.parametrize("seed", [0, 1])
def test_fp32_stalls_below_its_floor_and_fp64_finishes(seed):
    _, lp = scuc.make_instance("small", seed)
    stall = 1024
    opts = hprlp.Options(tol=TIGHT, precision=hprlp.HPR_FP32, max_iter=400000, stall_iters=stall)
    info, x, y, z = hprlp.solve(lp, opts)
    assert info.term == "stalled", info
    assert info.rel_kkt > TIGHT
    assert stall <= info.iters < opts.max_iter
    # the continuation: FP64 storage from that point reaches the tolerance
    cinfo, cx, cy, cz, continued = mixed.solve(lp, opts)
    assert continued and cinfo.term == "solved", cinfo
    assert cinfo.rel_kkt <= TIGHT
    assert cinfo.iters > info.iters
    ref = oracle.solve(lp, oracle.Options(tol=TIGHT, max_iter=400000))
    assert ref.term == "solved"
    assert abs(cinfo.pobj - ref.pobj) <= 1e-7 * (1 + abs(ref.pobj))
    # the continued point, judged by the oracle's own FP64 KKT evaluator
    assert oracle.kkt(lp, cx, cy, cz)["rel_kkt"] <= 2 * TIGHT


def test_fp64_storage_never_stalls():
    _, lp = scuc.make_instance("small", 0)
    info, *_ = hprlp.solve(lp, hprlp.Options(tol=0.0, precision=hprlp.HPR_FP64, max_iter=6000, stall_iters=64))
    assert info.term == "iter_limit" and info.iters == 6000


def test_stall_test_off_runs_to_the_limit():
    _, lp = scuc.make_instance("small", 0)
    info, *_ = hprlp.solve(lp, hprlp.Options(tol=TIGHT, precision=hprlp.HPR_FP32, max_iter=20000, stall_iters=0))
    assert info.term == "iter_limit" and info.iters == 20000


def test_batch_members_continue_in_fp64():
    """A batch of two LPs that cannot reach the tolerance with FP32 storage: both stall and are
    continued together as one FP64 batch from their points."""
    lps = [scuc.make_instance("small", s)[1] for s in (0, 1)]
    opts = hprlp.Options(tol=TIGHT, precision=hprlp.HPR_FP32, max_iter=400000, stall_iters=1024)
    b = hprlp.hpr_batch_create(lps, opts)
    try:
        infos = hprlp.hpr_batch_solve(b)
        assert all(i.term == "stalled" for i in infos), [i.term for i in infos]
        out, sols = mixed.continue_stalled(lps, opts, infos, lambda i: hprlp.hpr_batch_get_solution(b, i))
    finally:
        hprlp.hpr_batch_destroy(b)
    assert sorted(sols) == [0, 1]
    for k, lp in enumerate(lps):
        assert out[k].term == "solved" and out[k].rel_kkt <= TIGHT
        ref = oracle.solve(lp, oracle.Options(tol=TIGHT, max_iter=400000))
        assert abs(out[k].pobj - ref.pobj) <= 1e-7 * (1 + abs(ref.pobj))
        assert oracle.kkt(lp, *sols[k])["rel_kkt"] <= 2 * TIGHT
