"""Batched solves: many uneven LPs in one pooled problem (one launch per half-iteration
for all of them, per-LP control on the device, graph-captured iteration blocks).

Each LP of a batch must follow the single-LP schedule exactly, so short runs are compared
element by element with the CPU oracle run on that LP alone."""
import numpy as np
import pytest

import oracle
from paper_2510_10891_amd import fixing, hprlp, scuc
from tests.test_gpu_parity import FP32_RTOL, FP64_RTOL, assert_close, assert_parity, ragged_lp

pytestmark = pytest.mark.gpu


def uneven_batch():
    lps = [scuc.make_instance("small", s)[1] for s in range(3)]
    lps += [ragged_lp(s, m=150 + 60 * s, n=300 + 50 * s) for s in range(3)]
    lps += [scuc.random_lp(np.random.default_rng(s), 5, 4) for s in range(2)]
    return lps


@pytest.mark.parametrize("use_graph", [1, 0])
@pytest.mark.parametrize("K", [1, 65, 300])
def test_batch_iterates_match_oracle_per_lp(K, use_graph):
    lps = uneven_batch()
    out = hprlp.batch_solve(lps, hprlp.Options(tol=0.0, max_iter=K, use_graph=use_graph))
    for lp, (info, x, y, z) in zip(lps, out):
        o = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=K))
        assert_parity(o, info, x, y, z, FP64_RTOL)


def test_batch_full_solves_match_single_solves():
    """With the same schedule (U fixed) a batch member is bitwise the single solve."""
    lps = [scuc.make_instance("small", s)[1] for s in range(8)]
    out = hprlp.batch_solve(lps, hprlp.Options(tol=1e-4, max_iter=200000, unroll=4))
    for lp, (info, x, y, z) in zip(lps, out):
        assert info.term == "solved"
        assert oracle.kkt(lp, x, y, z)["rel_kkt"] <= 1e-4 * (1 + 1e-6)
        single, xs, ys, zs = hprlp.solve(lp, hprlp.Options(tol=1e-4, max_iter=200000, unroll=4))
        assert single.iters == info.iters and single.restarts == info.restarts
        assert np.array_equal(xs, x) and np.array_equal(ys, y)


def test_graph_and_direct_launches_are_bitwise_identical():
    """Same schedule (U fixed: the tuner's timed choice may differ between two engines and U
    sets the summation order), graph replay vs direct launches: identical bits."""
    lps = uneven_batch()
    a = hprlp.batch_solve(lps, hprlp.Options(tol=1e-6, max_iter=20000, use_graph=1, unroll=4))
    b = hprlp.batch_solve(lps, hprlp.Options(tol=1e-6, max_iter=20000, use_graph=0, unroll=4))
    for (ia, xa, ya, za), (ib, xb, yb, zb) in zip(a, b):
        assert ia.iters == ib.iters and ia.term == ib.term
        assert np.array_equal(xa, xb) and np.array_equal(ya, yb) and np.array_equal(za, zb)


def test_unsolvable_member_does_not_hold_back_the_others():
    bad = scuc.LP(1, 2, np.array([0, 2], np.int64), np.array([0, 1], np.int32), np.array([1.0, 1.0]),
                  np.array([3.0]), np.array([np.inf]), np.zeros(2), np.ones(2), np.ones(2))
    lps = [scuc.make_instance("small", 0)[1], bad, scuc.make_instance("small", 1)[1]]
    out = hprlp.batch_solve(lps, hprlp.Options(tol=1e-4, max_iter=6000))
    assert out[0][0].term == "solved" and out[2][0].term == "solved"
    assert out[1][0].term == "primal_infeasible" and out[1][0].iters < 6000
    for lp, (info, x, y, z) in zip(lps, out):
        if info.term == "solved":
            assert oracle.kkt(lp, x, y, z)["rel_kkt"] <= 1e-4 * (1 + 1e-6)


def test_fp32_batch_reaches_tolerance_in_fp64():
    lps = [scuc.make_instance("small", s)[1] for s in range(4, 10)]
    out = hprlp.batch_solve(lps, hprlp.Options(tol=1e-4, precision=hprlp.HPR_FP32, max_iter=200000))
    for lp, (info, x, y, z) in zip(lps, out):
        assert info.term == "solved"
        ev = oracle.kkt(lp, x, y, z)
        assert ev["rel_kkt"] <= 1e-4 * (1 + 1e-6)
        assert abs(ev["rel_kkt"] - info.rel_kkt) <= 1e-6 + 1e-3 * info.rel_kkt


def test_batch_bounds_and_starts_per_lp():
    datas = [scuc.make_instance("small", s) for s in (2, 3)]
    lps = [lp for _, lp in datas]
    b = hprlp.hpr_batch_create(lps, hprlp.Options(tol=0.0, max_iter=130, warm_fallback=0))
    data, lp = datas[1]
    G = data.cfg.n_gen
    lo, hi = lp.col_lo.copy(), lp.col_hi.copy()
    cols = scuc.col_index(G, np.arange(6), scuc.U, 1)
    lo[cols] = hi[cols] = 1.0
    hprlp.hpr_batch_set_bounds(b, 1, lo, hi)
    rng = np.random.default_rng(0)
    x0 = rng.uniform(0, 1, lps[0].n)
    hprlp.hpr_batch_set_start(b, 0, x0, None)
    infos = hprlp.hpr_batch_solve(b)
    o0 = oracle.solve(lps[0], oracle.Options(tol=0.0, max_iter=130), x0=x0)
    assert_parity(o0, infos[0], *hprlp.hpr_batch_get_solution(b, 0), FP64_RTOL)
    o1 = oracle.solve(lp.replace(col_lo=lo, col_hi=hi), oracle.Options(tol=0.0, max_iter=130))
    assert_parity(o1, infos[1], *hprlp.hpr_batch_get_solution(b, 1), FP64_RTOL)
    hprlp.hpr_batch_destroy(b)


def _reduced(count=12, classes=3):
    from paper_2510_10891_amd import fixing
    return [p.lp for p in fixing.make_reduced_batch(count=count, seed0=100, classes=classes)]


def test_reduced_batch_iterates_match_oracle_per_lp():
    """Reduced LPs of successive-fixing rounds (uneven sizes), 65 iterations."""
    lps = _reduced()
    out = hprlp.batch_solve(lps, hprlp.Options(tol=0.0, max_iter=65))
    for lp, (info, x, y, z) in zip(lps, out):
        o = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=65))
        assert_parity(o, info, x, y, z, FP64_RTOL)


@pytest.mark.parametrize("precision", [hprlp.HPR_FP64, hprlp.HPR_FP32])
def test_reduced_batch_reaches_tolerance(precision):
    lps = _reduced(count=16, classes=4)
    out = hprlp.batch_solve(lps, hprlp.Options(tol=1e-4, precision=precision, max_iter=100000))
    for lp, (info, x, y, z) in zip(lps, out):
        assert info.term == "solved", (lp.meta["parent"], info)
        ev = oracle.kkt(lp, x, y, z)
        assert ev["rel_kkt"] <= 1e-4 * (1 + 1e-6)


def test_warm_start_fallback_rejects_a_bad_start():
    """A broken start (1e6 on columns without an upper bound: the first check's rel_kkt is
    ~1e6 times the cold one) is rejected: the solve runs from zero, exactly as the cold
    solve; a start at the solution is kept."""
    lp = ragged_lp(1, bounded=False)
    cold, xc, yc, zc = hprlp.solve(lp, hprlp.Options(tol=1e-6, max_iter=200000, unroll=4))
    assert cold.term == "solved"
    bad = np.full(lp.n, 1e6)
    ib, xb, yb, zb = hprlp.solve(lp, hprlp.Options(tol=1e-6, max_iter=200000, unroll=4), x0=bad)
    assert ib.warm_start == 0 and ib.iters == cold.iters and np.array_equal(xb, xc)
    good, *_ = hprlp.solve(lp, hprlp.Options(tol=1e-6, max_iter=200000, unroll=4), x0=xc, y0=yc)
    assert good.warm_start == 1 and good.iters < cold.iters


def test_per_lp_time_to_stop_follows_the_checks():
    """hpr_info.solve_s of a batch member is the time to the check at which it stopped: within
    the call's wall time, equal for LPs that stop at the same check, and ordered like the
    iteration counts otherwise."""
    import time
    lps = [scuc.make_instance("small", s)[1] for s in range(6)]
    b = hprlp.hpr_batch_create(lps, hprlp.Options(tol=1e-4, max_iter=200000))
    try:
        t0 = time.perf_counter()
        infos = hprlp.hpr_batch_solve(b)
        wall = time.perf_counter() - t0
    finally:
        hprlp.hpr_batch_destroy(b)
    assert all(i.term == "solved" for i in infos)
    for i in infos:
        assert 0.0 < i.solve_s <= wall
    for a in infos:
        for c in infos:
            if a.iters == c.iters:
                assert a.solve_s == c.solve_s
            elif a.iters < c.iters:
                assert a.solve_s <= c.solve_s


def spread_lp(seed, m=64, n=12000, row_len=2000):
    """Rows of 2,000 entries spread over 12,000 columns: a block of 4 such rows (64 lanes each)
    uses three 4,096-column windows, none of which holds half of its entries, so only sliced
    windows serve it."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(m), row_len)
    cols = np.concatenate([np.sort(rng.choice(n, row_len, replace=False)) for _ in range(m)])
    A = sp.csr_matrix((rng.standard_normal(m * row_len) / np.sqrt(row_len), (rows, cols)), shape=(m, n))
    A.sort_indices()
    xf = rng.uniform(-0.5, 0.5, n)
    ax = A @ xf
    return scuc.LP(m, n, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.copy(),
                   ax - rng.uniform(0.1, 1, m), ax + rng.uniform(0.1, 1, m), -np.ones(n), np.ones(n),
                   rng.standard_normal(n), 0.0)


def test_batch_with_sliced_windows_matches_oracle_per_lp():
    """A batch whose members' rows span many windows (sliced LDS windows, lds_windows = 3) and
    narrow ones: each member's iterates against the oracle run on that LP alone."""
    lps = [spread_lp(s) for s in range(3)] + [ragged_lp(s, m=200, n=400) for s in range(2)]
    opts = hprlp.Options(tol=0.0, max_iter=130, lds_windows=3, unroll=2, profile=1)
    b = hprlp.hpr_batch_create(lps, opts)
    try:
        infos = hprlp.hpr_batch_solve(b)
        ks = hprlp.hpr_batch_get_kernel_stats(b)
        sols = [hprlp.hpr_batch_get_solution(b, i) for i in range(len(lps))]
    finally:
        hprlp.hpr_batch_destroy(b)
    assert ks["sliced_blocks_a"] + ks["sliced_blocks_at"] > 0, ks
    for lp, info, (x, y, z) in zip(lps, infos, sols):
        o = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=130))
        assert_parity(o, info, x, y, z, FP64_RTOL)


@pytest.mark.parametrize("use_graph", [0, 1])
def test_batch_with_blocks_in_rounds_matches_oracle_per_lp(use_graph):
    """A batch of LPs whose rows of ~64 entries spread over 1,900 columns (FP64 windows of at most
    2,048 entries): their blocks of A take the rows in rounds sharing one window copy, beside a
    narrow member without such blocks; each member's iterates against the oracle run on that LP
    alone, through captured iteration blocks and direct launches."""
    lps = [scuc.random_lp(np.random.default_rng(s), 384 + 64 * s, 1900, density=64.0 / 1900) for s in range(3)]
    lps.append(ragged_lp(3, m=200, n=400))
    K = 130
    opts = hprlp.Options(tol=0.0, max_iter=K, lds_windows=1, unroll=2, use_graph=use_graph, profile=1)
    b = hprlp.hpr_batch_create(lps, opts)
    try:
        infos = hprlp.hpr_batch_solve(b)
        ks = hprlp.hpr_batch_get_kernel_stats(b)
        sols = [hprlp.hpr_batch_get_solution(b, i) for i in range(len(lps))]
    finally:
        hprlp.hpr_batch_destroy(b)
    assert ks["round_blocks_a"] > 0, ks
    for lp, info, (x, y, z) in zip(lps, infos, sols):
        o = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=K))
        assert_parity(o, info, x, y, z, FP64_RTOL)


@pytest.mark.parametrize("mode", [3, 4, 5])
@pytest.mark.parametrize("precision", [hprlp.HPR_FP64, hprlp.HPR_FP32])
def test_sliced_windows_of_a_with_rows_out_of_column_order(mode, precision):
    """Rows of A spread over three windows, given out of column order (the library stores them
    in column order, which the sliced windows rely on), forced through sliced windows of A with
    64 (mode 3), 16 (mode 4) or 8 (mode 5) lanes per row: iterates against the oracle."""
    lp = spread_lp(7)
    rng = np.random.default_rng(8)
    idx, val = lp.col_idx.copy(), lp.val.copy()
    for i in range(lp.m):
        a, b = lp.row_ptr[i], lp.row_ptr[i + 1]
        perm = a + rng.permutation(b - a)
        idx[a:b], val[a:b] = idx[perm], val[perm]
    lp = lp.replace(col_idx=idx, val=val)
    K = 130
    o = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=K))
    h = hprlp.hpr_create(lp, hprlp.Options(tol=0.0, max_iter=K, lds_windows=mode, unroll=2, precision=precision))
    try:
        info = hprlp.hpr_solve(h)
        x, y, z = hprlp.hpr_get_solution(h)
        ks = hprlp.hpr_get_kernel_stats(h)
    finally:
        hprlp.hpr_destroy(h)
    assert ks["sliced_blocks_a"] > 0, ks
    if precision == hprlp.HPR_FP64:
        assert_parity(o, info, x, y, z, FP64_RTOL)
    else:
        assert info.iters == o.iters
        assert_close(x, o.x, FP32_RTOL * 10 * K, "x")
        assert_close(y, o.y, FP32_RTOL * 10 * K, "y")


def test_stored_fixings_batch_reaches_tolerance():
    """The first ten members of the mixed batch with the stored fixings (Algorithm 1 on solved
    relaxations), as one FP32 batch with the stall test and the FP64 continuation: every
    member ends solved, judged by the oracle's FP64 KKT evaluator."""
    import os
    from paper_2510_10891_amd import mixed
    recs = fixing.load_fixings(os.path.join(os.path.dirname(__file__), "golden", "fixing_masks_mixed.json"))
    lps = [p.lp for p in fixing.make_reduced_batch(count=10, seed0=100, fixings=recs[:10])]
    opts = hprlp.Options(tol=1e-4, precision=hprlp.HPR_FP32, max_iter=100000, stall_iters=8192)
    b = hprlp.hpr_batch_create(lps, opts)
    try:
        infos = hprlp.hpr_batch_solve(b)
        infos, cont = mixed.continue_stalled(lps, opts, infos, lambda i: hprlp.hpr_batch_get_solution(b, i))
        sols = [cont[i] if i in cont else hprlp.hpr_batch_get_solution(b, i) for i in range(len(lps))]
    finally:
        hprlp.hpr_batch_destroy(b)
    for lp, info, (x, y, z) in zip(lps, infos, sols):
        assert info.term == "solved", (lp.meta["parent"], info)
        assert oracle.kkt(lp, x, y, z)["rel_kkt"] <= 1e-4 * (1 + 1e-6)


def test_stored_fixings_infeasible_members_are_certified():
    """Members 40-60 (step 5) of the mixed batch, 30-bus parents: the batch certifies primal
    infeasibility exactly for the members HiGHS finds infeasible (45, 55, 60) and solves the
    others."""
    import os
    from tests.test_fixing import _highs_status
    recs = fixing.load_fixings(os.path.join(os.path.dirname(__file__), "golden", "fixing_masks_mixed.json"))
    idx = [40, 45, 50, 55, 60]
    lps = [fixing.reduced_lp(fixing.BATCH_PARENTS[0], 100 + i, 0.0, fixing=recs[i]).lp for i in idx]
    infos = [r[0] for r in hprlp.batch_solve(lps, hprlp.Options(tol=1e-4, precision=hprlp.HPR_FP32, max_iter=100000))]
    for i, lp, info in zip(idx, lps, infos):
        expect = "solved" if _highs_status(lp) == 0 else "primal_infeasible"
        assert info.term == expect, (i, info)
