"""GPU parity: the HIP solver against the CPU oracle, through the C interface.

Short runs (tol = 0, a fixed iteration count) must reproduce the oracle's iterates
element by element: same scaling, lambda, iteration, check schedule, restarts and
sigma. FP64 agrees to rounding (1e-8 relative); FP32 storage to FP32 rounding over a
few iterations. Full solves are judged by the oracle's FP64 KKT evaluator.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2510_10891_amd import fixing, hprlp, scuc
from tests.helpers import highs, rel

pytestmark = pytest.mark.gpu

FP64_RTOL = 1e-8
FP32_RTOL = 2e-5


def ragged_lp(seed, m=400, n=900, bounded=True):
    """Random feasible LP whose row and column lengths span every lane-group bin
    (empty rows and columns, 1-3 entries, tens, hundreds, > 256) and a ragged tail."""
    rng = np.random.default_rng(seed)
    empty_cols = set(rng.choice(n, 7, replace=False).tolist())
    usable = np.array([j for j in range(n) if j not in empty_cols])
    lens = rng.choice([0, 1, 2, 3, 5, 9, 17, 33, 70, 140, 300, 700], size=m,
                      p=[.04, .12, .12, .12, .1, .1, .1, .08, .08, .06, .05, .03])
    rows, cols, vals = [], [], []
    for i, L in enumerate(lens):
        cs = np.sort(rng.choice(usable, size=min(L, len(usable)), replace=False))
        rows += [i] * len(cs)
        cols += cs.tolist()
        vals += rng.standard_normal(len(cs)).tolist()
    import scipy.sparse as sp
    A = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    A.sort_indices()
    l = -rng.uniform(0.5, 2, n)
    u = rng.uniform(0.5, 2, n)
    if not bounded:
        u[rng.random(n) < 0.2] = np.inf
        l[rng.random(n) < 0.1] = -np.inf
    xf = np.clip(rng.uniform(-0.5, 0.5, n), l, u)
    ax = A @ xf
    kind = rng.random(m)
    lo = np.where(kind < 0.7, ax - rng.uniform(0, 1, m), -np.inf)
    hi = np.where(kind > 0.3, ax + rng.uniform(0, 1, m), np.inf)
    eq = kind < 0.1
    lo[eq] = hi[eq] = ax[eq]
    empty = np.diff(A.indptr) == 0
    lo[empty] = np.minimum(lo[empty], 0.0)
    hi[empty] = np.maximum(hi[empty], 0.0)
    c = rng.standard_normal(n)
    return scuc.LP(m, n, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.copy(),
                   lo, hi, l, u, c, 0.25)


def run_both(lp, K, precision=hprlp.HPR_FP64, unroll=0, **kw):
    o = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=K, **kw))
    opts = hprlp.Options(tol=0.0, max_iter=K, precision=precision, unroll=unroll,
                         **{("lambda_" if k == "lambda_in" else k): v for k, v in kw.items()
                            if k not in ("use_pc", "use_bc", "ruiz_iters")})
    if "use_pc" in kw or "use_bc" in kw or "ruiz_iters" in kw:
        mask = (hprlp.HPR_SCALE_PC if kw.get("use_pc", True) else 0) | \
               (hprlp.HPR_SCALE_BC if kw.get("use_bc", True) else 0) | \
               (hprlp.HPR_SCALE_RUIZ if kw.get("ruiz_iters", 0) else 0)
        opts.scaling = mask
        opts.ruiz_iters = kw.get("ruiz_iters", 10)
    info, x, y, z = hprlp.solve(lp, opts)
    return o, info, x, y, z


def assert_close(a, b, rtol, what):
    scale = 1.0 + np.abs(b).max(initial=0.0)
    err = np.abs(a - b).max(initial=0.0)
    assert err <= rtol * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e}"


def assert_parity(o, info, x, y, z, rtol):
    assert info.iters == o.iters
    assert info.restarts == o.restarts
    assert abs(info.lam - o.lam) <= 1e-12 * o.lam
    assert_close(x, o.x, rtol, "x")
    assert_close(y, o.y, rtol, "y")
    assert_close(z, o.z, rtol, "z")
    assert abs(info.pobj - o.pobj) <= rtol * (1 + abs(o.pobj))


def wide_lp(seed, m=300, n=70000):
    """Rows whose columns span more than 65536 (read through 32-bit indices) mixed with
    narrow rows (16-bit offsets from the row's smallest column)."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for i in range(m):
        L = int(rng.choice([2, 5, 20, 90, 400]))
        if i % 3 == 0:      # wide: both ends of the column range
            cs = np.unique(np.r_[rng.integers(0, 200, L // 2 + 1), rng.integers(n - 2000, n, L - L // 2)])
        else:               # narrow: a window of 30000 columns
            a = int(rng.integers(0, n - 30000))
            cs = np.unique(rng.integers(a, a + 30000, L))
        rows += [i] * len(cs)
        cols += cs.tolist()
        vals += rng.standard_normal(len(cs)).tolist()
    import scipy.sparse as sp
    A = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    A.sort_indices()
    l, u = -np.ones(n), np.ones(n)
    xf = rng.uniform(-0.5, 0.5, n)
    ax = A @ xf
    lo, hi = ax - rng.uniform(0.1, 1, m), ax + rng.uniform(0.1, 1, m)
    return scuc.LP(m, n, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.copy(), lo, hi, l, u,
                   rng.standard_normal(n), 0.0)


# ----------------------------------------------------------------------------- short-run parity

@pytest.mark.parametrize("precision", [hprlp.HPR_FP64, hprlp.HPR_FP32])
def test_wide_and_narrow_rows_match_oracle(precision):
    lp = wide_lp(0)
    K = 130 if precision == hprlp.HPR_FP64 else 2
    o, info, x, y, z = run_both(lp, K, precision=precision)
    if precision == hprlp.HPR_FP64:
        assert_parity(o, info, x, y, z, FP64_RTOL)
    else:
        assert info.iters == o.iters
        assert_close(x, o.x, FP32_RTOL * 20, "x")
        assert_close(y, o.y, FP32_RTOL * 20, "y")


@pytest.mark.parametrize("K", [1, 2, 64, 65, 66, 200, 513])
@pytest.mark.parametrize("seed", [0, 1])
def test_fp64_iterates_match_oracle_ragged(seed, K):
    lp = ragged_lp(seed, bounded=(seed == 0))
    o, info, x, y, z = run_both(lp, K)
    assert_parity(o, info, x, y, z, FP64_RTOL)


@pytest.mark.parametrize("unroll", [1, 2, 4, 8])
@pytest.mark.parametrize("precision", [hprlp.HPR_FP64, hprlp.HPR_FP32])
def test_every_schedule_matches_oracle(unroll, precision):
    """Each lane-group schedule (U quads per lane and pass, bins following U)."""
    lp = ragged_lp(4, bounded=False)
    K = 130 if precision == hprlp.HPR_FP64 else 2
    o, info, x, y, z = run_both(lp, K, precision=precision, unroll=unroll)
    if precision == hprlp.HPR_FP64:
        assert_parity(o, info, x, y, z, FP64_RTOL)
    else:
        assert info.iters == o.iters
        assert_close(x, o.x, FP32_RTOL * 20, "x")
        assert_close(y, o.y, FP32_RTOL * 20, "y")


@pytest.mark.parametrize("K", [1, 65, 1000])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fp64_iterates_match_oracle_small_scuc(seed, K):
    _, lp = scuc.make_instance("small", seed)
    o, info, x, y, z = run_both(lp, K)
    assert_parity(o, info, x, y, z, FP64_RTOL)


@pytest.mark.parametrize("variant", [dict(use_pc=False, use_bc=False), dict(ruiz_iters=10),
                                     dict(restart=False, sigma_update=False), dict(lambda_in=0.9),
                                     dict(sigma_smoothing=0.5), dict(sigma_smoothing=0.25)])
def test_fp64_options_match_oracle(variant):
    _, lp = scuc.make_instance("small", 3)
    o, info, x, y, z = run_both(lp, 300, **variant)
    assert_parity(o, info, x, y, z, FP64_RTOL)


@pytest.mark.parametrize("variant", [dict(), dict(sigma_smoothing_warm=1.0), dict(sigma_smoothing_warm=0.25)])
def test_warm_started_iterates_match_oracle(variant):
    """From a caller's start point (the warm sigma weight applies), iterations with restarts
    agree element by element with the oracle started from the same point."""
    _, lp = scuc.make_instance("small", 2)
    ref = oracle.solve(lp, oracle.Options(tol=1e-3, max_iter=100000))
    rng = np.random.default_rng(0)
    x0 = ref.x + 0.05 * rng.standard_normal(lp.n)
    y0 = ref.y * (1 + 0.2 * rng.standard_normal(lp.m))
    o = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=700, **variant), x0, y0)
    info, x, y, z = hprlp.solve(lp, hprlp.Options(tol=0.0, max_iter=700, warm_fallback=0, **variant), x0=x0, y0=y0)
    assert o.restarts > 0 and info.warm_start == 1
    assert_parity(o, info, x, y, z, FP64_RTOL)


@pytest.mark.parametrize("K", [1, 2, 65])
def test_fp32_iterates_track_oracle(K):
    lp = ragged_lp(2)
    o, info, x, y, z = run_both(lp, K, precision=hprlp.HPR_FP32)
    assert info.iters == o.iters
    assert_close(x, o.x, FP32_RTOL * 10 * K, "x")
    assert_close(y, o.y, FP32_RTOL * 10 * K, "y")


# ----------------------------------------------------------------------------- full solves

@pytest.mark.parametrize("precision", [hprlp.HPR_FP64, hprlp.HPR_FP32])
@pytest.mark.parametrize("seed", range(10))
def test_small_scuc_reaches_tolerance(seed, precision):
    _, lp = scuc.make_instance("small", seed)
    info, x, y, z = hprlp.solve(lp, hprlp.Options(tol=1e-4, precision=precision, max_iter=200000))
    assert info.term == "solved"
    ev = oracle.kkt(lp, x, y, z)
    assert ev["rel_kkt"] <= 1e-4 * (1 + 1e-6), ev
    assert abs(ev["rel_kkt"] - info.rel_kkt) <= 1e-6 + 1e-3 * info.rel_kkt
    ref, _, _ = highs(lp)
    assert rel(info.pobj, ref) < 2e-3
    if precision == hprlp.HPR_FP64:
        o = oracle.solve(lp, oracle.Options(tol=1e-4, max_iter=200000))
        assert o.iters == info.iters


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fp64_tight_tolerance_matches_oracle_objective(seed):
    _, lp = scuc.make_instance("small", seed)
    info, x, y, z = hprlp.solve(lp, hprlp.Options(tol=1e-8, max_iter=400000))
    o = oracle.solve(lp, oracle.Options(tol=1e-8, max_iter=400000))
    assert info.term == "solved" and o.term == "solved"
    assert rel(info.pobj, o.pobj) < 1e-6
    assert oracle.kkt(lp, x, y, z)["rel_kkt"] <= 1e-8 * 1.001


@pytest.mark.parametrize("seed", range(4))
def test_tiny_lps_match_brute_force(seed):
    lp = scuc.random_lp(np.random.default_rng(seed), 5, 4)
    obj, _ = oracle.brute_force(lp)
    info, x, y, z = hprlp.solve(lp, hprlp.Options(tol=1e-9, max_iter=200000))
    assert info.term == "solved"
    assert rel(info.pobj, obj) < 1e-6


def test_medium_full_size_parity_and_tolerance():
    """The 2,000-bus instance at full size: 65 iterations element by element against the
    oracle, then FP64 and FP32 solves to 1e-4 judged by the FP64 KKT evaluator."""
    _, lp = scuc.make_instance("medium", 0)
    o, info, x, y, z = run_both(lp, 65)
    assert_parity(o, info, x, y, z, FP64_RTOL)
    for precision in (hprlp.HPR_FP64, hprlp.HPR_FP32):
        info, x, y, z = hprlp.solve(lp, hprlp.Options(tol=1e-4, precision=precision, max_iter=100000))
        assert info.term == "solved", info
        ev = oracle.kkt(lp, x, y, z)
        assert ev["rel_kkt"] <= 1e-4 * (1 + 1e-6), ev


def _run_mode(lp, K, mode, precision):
    h = hprlp.hpr_create(lp, hprlp.Options(tol=0.0, max_iter=K, unroll=2, lds_windows=mode, lambda_=1.0,
                                           precision=precision, profile=1))
    try:
        info = hprlp.hpr_solve(h)
        x, y, z = hprlp.hpr_get_solution(h)
        ks = hprlp.hpr_get_kernel_stats(h)
    finally:
        hprlp.hpr_destroy(h)
    return info, x, y, z, ks


@pytest.mark.parametrize("formulation", ["compact", "full"])
def test_lds_window_modes_agree_bitwise(formulation):
    """The gather paths global memory, full LDS windows and split windows read the same values
    in the same order: for a fixed lane schedule the iterates agree bitwise across lds_windows =
    0, 1, 2, and with the oracle to rounding (FP64). Sliced windows (mode 3) add a straddling
    quad's entries in two passes, so they agree to rounding. 2,000-bus matrices, where every
    mode has blocks to act on (the schedule's block counts say which mode ran)."""
    _, lp = scuc.make_instance("medium", 0, formulation=formulation)
    if formulation == "full":
        lp = fixing.presolve_free_singletons(lp).lp
    precisions = (hprlp.HPR_FP64, hprlp.HPR_FP32) if formulation == "compact" else (hprlp.HPR_FP64,)
    K = 65
    o = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=K, lambda_in=1.0)) if formulation == "compact" else None
    for precision in precisions:
        runs = []
        for mode in (0, 1, 2):
            runs.append(_run_mode(lp, K, mode, precision))
        k0, k1, k2 = (r[4] for r in runs)
        assert k0["full_blocks_a"] == k0["split_blocks_a"] == k0["full_blocks_at"] == k0["split_blocks_at"] == 0
        assert k1["split_blocks_a"] == k1["split_blocks_at"] == 0 and k1["full_blocks_a"] > 0
        assert k2["split_blocks_a"] + k2["split_blocks_at"] > 0
        for info, x, y, z, _ in runs[1:]:
            assert info.iters == runs[0][0].iters
            assert np.array_equal(x, runs[0][1]) and np.array_equal(y, runs[0][2]) and np.array_equal(z, runs[0][3])
        if o is not None and precision == hprlp.HPR_FP64:
            info, x, y, z, _ = runs[2]
            assert_parity(o, info, x, y, z, FP64_RTOL)
        if formulation == "full":
            info, x, y, z, k3 = _run_mode(lp, K, 3, precision)
            assert k3["sliced_blocks_a"] > 0
            assert info.iters == runs[0][0].iters
            assert_close(x, runs[0][1], FP64_RTOL, "x")
            assert_close(y, runs[0][2], FP64_RTOL, "y")


@pytest.mark.parametrize("mode", [6, 7])
def test_lane_capped_window_modes_match_oracle(mode):
    """Every row of the 2,000-bus matrices given at most 16 (mode 6) or 8 (mode 7) lanes, so
    that full and split windows are shared by more rows: 65 FP64 iterations against the oracle."""
    _, lp = scuc.make_instance("medium", 0)
    K = 65
    o = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=K, lambda_in=1.0))
    info, x, y, z, ks = _run_mode(lp, K, mode, hprlp.HPR_FP64)
    assert ks["full_blocks_a"] > 0
    assert_parity(o, info, x, y, z, FP64_RTOL)


@pytest.mark.parametrize("precision,n", [(hprlp.HPR_FP64, 1900), (hprlp.HPR_FP32, 2600)])
def test_blocks_in_rounds_match_oracle(precision, n):
    """Rows of ~64 entries spread over n columns (8 or 16 lanes each with U = 2): the blocks of A
    get full windows wider than half the LDS window (8 KB) and take their rows in rounds, up to
    4 x 256/G rows per window copy. FP64: 65 iterations against the oracle. FP32: 2 against the
    oracle, and 65 against the same solve with the vector gathered from global memory
    (lds_windows = 0: no windows, one round per block)."""
    lp = scuc.random_lp(np.random.default_rng(7), 512, n, density=64.0 / n)
    K = 65
    info, x, y, z, ks = _run_mode(lp, K, 1, precision)
    assert ks["round_blocks_a"] > 0 and ks["win_mode_a"] == 1
    if precision == hprlp.HPR_FP64:
        o = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=K, lambda_in=1.0))
        assert_parity(o, info, x, y, z, FP64_RTOL)
        return
    o = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=2, lambda_in=1.0))
    i2, x2, y2, _, k2 = _run_mode(lp, 2, 1, precision)
    assert k2["round_blocks_a"] > 0 and i2.iters == o.iters
    assert_close(x2, o.x, FP32_RTOL * 20, "x")
    assert_close(y2, o.y, FP32_RTOL * 20, "y")
    i0, x0, y0, _, k0 = _run_mode(lp, K, 0, precision)
    assert k0["round_blocks_a"] == 0 and i0.iters == info.iters
    assert_close(x, x0, FP32_RTOL, "x")
    assert_close(y, y0, FP32_RTOL, "y")


def test_packed_quads_cover_both_index_paths():
    """Quads of narrow rows whose first offset fits 13 bits and gaps 6 bits can be read as one
    packed word, the others through their 16-bit offsets as well; a matrix reads the packed words
    only from 90% packed quads on. The 2,000-bus matrices pack ~98% (their parity and bitwise-mode tests above run on
    packed words with the 2% read through offsets); a ragged LP packs some quads, stays below the
    threshold and reads offsets only, and matches the oracle too."""
    _, lp = scuc.make_instance("medium", 0)
    h = hprlp.hpr_create(lp, hprlp.Options(max_iter=1))
    try:
        ks = hprlp.hpr_get_kernel_stats(h)
    finally:
        hprlp.hpr_destroy(h)
    for side in ("a", "at"):
        assert ks[f"packed_quads_{side}"] >= 0.95 * ks[f"narrow_quads_{side}"] > 0
        assert ks[f"packed_{side}"] == 1
    lp = ragged_lp(2)
    K = 65
    o = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=K, lambda_in=1.0))
    info, x, y, z, ks = _run_mode(lp, K, 0, hprlp.HPR_FP64)
    for side in ("a", "at"):
        assert 0 < ks[f"packed_quads_{side}"] < ks[f"narrow_quads_{side}"]
        assert ks[f"packed_{side}"] == int(ks[f"packed_quads_{side}"] >= 0.9 * ks[f"narrow_quads_{side}"])
    assert_parity(o, info, x, y, z, FP64_RTOL)


@pytest.mark.parametrize("mode", [0, 1, 3])
def test_rows_given_out_of_column_order(mode):
    """CSR rows whose entries are not in column order (allowed by the interface) are stored in
    column order by the library, which the sliced windows rely on: the same iterates as the
    oracle on the shuffled input, for every gather path."""
    lp = wide_lp(1)
    rng = np.random.default_rng(5)
    idx, val = lp.col_idx.copy(), lp.val.copy()
    for i in range(lp.m):
        a, b = lp.row_ptr[i], lp.row_ptr[i + 1]
        perm = a + rng.permutation(b - a)
        idx[a:b], val[a:b] = idx[perm], val[perm]
    shuffled = lp.replace(col_idx=idx, val=val)
    o = oracle.solve(shuffled, oracle.Options(tol=0.0, max_iter=130))
    info, x, y, z = hprlp.solve(shuffled, hprlp.Options(tol=0.0, max_iter=130, lds_windows=mode, unroll=2))
    assert_parity(o, info, x, y, z, FP64_RTOL)


def test_medium_objective_matches_interior_point_golden():
    """The 2,000-bus instance solved to 1e-6 in FP64 reaches the optimal objective that an
    independent interior-point solver (HiGHS, stored under tests/golden/) found for it."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "highs_medium_seed0.json")) as f:
        gold = json.load(f)
    _, lp = scuc.make_instance(gold["preset"], gold["seed"])
    assert (lp.m, lp.n, lp.nnz) == (gold["m"], gold["n"], gold["nnz"])
    info, x, y, z = hprlp.solve(lp, hprlp.Options(tol=1e-6, max_iter=400000))
    assert info.term == "solved", info
    ev = oracle.kkt(lp, x, y, z)
    assert ev["rel_kkt"] <= 1e-6 * (1 + 1e-6), ev
    assert rel(ev["pobj"], gold["objective"]) < 2e-5, (ev["pobj"], gold["objective"])


# ----------------------------------------------------------------------------- handle semantics

def test_fixing_bounds_then_resolve_matches_oracle():
    data, lp = scuc.make_instance("small", 4)
    G, T = data.cfg.n_gen, data.cfg.T
    lo, hi = lp.col_lo.copy(), lp.col_hi.copy()
    for g in range(0, G, 3):            # fix u of every third unit on for the first 8 hours
        cols = scuc.col_index(G, np.arange(8), scuc.U, g)
        lo[cols] = hi[cols] = 1.0
    fixed = lp.replace(col_lo=lo, col_hi=hi)
    h = hprlp.hpr_create(lp, hprlp.Options(tol=0.0, max_iter=300))
    hprlp.hpr_solve(h)
    hprlp.hpr_set_bounds(h, lo, hi)
    info = hprlp.hpr_solve(h)
    x, y, z = hprlp.hpr_get_solution(h)
    o = oracle.solve(fixed, oracle.Options(tol=0.0, max_iter=300))
    assert_parity(o, info, x, y, z, FP64_RTOL)


def test_warm_start_from_solution_converges_at_once():
    _, lp = scuc.make_instance("small", 1)
    info, x, y, z = hprlp.solve(lp, hprlp.Options(tol=1e-7, max_iter=200000))
    assert info.term == "solved"
    info2, *_ = hprlp.solve(lp, hprlp.Options(tol=1e-6, max_iter=200000), x0=x, y0=y)
    assert info2.term == "solved" and info2.iters < info.iters / 4
    o = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=130), x0=x, y0=y)
    i3, x3, y3, z3 = hprlp.solve(lp, hprlp.Options(tol=0.0, max_iter=130, warm_fallback=0), x0=x, y0=y)
    assert i3.warm_start == 1
    assert_parity(o, i3, x3, y3, z3, FP64_RTOL)


def test_repeat_solves_are_bitwise_identical():
    _, lp = scuc.make_instance("small", 2)
    h = hprlp.hpr_create(lp, hprlp.Options(tol=1e-6))
    a = hprlp.hpr_solve(h)
    xa, ya, za = hprlp.hpr_get_solution(h)
    b = hprlp.hpr_solve(h)
    xb, yb, zb = hprlp.hpr_get_solution(h)
    assert a.iters == b.iters and a.pobj == b.pobj
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb) and np.array_equal(za, zb)


def test_get_solution_before_solve_is_a_state_error():
    _, lp = scuc.make_instance("small", 0)
    h = hprlp.hpr_create(lp)
    with pytest.raises(hprlp.HprError) as e:
        hprlp.hpr_get_solution(h)
    assert e.value.code == hprlp.HPR_ERR_STATE


# ----------------------------------------------------------------------------- edge cases

def test_box_only_lp_without_rows():
    rng = np.random.default_rng(0)
    n = 37
    c = rng.standard_normal(n)
    l, u = -rng.uniform(0.5, 2, n), rng.uniform(0.5, 2, n)
    lp = scuc.LP(0, n, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0), np.zeros(0),
                 np.zeros(0), l, u, c, 1.5)
    info, x, y, z = hprlp.solve(lp, hprlp.Options(tol=1e-10, max_iter=1000))
    assert info.term == "solved"
    assert np.allclose(x, np.where(c > 0, l, u), atol=1e-10)
    o = oracle.solve(lp, oracle.Options(tol=1e-10, max_iter=1000))
    assert o.iters == info.iters


def _infeasible_lps():
    """(name, LP) of LPs without a feasible point (an independent solver agrees in the CPU
    tests of the oracle's certificate)."""
    out = [("box_too_small", scuc.LP(1, 2, np.array([0, 2], np.int64), np.array([0, 1], np.int32),
                                     np.array([1.0, 1.0]), np.array([3.0]), np.array([np.inf]), np.zeros(2),
                                     np.ones(2), np.ones(2)))]
    for seed in range(3):
        rng = np.random.default_rng(seed)
        base = scuc.random_lp(rng, 6, 5)
        a = rng.standard_normal(5)
        reach = np.where(a > 0, a * base.col_hi, a * base.col_lo).sum()
        import scipy.sparse as sp
        A = sp.vstack([base.to_scipy(), sp.csr_matrix(a[None, :])]).tocsr()
        A.sort_indices()
        out.append((f"random_{seed}", scuc.LP(base.m + 1, base.n, A.indptr.astype(np.int64),
                                              A.indices.astype(np.int32), A.data.copy(),
                                              np.r_[base.row_lo, reach + 1.0], np.r_[base.row_hi, np.inf],
                                              base.col_lo, base.col_hi, base.c)))
    data, lp = scuc.make_instance("small", 3)
    G, T = data.cfg.n_gen, data.cfg.T
    r1 = oracle.solve(lp, oracle.Options(tol=1e-6, max_iter=200000))
    u, v, w = fixing.gather_binaries(r1.x, G, T)
    fixed, ur, vr, wr = fixing.fixing_strategy(u, v, w, 0.1)
    lo, hi = fixing.fix_bounds(lp, G, T, fixed, ur, vr, wr)
    out.append(("scuc30_fixed", lp.replace(col_lo=lo, col_hi=hi)))
    return out


@pytest.mark.parametrize("case", range(5))
def test_infeasible_lps_are_certified_at_the_oracles_check(case):
    """The primal infeasibility certificate fires at the same check as in the oracle (FP64),
    and with FP32 storage after the FP64 confirmation."""
    name, lp = _infeasible_lps()[case]
    o = oracle.solve(lp, oracle.Options(tol=1e-6, max_iter=200000))
    assert o.term == "primal_infeasible", name
    info, x, y, z = hprlp.solve(lp, hprlp.Options(tol=1e-6, max_iter=200000))
    assert info.term == "primal_infeasible" and info.iters == o.iters, (name, info.iters, o.iters)
    info32, *_ = hprlp.solve(lp, hprlp.Options(tol=1e-6, max_iter=200000, precision=hprlp.HPR_FP32))
    assert info32.term == "primal_infeasible", name


def test_single_iteration_and_short_final_block():
    lp = ragged_lp(3)
    for K in (1, 3, 64, 127, 129):
        o, info, x, y, z = run_both(lp, K)
        assert info.term == "iter_limit" and info.iters == K
        assert_parity(o, info, x, y, z, FP64_RTOL)


def _unbounded_lps():
    from tests.test_oracle_unbounded import BOUNDED, UNBOUNDED
    return sorted(UNBOUNDED.items()), sorted(BOUNDED.items())


@pytest.mark.parametrize("case", range(10))
def test_unbounded_lps_are_certified_at_the_oracles_check(case):
    """The dual infeasibility test (a ray from the step's primal move) fires at the same check
    as in the oracle (FP64), and with FP32 storage after the FP64 confirmation."""
    name, lp = _unbounded_lps()[0][case]
    o = oracle.solve(lp, oracle.Options(tol=1e-8, max_iter=200000))
    assert o.term == "dual_infeasible", name
    info, x, y, z = hprlp.solve(lp, hprlp.Options(tol=1e-8, max_iter=200000))
    assert info.term == "dual_infeasible" and info.iters == o.iters, (name, info.iters, o.iters)
    # FP32 storage: the same test at a 1e-3 margin (the ray is a difference of FP32 iterates)
    info32, *_ = hprlp.solve(lp, hprlp.Options(tol=1e-8, max_iter=200000, precision=hprlp.HPR_FP32))
    assert info32.term == "dual_infeasible", name


@pytest.mark.parametrize("case", range(7))
def test_bounded_lps_with_unbounded_columns_match_the_oracle(case):
    """LPs with unbounded columns but a finite optimum are solved, never reported without one,
    in FP64 at the oracle's iteration and in FP32 storage at the wider ray margin."""
    name, lp = _unbounded_lps()[1][case]
    o = oracle.solve(lp, oracle.Options(tol=1e-9, max_iter=400000))
    info, x, y, z = hprlp.solve(lp, hprlp.Options(tol=1e-9, max_iter=400000))
    assert o.term == "solved" and info.term == "solved" and info.iters == o.iters, (name, info.iters, o.iters)
    assert abs(info.pobj - o.pobj) <= 1e-8 * (1 + abs(o.pobj))
    info32, x32, y32, z32 = hprlp.solve(lp, hprlp.Options(tol=1e-5, max_iter=400000, precision=hprlp.HPR_FP32))
    assert info32.term == "solved", (name, info32.term)
    assert abs(info32.pobj - o.pobj) <= 1e-3 * (1 + abs(o.pobj))


def test_torch_sees_the_gpu_after_the_library_solved_first():
    """In a fresh process: a solve through the library, and only then torch's first use of the
    GPU (the binding imports torch before loading the library, so both use one HIP runtime)."""
    pytest.importorskip("torch")
    code = ("from paper_2510_10891_amd import hprlp, scuc\n"
            "_, lp = scuc.make_instance('small', 0)\n"
            "info, *_ = hprlp.solve(lp, hprlp.Options(tol=1e-4, max_iter=20000))\n"
            "assert info.term == 'solved', info.term\n"
            "import torch\n"
            "assert torch.cuda.is_available()\n"
            "assert float((torch.ones(4, device='cuda:0') * 2).sum().item()) == 8.0\n"
            "print('ok')\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:] + r.stderr[-2000:]


def test_create_from_device_arrays_matches_host_arrays():
    """hpr_lp.on_device = 1 with torch-allocated arrays: the same scaling, schedule and solve as
    from host arrays (iterates bit for bit); wrong dtypes are refused by the binding."""
    torch = pytest.importorskip("torch")
    _, lp = scuc.make_instance("small", 2)
    dev = torch.device("cuda:0")

    def t(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a, dt)).to(dev)

    arrays = (t(lp.row_ptr, np.int64), t(lp.col_idx, np.int32), t(lp.val, np.float64), t(lp.row_lo, np.float64),
              t(lp.row_hi, np.float64), t(lp.col_lo, np.float64), t(lp.col_hi, np.float64), t(lp.c, np.float64))
    dlp = hprlp.DeviceLP(lp.m, lp.n, *arrays, lp.obj_offset)
    torch.cuda.synchronize()
    opts = hprlp.Options(tol=1e-6, max_iter=100000, unroll=2, lds_windows=2,
                         stream=torch.cuda.current_stream().cuda_stream)
    h = hprlp.hpr_create_device(dlp, opts)
    try:
        info = hprlp.hpr_solve(h)
        x, y, z = hprlp.hpr_get_solution(h)
    finally:
        hprlp.hpr_destroy(h)
    info2, x2, y2, z2 = hprlp.solve(lp, opts)
    assert info.term == "solved" and info.iters == info2.iters
    assert np.array_equal(x, x2) and np.array_equal(y, y2) and np.array_equal(z, z2)
    with pytest.raises(ValueError):
        hprlp.DeviceLP(lp.m, lp.n, arrays[0].to(torch.int32), *arrays[1:], lp.obj_offset)


def test_tuner_choice_is_reused_for_a_matrix_of_the_same_signature():
    """The schedule tuner's pick (U, window mode, load kind) is kept per coarse matrix signature:
    a second handle of the same LP takes it without timing anything, and solves bit for bit as
    the first."""
    lp = ragged_lp(123, m=700, n=1500)
    runs = []
    for _ in range(2):
        h = hprlp.hpr_create(lp, hprlp.Options(tol=0.0, max_iter=65))
        try:
            info = hprlp.hpr_solve(h)
            x, y, z = hprlp.hpr_get_solution(h)
            runs.append((info, x, y, hprlp.hpr_get_kernel_stats(h)))
        finally:
            hprlp.hpr_destroy(h)
    (i1, x1, y1, k1), (i2, x2, y2, k2) = runs
    assert k2["setup_phases_s"]["tune"] < k1["setup_phases_s"]["tune"]
    for key in ("unroll_a", "unroll_at", "nt_a", "nt_at", "full_blocks_a", "split_blocks_a", "sliced_blocks_a",
                "full_blocks_at", "split_blocks_at", "sliced_blocks_at"):
        assert k1[key] == k2[key], key
    assert np.array_equal(x1, x2) and np.array_equal(y1, y2)
