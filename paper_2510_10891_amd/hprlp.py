"""Python binding of libhprlp.so (the C interface in include/hprlp.h).

Argument marshalling only: every step of the solve runs in the library's HIP kernels.
Loading fails with an error when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, fields

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhprlp.so")

HPR_OK, HPR_ERR_INVALID, HPR_ERR_NOMEM, HPR_ERR_HIP, HPR_ERR_STATE = 0, -1, -2, -3, -4
HPR_SOLVED, HPR_ITER_LIMIT, HPR_TIME_LIMIT, HPR_NUMERIC_FAIL, HPR_PRIMAL_INFEASIBLE = 1, 2, 3, 4, 5
HPR_DUAL_INFEASIBLE, HPR_STALLED = 6, 7
HPR_FP64, HPR_FP32 = 0, 1
HPR_SCALE_PC, HPR_SCALE_RUIZ, HPR_SCALE_BC = 1, 2, 4
TERM_NAMES = {HPR_SOLVED: "solved", HPR_ITER_LIMIT: "iter_limit", HPR_TIME_LIMIT: "time_limit",
              HPR_NUMERIC_FAIL: "numeric_fail", HPR_PRIMAL_INFEASIBLE: "primal_infeasible",
              HPR_DUAL_INFEASIBLE: "dual_infeasible", HPR_STALLED: "stalled"}


class HprError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class hpr_lp(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("row_lo", C.c_void_p), ("row_hi", C.c_void_p), ("col_lo", C.c_void_p),
                ("col_hi", C.c_void_p), ("c", C.c_void_p), ("obj_offset", C.c_double),
                ("on_device", C.c_int32)]


class hpr_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int64), ("time_limit_s", C.c_double),
                ("precision", C.c_int32), ("scaling", C.c_int32), ("ruiz_iters", C.c_int32),
                ("check_every", C.c_int32), ("sigma0", C.c_double), ("lambda_", C.c_double),
                ("seed", C.c_uint64), ("restart", C.c_int32), ("sigma_update", C.c_int32),
                ("sigma_smoothing", C.c_double), ("sigma_smoothing_warm", C.c_double), ("power_max_iter", C.c_int32), ("power_tol", C.c_double), ("profile", C.c_int32),
                ("unroll", C.c_int32), ("lds_windows", C.c_int32), ("use_graph", C.c_int32),
                ("warm_fallback", C.c_int32), ("warm_fallback_ratio", C.c_double), ("stall_iters", C.c_int64),
                ("stream", C.c_void_p)]


class hpr_kernel_stats(C.Structure):
    _fields_ = [("primal_ms", C.c_double), ("dual_ms", C.c_double), ("samples", C.c_int64),
                ("unroll_a", C.c_int32), ("unroll_at", C.c_int32), ("nontemporal_a", C.c_int32),
                ("nontemporal_at", C.c_int32), ("full_blocks_a", C.c_int32), ("split_blocks_a", C.c_int32),
                ("full_blocks_at", C.c_int32), ("split_blocks_at", C.c_int32), ("blocks_a", C.c_int32),
                ("blocks_at", C.c_int32), ("sliced_blocks_a", C.c_int32), ("sliced_blocks_at", C.c_int32),
                ("setup_prep_s", C.c_double), ("setup_upload_s", C.c_double), ("setup_tune_s", C.c_double),
                ("setup_power_s", C.c_double), ("narrow_quads_a", C.c_int64), ("packed_quads_a", C.c_int64),
                ("narrow_quads_at", C.c_int64), ("packed_quads_at", C.c_int64), ("packed_a", C.c_int32),
                ("packed_at", C.c_int32), ("win_mode_a", C.c_int32), ("win_mode_at", C.c_int32),
                ("round_blocks_a", C.c_int32), ("round_blocks_at", C.c_int32)]


class hpr_info(C.Structure):
    _fields_ = [("term", C.c_int32), ("iters", C.c_int64), ("restarts", C.c_int64),
                ("pobj", C.c_double), ("dobj", C.c_double), ("rel_p", C.c_double),
                ("rel_d", C.c_double), ("rel_gap", C.c_double), ("rel_kkt", C.c_double),
                ("lambda_", C.c_double), ("sigma", C.c_double), ("setup_s", C.c_double),
                ("solve_s", C.c_double), ("warm_start", C.c_int32)]


_lib = None
EXPORTS = ("hpr_default_opts", "hpr_create", "hpr_set_bounds", "hpr_set_start", "hpr_solve",
           "hpr_get_solution", "hpr_get_kernel_stats", "hpr_fix_binaries", "hpr_destroy", "hpr_batch_create", "hpr_batch_size",
           "hpr_batch_set_bounds", "hpr_batch_set_start", "hpr_batch_solve", "hpr_batch_get_solution",
           "hpr_batch_get_kernel_stats", "hpr_batch_destroy", "hpr_probe_stream", "hpr_last_error")


def lib():
    """Load libhprlp.so (raises if it was not built).

    torch, when installed, is imported first. Its wheel ships HIP runtime libraries of its own;
    with torch imported first, the library and torch both ran on the GPU in one process, while
    loading the library first left torch without a GPU in that process (a test in a fresh process
    covers the order)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with python -m paper_2510_10891_amd.build")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(_LIB_PATH)
        L.hpr_last_error.restype = C.c_char_p
        for name in EXPORTS[1:-1]:
            getattr(L, name).restype = C.c_int
        L.hpr_default_opts.restype = None
        _lib = L
    return _lib


def hpr_last_error() -> str:
    return lib().hpr_last_error().decode()


def _check(rc):
    if rc != HPR_OK:
        raise HprError(rc, hpr_last_error())


@dataclass
class Options:
    """Python mirror of hpr_opts (defaults equal hpr_default_opts)."""
    tol: float = 1e-4
    max_iter: int = 1_000_000
    time_limit_s: float = 0.0
    precision: int = HPR_FP64
    scaling: int = HPR_SCALE_PC | HPR_SCALE_BC
    ruiz_iters: int = 10
    check_every: int = 64
    sigma0: float = 1.0
    lambda_: float = 0.0
    seed: int = 0
    restart: int = 1
    sigma_update: int = 1
    sigma_smoothing: float = 1.0
    sigma_smoothing_warm: float = 0.5
    power_max_iter: int = 200
    power_tol: float = 1e-6
    profile: int = 0
    unroll: int = 0
    lds_windows: int = -1
    use_graph: int = 1
    warm_fallback: int = 2
    warm_fallback_ratio: float = 1000.0
    stall_iters: int = 0
    stream: int = 0

    def to_c(self) -> hpr_opts:
        o = hpr_opts()
        for f in fields(self):
            setattr(o, f.name, getattr(self, f.name))
        o.stream = self.stream or None
        return o


def _kstats(s: hpr_kernel_stats) -> dict:
    return dict(primal_ms=s.primal_ms, dual_ms=s.dual_ms, samples=s.samples, unroll_a=s.unroll_a,
                unroll_at=s.unroll_at, nt_a=s.nontemporal_a, nt_at=s.nontemporal_at,
                full_blocks_a=s.full_blocks_a, split_blocks_a=s.split_blocks_a, full_blocks_at=s.full_blocks_at,
                split_blocks_at=s.split_blocks_at, blocks_a=s.blocks_a, blocks_at=s.blocks_at,
                sliced_blocks_a=s.sliced_blocks_a, sliced_blocks_at=s.sliced_blocks_at,
                setup_phases_s=dict(prep=round(s.setup_prep_s, 4), upload=round(s.setup_upload_s, 4),
                                    tune=round(s.setup_tune_s, 4), power=round(s.setup_power_s, 4)),
                narrow_quads_a=s.narrow_quads_a, packed_quads_a=s.packed_quads_a,
                narrow_quads_at=s.narrow_quads_at, packed_quads_at=s.packed_quads_at,
                packed_a=s.packed_a, packed_at=s.packed_at, win_mode_a=s.win_mode_a, win_mode_at=s.win_mode_at,
                round_blocks_a=s.round_blocks_a, round_blocks_at=s.round_blocks_at)


def hpr_default_opts() -> hpr_opts:
    o = hpr_opts()
    lib().hpr_default_opts(C.byref(o))
    return o


@dataclass
class Info:
    term: str
    iters: int
    restarts: int
    pobj: float
    dobj: float
    rel_p: float
    rel_d: float
    rel_gap: float
    rel_kkt: float
    lam: float
    sigma: float
    setup_s: float
    solve_s: float
    warm_start: int = 0


class _LPArrays:
    """Contiguous copies kept alive for the duration of a call."""

    def __init__(self, lp):
        f64 = lambda a: np.ascontiguousarray(a, np.float64)
        self.rp = np.ascontiguousarray(lp.row_ptr, np.int64)
        self.ci = np.ascontiguousarray(lp.col_idx, np.int32)
        self.v = f64(lp.val)
        self.lo, self.hi = f64(lp.row_lo), f64(lp.row_hi)
        self.l, self.u, self.c = f64(lp.col_lo), f64(lp.col_hi), f64(lp.c)
        m, n = int(lp.m), int(lp.n)
        if len(self.v) != len(self.ci):
            raise ValueError("col_idx and val differ in length")
        if m > 0 and len(self.rp) != m + 1:
            raise ValueError(f"row_ptr has {len(self.rp)} entries, expected m + 1 = {m + 1}")
        if len(self.lo) != m or len(self.hi) != m:
            raise ValueError(f"row_lo / row_hi have {len(self.lo)} / {len(self.hi)} entries, expected m = {m}")
        if not (len(self.l) == len(self.u) == len(self.c) == n):
            raise ValueError(f"col_lo / col_hi / c have {len(self.l)} / {len(self.u)} / {len(self.c)} entries, "
                             f"expected n = {n}")
        nnz = len(self.ci)   # the library checks row_ptr[m] == nnz
        ptr = lambda a: a.ctypes.data if a.size else None
        self.s = hpr_lp(lp.m, lp.n, nnz, ptr(self.rp), ptr(self.ci), ptr(self.v), ptr(self.lo),
                        ptr(self.hi), ptr(self.l), ptr(self.u), ptr(self.c), float(lp.obj_offset), 0)


class DeviceLP:
    """An LP whose arrays are torch tensors on the GPU (hpr_lp.on_device = 1): int64 row_ptr,
    int32 col_idx, float64 val and bounds and cost, as in hprlp.h. The tensors are kept alive
    with the struct; the library copies what it needs during hpr_create."""

    def __init__(self, m, n, row_ptr, col_idx, val, row_lo, row_hi, col_lo, col_hi, c, obj_offset=0.0):
        import torch
        want = [(row_ptr, torch.int64, m + 1, "row_ptr"), (col_idx, torch.int32, None, "col_idx"),
                (val, torch.float64, None, "val"), (row_lo, torch.float64, m, "row_lo"),
                (row_hi, torch.float64, m, "row_hi"), (col_lo, torch.float64, n, "col_lo"),
                (col_hi, torch.float64, n, "col_hi"), (c, torch.float64, n, "c")]
        for t, dt, length, name in want:
            if not (t.is_cuda and t.dtype == dt and t.is_contiguous() and t.dim() == 1):
                raise ValueError(f"{name} must be a contiguous 1-D {dt} CUDA tensor")
            if length is not None and t.numel() != length and not (name == "row_ptr" and m == 0):
                raise ValueError(f"{name} has {t.numel()} entries, expected {length}")
        if col_idx.numel() != val.numel():
            raise ValueError("col_idx and val differ in length")
        self.m, self.n = int(m), int(n)
        self.keep = [row_ptr, col_idx, val, row_lo, row_hi, col_lo, col_hi, c]
        ptr = lambda t: t.data_ptr() if t.numel() else None
        self.s = hpr_lp(self.m, self.n, int(col_idx.numel()), ptr(row_ptr), ptr(col_idx), ptr(val), ptr(row_lo),
                        ptr(row_hi), ptr(col_lo), ptr(col_hi), ptr(c), float(obj_offset), 1)


def hpr_create_device(dlp: DeviceLP, opts: Options | None = None) -> "Handle":
    """hpr_create from device arrays (DeviceLP)."""
    o = (opts or Options()).to_c()
    out = C.c_void_p()
    _check(lib().hpr_create(C.byref(dlp.s), C.byref(o), C.byref(out)))
    return Handle(out, dlp.m, dlp.n)


class Handle:
    """Owns an hpr_handle*; freed by hpr_destroy (or when garbage collected)."""

    def __init__(self, ptr, m, n):
        self.ptr, self.m, self.n = ptr, m, n

    def __del__(self):
        if getattr(self, "ptr", None):
            try:
                lib().hpr_destroy(self.ptr)
            except Exception:
                pass
            self.ptr = None


def hpr_create(lp, opts: Options | None = None) -> Handle:
    a = _LPArrays(lp)
    o = (opts or Options()).to_c()
    out = C.c_void_p()
    _check(lib().hpr_create(C.byref(a.s), C.byref(o), C.byref(out)))
    return Handle(out, lp.m, lp.n)


def hpr_destroy(h: Handle) -> None:
    if h.ptr:
        _check(lib().hpr_destroy(h.ptr))
        h.ptr = None


def _vec(a, length: int, name: str):
    """Contiguous FP64 copy of an optional vector whose length the library takes from m or n."""
    if a is None:
        return None
    a = np.ascontiguousarray(a, np.float64)
    if a.ndim != 1 or len(a) != length:
        raise ValueError(f"{name} has shape {a.shape}, expected ({length},)")
    return a


def hpr_set_bounds(h: Handle, col_lo=None, col_hi=None) -> None:
    lo, hi = _vec(col_lo, h.n, "col_lo"), _vec(col_hi, h.n, "col_hi")
    _check(lib().hpr_set_bounds(h.ptr, None if lo is None else lo.ctypes.data_as(C.c_void_p),
                                None if hi is None else hi.ctypes.data_as(C.c_void_p)))


def hpr_set_start(h: Handle, x0=None, y0=None) -> None:
    xa, ya = _vec(x0, h.n, "x0"), _vec(y0, h.m, "y0")
    _check(lib().hpr_set_start(h.ptr, None if xa is None else xa.ctypes.data_as(C.c_void_p),
                               None if ya is None else ya.ctypes.data_as(C.c_void_p)))


def hpr_solve(h: Handle) -> Info:
    info = hpr_info()
    _check(lib().hpr_solve(h.ptr, C.byref(info)))
    return _info(info)


def hpr_get_solution(h: Handle):
    x = np.zeros(h.n)
    y = np.zeros(max(h.m, 1))
    z = np.zeros(h.n)
    _check(lib().hpr_get_solution(h.ptr, x.ctypes.data_as(C.c_void_p), y.ctypes.data_as(C.c_void_p),
                                  z.ctypes.data_as(C.c_void_p)))
    return x, y[:h.m], z


def hpr_fix_binaries(h: Handle, cols, tau: float, x=None, fixval=None):
    """Round and Algorithm 1 on the device (hpr_fix_binaries): cols [G][T][3] LP columns of
    (u, v, w), negative where presolve removed the column (its value then from fixval, same
    shape); x: original-space point, or None for the last solve's bar point on the device.
    Returns (fixed [G][T] bool, rounded [G][T][3] int8)."""
    cols = np.ascontiguousarray(cols, np.int32)
    if cols.ndim != 3 or cols.shape[2] != 3:
        raise ValueError(f"cols has shape {cols.shape}, expected (G, T, 3)")
    G, T = cols.shape[:2]
    fv = None
    if fixval is not None:
        fv = np.ascontiguousarray(fixval, np.float64)
        if fv.shape != cols.shape:
            raise ValueError(f"fixval has shape {fv.shape}, expected {cols.shape}")
    xa = _vec(x, h.n, "x")
    fixed = np.zeros((G, T), np.int8)
    rounded = np.zeros((G, T, 3), np.int8)
    _check(lib().hpr_fix_binaries(h.ptr, None if xa is None else xa.ctypes.data_as(C.c_void_p), C.c_int32(G),
                                  C.c_int32(T), cols.ctypes.data_as(C.c_void_p),
                                  None if fv is None else fv.ctypes.data_as(C.c_void_p), C.c_double(tau),
                                  fixed.ctypes.data_as(C.c_void_p), rounded.ctypes.data_as(C.c_void_p)))
    return fixed.astype(bool), rounded


def hpr_get_kernel_stats(h: Handle) -> dict:
    s = hpr_kernel_stats()
    _check(lib().hpr_get_kernel_stats(h.ptr, C.byref(s)))
    return _kstats(s)


def solve(lp, opts: Options | None = None, x0=None, y0=None):
    """Create, (optionally warm-start,) solve and fetch: returns (info, x, y, z)."""
    h = hpr_create(lp, opts)
    try:
        if x0 is not None or y0 is not None:
            hpr_set_start(h, x0, y0)
        info = hpr_solve(h)
        x, y, z = hpr_get_solution(h)
    finally:
        hpr_destroy(h)
    return info, x, y, z


# ----------------------------------------------------------------------------- batches

class Batch:
    """Owns an hpr_batch*; freed by hpr_batch_destroy (or when garbage collected)."""

    def __init__(self, ptr, sizes):
        self.ptr, self.sizes = ptr, sizes   # sizes: [(m, n)] per LP

    def __len__(self):
        return len(self.sizes)

    def __del__(self):
        if getattr(self, "ptr", None):
            try:
                lib().hpr_batch_destroy(self.ptr)
            except Exception:
                pass
            self.ptr = None


def _info(i: hpr_info) -> Info:
    return Info(TERM_NAMES.get(i.term, str(i.term)), i.iters, i.restarts, i.pobj, i.dobj, i.rel_p,
                i.rel_d, i.rel_gap, i.rel_kkt, i.lambda_, i.sigma, i.setup_s, i.solve_s, i.warm_start)


def hpr_batch_create(lps, opts: Options | None = None) -> Batch:
    arrs = [_LPArrays(lp) for lp in lps]
    structs = (hpr_lp * len(arrs))(*[a.s for a in arrs])
    o = (opts or Options()).to_c()
    out = C.c_void_p()
    _check(lib().hpr_batch_create(structs, len(arrs), C.byref(o), C.byref(out)))
    return Batch(out, [(lp.m, lp.n) for lp in lps])


def hpr_batch_destroy(b: Batch) -> None:
    if b.ptr:
        _check(lib().hpr_batch_destroy(b.ptr))
        b.ptr = None


def hpr_batch_set_bounds(b: Batch, i: int, col_lo=None, col_hi=None) -> None:
    n = b.sizes[i][1]
    lo, hi = _vec(col_lo, n, "col_lo"), _vec(col_hi, n, "col_hi")
    _check(lib().hpr_batch_set_bounds(b.ptr, C.c_int32(i),
                                      None if lo is None else lo.ctypes.data_as(C.c_void_p),
                                      None if hi is None else hi.ctypes.data_as(C.c_void_p)))


def hpr_batch_set_start(b: Batch, i: int, x0=None, y0=None) -> None:
    m, n = b.sizes[i]
    xa, ya = _vec(x0, n, "x0"), _vec(y0, m, "y0")
    _check(lib().hpr_batch_set_start(b.ptr, C.c_int32(i),
                                     None if xa is None else xa.ctypes.data_as(C.c_void_p),
                                     None if ya is None else ya.ctypes.data_as(C.c_void_p)))


def hpr_batch_solve(b: Batch):
    infos = (hpr_info * len(b))()
    _check(lib().hpr_batch_solve(b.ptr, infos))
    return [_info(i) for i in infos]


def hpr_batch_get_solution(b: Batch, i: int):
    m, n = b.sizes[i]
    x, y, z = np.zeros(n), np.zeros(max(m, 1)), np.zeros(n)
    _check(lib().hpr_batch_get_solution(b.ptr, C.c_int32(i), x.ctypes.data_as(C.c_void_p),
                                        y.ctypes.data_as(C.c_void_p), z.ctypes.data_as(C.c_void_p)))
    return x, y[:m], z


def hpr_batch_get_kernel_stats(b: Batch) -> dict:
    s = hpr_kernel_stats()
    _check(lib().hpr_batch_get_kernel_stats(b.ptr, C.byref(s)))
    return _kstats(s)


def batch_solve(lps, opts: Options | None = None, starts=None):
    """Create, (optionally warm-start,) solve and fetch a batch: returns [(info, x, y, z)]."""
    b = hpr_batch_create(lps, opts)
    try:
        if starts is not None:
            for i, (x0, y0) in enumerate(starts):
                if x0 is not None or y0 is not None:
                    hpr_batch_set_start(b, i, x0, y0)
        infos = hpr_batch_solve(b)
        out = [(infos[i], *hpr_batch_get_solution(b, i)) for i in range(len(b))]
    finally:
        hpr_batch_destroy(b)
    return out


def hpr_probe_stream(nbytes: int = 1 << 30, reps: int = 20):
    """(read GB/s, copy GB/s) of plain streaming kernels on the current device."""
    r, c = C.c_double(), C.c_double()
    _check(lib().hpr_probe_stream(C.c_int64(nbytes), C.c_int32(reps), C.byref(r), C.byref(c)))
    return r.value, c.value
