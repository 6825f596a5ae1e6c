"""CPU FP64 oracle of the paper's LP method.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU solver. It shares no code with the
GPU library; the only module both sides use is the input generator.

Contents
  * ``solve`` / ``hpr_step`` / ``scaling`` / ``kkt_c``: ctypes bindings of the plain C
    implementation in ``hpr_oracle.c`` (scaling of Section III-A, power method for
    lambda, the iteration eq.(hpr), KKT checks with restarts and sigma adaptation);
  * ``kkt``: an independent numpy evaluator of the relative KKT residuals of a point
    (the normalised residual map R of Theorem 1 plus the duality gap);
  * ``brute_force``: exact LP optimum of tiny bounded LPs by vertex enumeration, with
    the dual multipliers of a non-degenerate optimal vertex.
"""
from __future__ import annotations

import ctypes as C
import itertools
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hpr_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP for row loops only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _LP(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("row_lo", C.c_void_p), ("row_hi", C.c_void_p), ("col_lo", C.c_void_p),
                ("col_hi", C.c_void_p), ("c", C.c_void_p), ("obj_offset", C.c_double)]


class _Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int64), ("check_every", C.c_int32),
                ("ruiz_iters", C.c_int32), ("use_pc", C.c_int32), ("use_bc", C.c_int32),
                ("restart", C.c_int32), ("sigma_update", C.c_int32), ("sigma0", C.c_double),
                ("lambda_in", C.c_double), ("seed", C.c_uint64), ("power_max_iter", C.c_int32),
                ("power_tol", C.c_double), ("time_limit", C.c_double), ("sigma_smoothing", C.c_double),
                ("sigma_smoothing_warm", C.c_double),
                ("x0", C.c_void_p), ("y0", C.c_void_p)]


class _Info(C.Structure):
    _fields_ = [("term", C.c_int32), ("iters", C.c_int64), ("restarts", C.c_int64),
                ("pobj", C.c_double), ("dobj", C.c_double), ("rel_p", C.c_double),
                ("rel_d", C.c_double), ("rel_gap", C.c_double), ("rel_kkt", C.c_double),
                ("lambda_", C.c_double), ("sigma", C.c_double), ("setup_s", C.c_double),
                ("solve_s", C.c_double)]


TERM = {1: "solved", 2: "iter_limit", 3: "time_limit", 4: "numeric_fail", 5: "primal_infeasible",
        6: "dual_infeasible"}
_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.orc_solve.restype = C.c_int
        _lib.orc_kkt.restype = C.c_int
        _lib.orc_scaling.restype = C.c_int
        _lib.orc_hpr_step.restype = C.c_int
        _lib.orc_validate.restype = C.c_int
        _lib.orc_num_threads.restype = C.c_int
        _lib.orc_start_value.restype = C.c_double
        _lib.orc_start_value.argtypes = [C.c_uint64, C.c_uint64]
        _lib.orc_solve_trace.restype = C.c_int
        _lib.orc_restart_rule.restype = C.c_int
        _lib.orc_restart_rule.argtypes = [C.c_void_p, C.c_double, C.c_int64, C.c_int64, C.c_int32]
        _lib.orc_sigma_next.restype = C.c_double
        _lib.orc_sigma_next.argtypes = [C.c_double] * 5
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class _Pinned:
    """Keeps the contiguous copies alive while C reads them."""

    def __init__(self, lp):
        self.rp = np.ascontiguousarray(lp.row_ptr, np.int64)
        self.ci = np.ascontiguousarray(lp.col_idx, np.int32)
        self.v = _f64(lp.val)
        self.lo, self.hi = _f64(lp.row_lo), _f64(lp.row_hi)
        self.l, self.u, self.c = _f64(lp.col_lo), _f64(lp.col_hi), _f64(lp.c)
        self.s = _LP(lp.m, lp.n, len(self.ci),
                     self.rp.ctypes.data, self.ci.ctypes.data, self.v.ctypes.data,
                     self.lo.ctypes.data, self.hi.ctypes.data, self.l.ctypes.data,
                     self.u.ctypes.data, self.c.ctypes.data, float(lp.obj_offset))


@dataclass
class Options:
    tol: float = 1e-4
    max_iter: int = 100000
    check_every: int = 64
    ruiz_iters: int = 0
    use_pc: bool = True
    use_bc: bool = True
    restart: bool = True
    sigma_update: bool = True
    sigma0: float = 1.0
    lambda_in: float = 0.0
    seed: int = 0
    power_max_iter: int = 200
    power_tol: float = 1e-6
    time_limit: float = 0.0
    sigma_smoothing: float = 1.0
    sigma_smoothing_warm: float = 0.5


def _opts(o: Options, x0=None, y0=None):
    return _Opts(o.tol, o.max_iter, o.check_every, o.ruiz_iters, int(o.use_pc), int(o.use_bc),
                 int(o.restart), int(o.sigma_update), o.sigma0, o.lambda_in, o.seed,
                 o.power_max_iter, o.power_tol, o.time_limit, o.sigma_smoothing, o.sigma_smoothing_warm,
                 x0.ctypes.data if x0 is not None else None,
                 y0.ctypes.data if y0 is not None else None)


@dataclass
class Result:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
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


def solve(lp, opts: Options | None = None, x0=None, y0=None) -> Result:
    """Run the C oracle solver; returns the unscaled (x, y, z) of its last check."""
    lib = _load()
    opts = opts or Options()
    p = _Pinned(lp)
    x0a = _f64(x0) if x0 is not None else None
    y0a = _f64(y0) if y0 is not None else None
    o = _opts(opts, x0a, y0a)
    x = np.zeros(lp.n)
    y = np.zeros(max(lp.m, 1))
    z = np.zeros(lp.n)
    info = _Info()
    rc = lib.orc_solve(C.byref(p.s), C.byref(o), x.ctypes.data_as(C.c_void_p),
                       y.ctypes.data_as(C.c_void_p), z.ctypes.data_as(C.c_void_p), C.byref(info))
    if rc != 0:
        raise ValueError("oracle rejected the problem or options")
    return Result(x, y[:lp.m], z, TERM[info.term], info.iters, info.restarts, info.pobj, info.dobj,
                  info.rel_p, info.rel_d, info.rel_gap, info.rel_kkt, info.lambda_, info.sigma,
                  info.setup_s, info.solve_s)


TRACE_FIELDS = ("it", "k", "r", "r0", "r_prev", "restart", "sigma", "sigma_next", "ndx", "ndy")


def solve_trace(lp, opts: Options | None = None, x0=None, y0=None, vec_check: int = -1,
                cap: int = 100000):
    """``solve`` that also returns its check trace (test use).

    Returns (result, trace, vecs): trace is a dict of arrays, one entry per check that
    reached the restart decision (fields TRACE_FIELDS: iteration index, steps since the
    last restart, merit r, r0 and r_prev before the decision, the decision, sigma before
    and after it, the norms of the anchor move). vecs is None, or for the check with
    record index vec_check a dict of the scaled vectors the decision used: x (the
    step's start), xbar, x0 (the anchor), y, ybar, y0.
    """
    lib = _load()
    opts = opts or Options()
    p = _Pinned(lp)
    x0a = _f64(x0) if x0 is not None else None
    y0a = _f64(y0) if y0 is not None else None
    o = _opts(opts, x0a, y0a)
    x, y, z = np.zeros(lp.n), np.zeros(max(lp.m, 1)), np.zeros(lp.n)
    info = _Info()
    tr = np.zeros((cap, len(TRACE_FIELDS)))
    ntr = C.c_int64(0)
    vecs = np.zeros(3 * (lp.n + lp.m)) if vec_check >= 0 else None
    rc = lib.orc_solve_trace(C.byref(p.s), C.byref(o), x.ctypes.data_as(C.c_void_p),
                             y.ctypes.data_as(C.c_void_p), z.ctypes.data_as(C.c_void_p), C.byref(info),
                             tr.ctypes.data_as(C.c_void_p), C.c_int64(cap), C.byref(ntr),
                             C.c_int64(vec_check),
                             vecs.ctypes.data_as(C.c_void_p) if vecs is not None else None)
    if rc != 0:
        raise ValueError("oracle rejected the problem or options")
    res = Result(x, y[:lp.m], z, TERM[info.term], info.iters, info.restarts, info.pobj, info.dobj,
                 info.rel_p, info.rel_d, info.rel_gap, info.rel_kkt, info.lambda_, info.sigma,
                 info.setup_s, info.solve_s)
    tr = tr[:ntr.value]
    trace = {f: tr[:, i] for i, f in enumerate(TRACE_FIELDS)}
    vd = None
    if vecs is not None:
        n, m = lp.n, lp.m
        vd = dict(x=vecs[:n], xbar=vecs[n:2 * n], x0=vecs[2 * n:3 * n],
                  y=vecs[3 * n:3 * n + m], ybar=vecs[3 * n + m:3 * n + 2 * m],
                  y0=vecs[3 * n + 2 * m:3 * n + 3 * m])
    return res, trace, vd


class RestartRule:
    """The oracle's restart rule as a state machine (test use): feed one check at a time."""

    def __init__(self, enabled: bool = True):
        self.state = np.zeros(3)
        self.enabled = enabled

    def __call__(self, r: float, k: int, done: int) -> bool:
        return bool(_load().orc_restart_rule(self.state.ctypes.data_as(C.c_void_p), float(r),
                                             int(k), int(done), int(self.enabled)))

    @property
    def r0(self) -> float:
        return float(self.state[0])

    @property
    def r_prev(self) -> float:
        return float(self.state[1])


def sigma_next(sigma: float, ndx: float, ndy: float, lam: float, w: float = 1.0) -> float:
    """The oracle's sigma update at a restart, from the norms of the anchor move."""
    return float(_load().orc_sigma_next(sigma, ndx, ndy, lam, w))


def validate(lp) -> bool:
    return _load().orc_validate(C.byref(_Pinned(lp).s)) == 0


def kkt_c(lp, x, y, z) -> dict:
    """The C oracle's own KKT evaluator (used for its stopping test)."""
    lib = _load()
    p = _Pinned(lp)
    out = np.zeros(8)
    xa, ya, za = _f64(x), _f64(np.r_[y, 0.0]), _f64(z)
    lib.orc_kkt(C.byref(p.s), xa.ctypes.data_as(C.c_void_p), ya.ctypes.data_as(C.c_void_p),
                za.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p))
    return dict(rel_p=out[0], rel_d=out[1], rel_gap=out[2], rel_kkt=out[3], pobj=out[4],
                dobj=out[5], R=out[6])


def scaling(lp, opts: Options | None = None):
    """(Dr, Dc, beta_b, beta_c, lambda, power iterations) as the oracle computes them."""
    lib = _load()
    opts = opts or Options()
    p = _Pinned(lp)
    dr = np.zeros(max(lp.m, 1))
    dc = np.zeros(lp.n)
    out = np.zeros(4)
    rc = lib.orc_scaling(C.byref(p.s), C.byref(_opts(opts)), dr.ctypes.data_as(C.c_void_p),
                         dc.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return dr[:lp.m], dc, out[0], out[1], out[2], int(out[3])


def start_vector(seed: int, m: int) -> np.ndarray:
    """Power-method start vector (SplitMix64 draws mapped to [-1, 1))."""
    lib = _load()
    return np.array([lib.orc_start_value(seed, i) for i in range(m)])


def hpr_step(lp, sigma, lam, k, x0, y0, x, y):
    """One step of eq.(hpr) on the unscaled problem. Returns (x_next, y_next, xbar, ybar, zbar)."""
    lib = _load()
    p = _Pinned(lp)
    x0a, y0a = _f64(x0), _f64(np.r_[y0, 0.0])
    xa, ya = _f64(x).copy(), _f64(np.r_[y, 0.0]).copy()
    xb, zb = np.zeros(lp.n), np.zeros(lp.n)
    yb = np.zeros(lp.m + 1)
    lib.orc_hpr_step(C.byref(p.s), C.c_double(sigma), C.c_double(lam), C.c_int64(k),
                     x0a.ctypes.data_as(C.c_void_p), y0a.ctypes.data_as(C.c_void_p),
                     xa.ctypes.data_as(C.c_void_p), ya.ctypes.data_as(C.c_void_p),
                     xb.ctypes.data_as(C.c_void_p), yb.ctypes.data_as(C.c_void_p),
                     zb.ctypes.data_as(C.c_void_p))
    return xa, ya[:lp.m], xb, yb[:lp.m], zb


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(n: int) -> int:
    """Threads of the oracle's row loops from now on; returns the number in use."""
    return _load().orc_set_num_threads(int(n))


# ----------------------------------------------------------------------------- numpy KKT

def _finite_side(lo, hi):
    fl, fh = np.isfinite(lo), np.isfinite(hi)
    b = np.zeros_like(lo)
    both = fl & fh
    b[both] = np.where(np.abs(lo[both]) > np.abs(hi[both]), lo[both], hi[both])
    b[fl & ~fh] = lo[fl & ~fh]
    b[fh & ~fl] = hi[fh & ~fl]
    return b


def _bound_term(bound_lo, bound_hi, mult):
    """sum(lo * mult+ - hi * mult-) with 0 * inf = 0; returns (value, infinite?)."""
    pos, neg = np.maximum(mult, 0.0), np.maximum(-mult, 0.0)
    bad = ((pos > 0) & ~np.isfinite(bound_lo)) | ((neg > 0) & ~np.isfinite(bound_hi))
    lo = np.where(pos > 0, bound_lo, 0.0)
    hi = np.where(neg > 0, bound_hi, 0.0)
    return float(np.sum(lo * pos) - np.sum(hi * neg)), bool(bad.any())


def kkt(lp, x, y, z) -> dict:
    """Relative KKT residuals of (x, y, z) on the original LP (numpy, FP64).

    Primal: ||max(lo - Ax, 0, Ax - hi)|| / (1 + ||b||), b the finite row sides.
    Dual:   ||c - A^T y - z|| / (1 + ||c||).
    Gap:    |pobj - dobj| / (1 + |pobj| + |dobj|) with the Lagrangian dual
            dobj = sum(lo y+ - hi y-) + sum(l z+ - u z-) + offset (1 if it is -inf).
    """
    A = lp.to_scipy()
    x, y, z = np.asarray(x, float), np.asarray(y, float), np.asarray(z, float)
    ax = A @ x
    rp = np.maximum(np.maximum(lp.row_lo - ax, 0.0), ax - lp.row_hi)
    b = _finite_side(lp.row_lo, lp.row_hi)
    rel_p = np.linalg.norm(rp) / (1.0 + np.linalg.norm(b))
    rd = lp.c - A.T @ y - z
    rel_d = np.linalg.norm(rd) / (1.0 + np.linalg.norm(lp.c))
    pobj = float(lp.c @ x + lp.obj_offset)
    ty, iy = _bound_term(lp.row_lo, lp.row_hi, y)
    tz, iz = _bound_term(lp.col_lo, lp.col_hi, z)
    dobj = ty + tz + lp.obj_offset
    if iy or iz:
        rel_gap, dobj = 1.0, -np.inf
    else:
        rel_gap = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj))
    return dict(rel_p=float(rel_p), rel_d=float(rel_d), rel_gap=float(rel_gap),
                rel_kkt=float(max(rel_p, rel_d, rel_gap)), pobj=pobj, dobj=float(dobj))


# ----------------------------------------------------------------------------- brute force

def brute_force(lp, feas_tol: float = 1e-9, batch: int = 20000):
    """Exact optimum of a tiny bounded LP by enumerating vertices.

    Every vertex lies on n linearly independent hyperplanes taken from the finite
    row sides a_i x = lo_i / hi_i and finite column bounds x_j = l_j / u_j. All
    n-subsets are solved (skipping near-singular ones), feasible solutions kept,
    and the smallest objective returned as (obj, x). Requires finite column bounds.
    """
    A = lp.to_scipy().toarray()
    n = lp.n
    if not (np.all(np.isfinite(lp.col_lo)) and np.all(np.isfinite(lp.col_hi))):
        raise ValueError("brute force needs a bounded box")
    H, h = [], []
    for i in range(lp.m):
        for v in {lp.row_lo[i], lp.row_hi[i]}:
            if np.isfinite(v):
                H.append(A[i]); h.append(v)
    for j in range(n):
        e = np.zeros(n); e[j] = 1.0
        for v in {lp.col_lo[j], lp.col_hi[j]}:
            H.append(e); h.append(v)
    H, h = np.array(H), np.array(h)
    best, best_x = np.inf, None
    combos = itertools.combinations(range(len(h)), n)
    while True:
        chunk = list(itertools.islice(combos, batch))
        if not chunk:
            break
        idx = np.array(chunk)
        Ms, rs = H[idx], h[idx]
        cond = np.linalg.cond(Ms)
        ok = np.isfinite(cond) & (cond < 1e12)
        if not ok.any():
            continue
        xs = np.linalg.solve(Ms[ok], rs[ok][..., None])[..., 0]
        ax = xs @ A.T
        scale = 1.0 + np.abs(ax)
        feas = (np.all(ax >= lp.row_lo - feas_tol * scale, axis=1)
                & np.all(ax <= lp.row_hi + feas_tol * scale, axis=1)
                & np.all(xs >= lp.col_lo - feas_tol, axis=1)
                & np.all(xs <= lp.col_hi + feas_tol, axis=1))
        if feas.any():
            obj = xs[feas] @ lp.c
            k = int(np.argmin(obj))
            if obj[k] < best:
                best, best_x = float(obj[k]), xs[feas][k]
    return best + lp.obj_offset, best_x


def vertex_duals(lp, x, act_tol: float = 1e-9):
    """Dual multipliers (y, z) at a vertex x when exactly n hyperplanes are active.

    Solves c = A_act^T y_act + z_act on the active set; returns None when the vertex is
    degenerate (more than n active) or the multipliers have the wrong sign (not optimal).
    """
    A = lp.to_scipy().toarray()
    m, n = lp.m, lp.n
    ax = A @ x
    cols, kinds = [], []
    for i in range(m):
        at_lo = np.isfinite(lp.row_lo[i]) and abs(ax[i] - lp.row_lo[i]) <= act_tol * (1 + abs(ax[i]))
        at_hi = np.isfinite(lp.row_hi[i]) and abs(ax[i] - lp.row_hi[i]) <= act_tol * (1 + abs(ax[i]))
        if at_lo or at_hi:
            cols.append(A[i]); kinds.append(("row", i, at_lo, at_hi))
    for j in range(n):
        at_lo = abs(x[j] - lp.col_lo[j]) <= act_tol
        at_hi = abs(x[j] - lp.col_hi[j]) <= act_tol
        if at_lo or at_hi:
            e = np.zeros(n); e[j] = 1.0
            cols.append(e); kinds.append(("col", j, at_lo, at_hi))
    if len(cols) != n:
        return None
    Mt = np.array(cols).T
    if np.linalg.cond(Mt) > 1e10:
        return None
    mult = np.linalg.solve(Mt, lp.c)
    y, z = np.zeros(m), np.zeros(n)
    for val, (kind, idx, at_lo, at_hi) in zip(mult, kinds):
        if val > 1e-12 and not at_lo:
            return None
        if val < -1e-12 and not at_hi:
            return None
        if kind == "row":
            y[idx] = val
        else:
            z[idx] = val
    return y, z
