"""The C interface without a GPU: the library loads, exports what include/hprlp.h
declares, and rejects bad input before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2510_10891_amd import hprlp
from paper_2510_10891_amd.scuc import LP
from tests.helpers import dense_lp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(hpr_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    L = hprlp.lib()
    names = declared_functions()
    assert "hpr_solve" in names and "hpr_create" in names
    for name in names:
        assert hasattr(L, name), name


def test_default_opts_match_python_mirror():
    o = hprlp.hpr_default_opts()
    p = hprlp.Options()
    for f in ("tol", "max_iter", "precision", "scaling", "ruiz_iters", "check_every", "sigma0",
              "restart", "sigma_update", "power_max_iter", "power_tol", "use_graph", "warm_fallback",
              "warm_fallback_ratio", "unroll", "lds_windows", "sigma_smoothing", "sigma_smoothing_warm",
              "profile"):
        assert getattr(o, f) == getattr(p, f), f


def _good():
    return dense_lp([[1.0, 2.0], [0.0, 1.0]], [0.0, -1.0], [1.0, np.inf], [0, 0], [1, 1], [1.0, -1.0])


BAD = {
    "nan value": lambda g: g.replace(val=np.array([np.nan, 2.0, 1.0])),
    "lo > hi": lambda g: g.replace(row_lo=np.array([2.0, -1.0])),
    "col lo > hi": lambda g: g.replace(col_lo=np.array([0.0, 2.0])),
    "inf cost": lambda g: g.replace(c=np.array([np.inf, 0.0])),
    "col out of range": lambda g: g.replace(col_idx=np.array([0, 2, 1], np.int32)),
    "repeated col": lambda g: g.replace(col_idx=np.array([1, 1, 1], np.int32)),
    "bad row_ptr end": lambda g: g.replace(row_ptr=np.array([0, 2, 4], np.int64)),
    "decreasing row_ptr": lambda g: g.replace(row_ptr=np.array([0, 3, 3], np.int64),
                                              col_idx=np.array([0, 1, 1], np.int32)),
    "lower bound +inf": lambda g: g.replace(row_lo=np.array([np.inf, -1.0]), row_hi=np.array([np.inf, np.inf])),
    "nan bound": lambda g: g.replace(col_hi=np.array([np.nan, 1.0])),
}


@pytest.mark.parametrize("case", sorted(BAD))
def test_create_rejects_bad_problem(case):
    lp = BAD[case](_good())
    with pytest.raises(hprlp.HprError) as e:
        hprlp.hpr_create(lp)
    assert e.value.code == hprlp.HPR_ERR_INVALID
    assert hprlp.hpr_last_error() != ""


def test_create_rejects_no_columns():
    lp = LP(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0), np.zeros(0), np.zeros(0),
            np.zeros(0), np.zeros(0), np.zeros(0))
    with pytest.raises(hprlp.HprError) as e:
        hprlp.hpr_create(lp)
    assert e.value.code == hprlp.HPR_ERR_INVALID


@pytest.mark.parametrize("opt", [dict(max_iter=0), dict(check_every=0), dict(sigma0=0.0), dict(sigma0=-1.0),
                                 dict(tol=-1.0), dict(precision=7), dict(power_max_iter=0),
                                 dict(lambda_=float("nan")), dict(warm_fallback_ratio=0.0), dict(warm_fallback=3),
                                 dict(unroll=3), dict(lds_windows=8), dict(lds_windows=-2),
                                 dict(sigma_smoothing=0.0), dict(sigma_smoothing=1.5),
                                 dict(sigma_smoothing_warm=0.0), dict(stall_iters=-1)])
def test_create_rejects_bad_options(opt):
    with pytest.raises(hprlp.HprError) as e:
        hprlp.hpr_create(_good(), hprlp.Options(**opt))
    assert e.value.code == hprlp.HPR_ERR_INVALID


def test_null_handles_are_rejected():
    L = hprlp.lib()
    assert L.hpr_solve(None, None) == hprlp.HPR_ERR_INVALID
    assert L.hpr_get_solution(None, None, None, None) == hprlp.HPR_ERR_INVALID
    assert L.hpr_set_bounds(None, None, None) == hprlp.HPR_ERR_INVALID
    assert L.hpr_set_start(None, None, None) == hprlp.HPR_ERR_INVALID
    assert L.hpr_destroy(None) == hprlp.HPR_OK
    assert L.hpr_create(None, None, None) == hprlp.HPR_ERR_INVALID
    out = C.c_void_p()
    assert L.hpr_create(None, None, C.byref(out)) == hprlp.HPR_ERR_INVALID


def test_batch_create_rejects_bad_member_and_counts():
    good = _good()
    bad = BAD["nan value"](good)
    with pytest.raises(hprlp.HprError) as e:
        hprlp.hpr_batch_create([good, good, bad])
    assert e.value.code == hprlp.HPR_ERR_INVALID
    assert "LP 2" in hprlp.hpr_last_error()
    L = hprlp.lib()
    out = C.c_void_p()
    arr = (hprlp.hpr_lp * 1)(hprlp._LPArrays(good).s)
    assert L.hpr_batch_create(arr, 0, None, C.byref(out)) == hprlp.HPR_ERR_INVALID
    assert L.hpr_batch_create(arr, 2000, None, C.byref(out)) == hprlp.HPR_ERR_INVALID
    assert L.hpr_batch_solve(None, None) == hprlp.HPR_ERR_INVALID
    assert L.hpr_batch_get_solution(None, 0, None, None, None) == hprlp.HPR_ERR_INVALID
    assert L.hpr_batch_destroy(None) == hprlp.HPR_OK


@pytest.mark.parametrize("field,length", [("row_ptr", 2), ("row_lo", 0), ("row_hi", 3), ("col_lo", 1),
                                          ("col_hi", 5), ("c", 1)])
def test_binding_rejects_arrays_of_the_wrong_length(field, length):
    """The library reads m + 1, m or n entries through raw pointers: short arrays are refused
    before the call."""
    good = _good()
    arr = getattr(good, field)
    bad = good.replace(**{field: np.resize(arr, length).astype(arr.dtype)})
    with pytest.raises(ValueError):
        hprlp._LPArrays(bad)


def test_binding_rejects_start_and_bounds_of_the_wrong_length():
    h = hprlp.Handle(None, 2, 3)
    with pytest.raises(ValueError):
        hprlp.hpr_set_start(h, np.zeros(2), None)
    with pytest.raises(ValueError):
        hprlp.hpr_set_start(h, None, np.zeros(3))
    with pytest.raises(ValueError):
        hprlp.hpr_set_bounds(h, np.zeros(4), None)
