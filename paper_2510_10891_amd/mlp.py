"""Python binding of the warm-start network calls of libhprlp.so (hpr_mlp_*).

Argument marshalling only: forward, gradients and Adam steps run in the library's kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from .hprlp import HPR_OK, HprError, lib

_F32P = C.POINTER(C.c_float)


def _setup():
    L = lib()
    if not getattr(L, "_mlp_ready", False):
        L.hpr_mlp_last_error.restype = C.c_char_p
        for name in ("hpr_mlp_create", "hpr_mlp_num_params", "hpr_mlp_set_params", "hpr_mlp_get_params",
                     "hpr_mlp_forward", "hpr_mlp_forward_device", "hpr_mlp_gradients", "hpr_mlp_train_step",
                     "hpr_mlp_destroy"):
            getattr(L, name).restype = C.c_int
        L._mlp_ready = True
    return L


def _check(rc):
    if rc != HPR_OK:
        raise HprError(rc, _setup().hpr_mlp_last_error().decode())


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def param_layout(sizes):
    """[(W offset, W shape, b offset, b size)] of the flat parameter array."""
    out, off = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        out.append((off, (a, b), off + a * b, b))
        off += a * b + b
    return out, off


def pack(Ws, bs):
    return np.concatenate([np.concatenate([np.ravel(W), np.ravel(b)]) for W, b in zip(Ws, bs)]).astype(np.float32)


def unpack(params, sizes):
    lay, _ = param_layout(sizes)
    Ws = [params[o:o + s[0] * s[1]].reshape(s) for o, s, _, _ in lay]
    bs = [params[bo:bo + n] for _, _, bo, n in lay]
    return Ws, bs


def init_params(sizes, seed=0):
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    Ws = [rng.standard_normal((a, b)) * np.sqrt(2.0 / a) for a, b in zip(sizes[:-1], sizes[1:])]
    bs = [np.zeros(b) for b in sizes[1:]]
    return pack(Ws, bs)


class MLP:
    def __init__(self, sizes, params=None, stream=None):
        L = _setup()
        self.sizes = [int(s) for s in sizes]
        arr = (C.c_int32 * len(self.sizes))(*self.sizes)
        p = None if params is None else _f32(params)
        out = C.c_void_p()
        _check(L.hpr_mlp_create(len(self.sizes) - 1, arr, None if p is None else p.ctypes.data_as(_F32P),
                                C.c_void_p(stream) if stream else None, C.byref(out)))
        self.ptr = out
        n = C.c_int64()
        _check(L.hpr_mlp_num_params(self.ptr, C.byref(n)))
        self.nparams = n.value

    def __del__(self):
        if getattr(self, "ptr", None):
            try:
                _setup().hpr_mlp_destroy(self.ptr)
            except Exception:
                pass
            self.ptr = None

    def set_params(self, params):
        p = _f32(params)
        assert p.size == self.nparams
        _check(_setup().hpr_mlp_set_params(self.ptr, p.ctypes.data_as(_F32P)))

    def get_params(self):
        p = np.zeros(self.nparams, np.float32)
        _check(_setup().hpr_mlp_get_params(self.ptr, p.ctypes.data_as(_F32P)))
        return p

    def forward(self, X):
        X = _f32(X)
        Y = np.zeros((X.shape[0], self.sizes[-1]), np.float32)
        _check(_setup().hpr_mlp_forward(self.ptr, X.ctypes.data_as(_F32P), C.c_int64(X.shape[0]),
                                        Y.ctypes.data_as(_F32P)))
        return Y

    def forward_device(self, x_ptr: int, n: int, y_ptr: int):
        """hpr_mlp_forward_device on caller-owned FP32 device arrays (e.g. torch tensors' data_ptr());
        enqueued on the handle's stream, no wait, no allocation."""
        _check(_setup().hpr_mlp_forward_device(self.ptr, C.c_void_p(x_ptr), C.c_int64(n), C.c_void_p(y_ptr)))

    def gradients(self, X, T):
        X, T = _f32(X), _f32(T)
        g = np.zeros(self.nparams, np.float32)
        loss = C.c_float()
        _check(_setup().hpr_mlp_gradients(self.ptr, X.ctypes.data_as(_F32P), T.ctypes.data_as(_F32P),
                                          C.c_int64(X.shape[0]), g.ctypes.data_as(_F32P), C.byref(loss)))
        return float(loss.value), g

    def train_step(self, X, T, lr):
        X, T = _f32(X), _f32(T)
        loss = C.c_float()
        _check(_setup().hpr_mlp_train_step(self.ptr, X.ctypes.data_as(_F32P), T.ctypes.data_as(_F32P),
                                           C.c_int64(X.shape[0]), C.c_float(lr), C.byref(loss)))
        return float(loss.value)
