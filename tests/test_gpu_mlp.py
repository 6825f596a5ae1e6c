"""The warm-start network's GPU kernels (MFMA BF16 products, FP32 accumulate, Adam)
against the FP64 reference in oracle/mlp.py.

The reference gets the BF16-rounded weights and inputs the GPU uses; what remains is the
BF16 rounding of hidden activations and gradients and the summation order, so results are
compared with relative tolerances derived from BF16's 8-bit mantissa (2^-8 ~ 4e-3 per
rounding, a few roundings per path): 2e-2 on norms of whole arrays."""
import numpy as np
import pytest

from oracle import mlp as ref
from paper_2510_10891_amd import mlp

pytestmark = pytest.mark.gpu


def bf16(a):
    """Round float32 values to the nearest BF16 (ties to even), returned as float64."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def relerr(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(1e-30, np.linalg.norm(np.ravel(b)))


def problem(sizes, rows, seed):
    rng = np.random.default_rng(seed)
    params = mlp.init_params(sizes, seed)
    params[-sizes[-1]:] = 0.1                    # nonzero output bias
    X = rng.standard_normal((rows, sizes[0])).astype(np.float32)
    T = rng.standard_normal((rows, sizes[-1])).astype(np.float32)
    return params, X, T


def reference(params, sizes, X):
    Ws, bs = mlp.unpack(params.astype(np.float64), sizes)
    Ws = [bf16(W) for W in Ws]                   # the products use BF16 weights
    return Ws, [np.asarray(b, np.float64) for b in bs], bf16(X)


SHAPES = [([12, 256, 256, 4], 1000), ([9, 256, 256, 1], 333), ([16, 32, 5], 17), ([3, 7], 64)]


@pytest.mark.parametrize("sizes,rows", SHAPES)
def test_forward_matches_reference(sizes, rows):
    params, X, _ = problem(sizes, rows, 0)
    net = mlp.MLP(sizes, params)
    Y = net.forward(X)
    Ws, bs, Xb = reference(params, sizes, X)
    out, _, _ = ref.forward(Xb, Ws, bs)
    assert relerr(Y, out) < 2e-2


@pytest.mark.parametrize("sizes,rows", SHAPES)
def test_gradients_match_reference(sizes, rows):
    params, X, T = problem(sizes, rows, 1)
    net = mlp.MLP(sizes, params)
    loss, g = net.gradients(X, T)
    Ws, bs, Xb = reference(params, sizes, X)
    rloss, dWs, dbs = ref.backward(Xb, Ws, bs, T.astype(np.float64))
    assert abs(loss - rloss) <= 2e-2 * rloss
    gW, gb = mlp.unpack(g, sizes)
    for i in range(len(Ws)):
        assert relerr(gW[i], dWs[i]) < 3e-2, f"dW{i}"
        assert relerr(gb[i], dbs[i]) < 3e-2, f"db{i}"


def test_adam_step_matches_reference():
    sizes, rows = [12, 256, 256, 4], 512
    params, X, T = problem(sizes, rows, 2)
    net = mlp.MLP(sizes, params)
    _, g = net.gradients(X, T)
    net.train_step(X, T, lr=1e-3)
    w, _, _ = ref.adam(params.astype(np.float64), g.astype(np.float64), np.zeros(params.size),
                       np.zeros(params.size), 1, lr=1e-3)
    assert np.abs(net.get_params() - w).max() <= 1e-6 + 1e-5 * np.abs(w).max()


def test_training_fits_a_smooth_target():
    rng = np.random.default_rng(4)
    sizes = [6, 256, 256, 2]
    X = rng.uniform(-1, 1, (4096, 6)).astype(np.float32)
    T = np.stack([np.sin(2 * X[:, 0]) * X[:, 1], np.maximum(X[:, 2], 0) + 0.5 * X[:, 3] ** 2], 1).astype(np.float32)
    net = mlp.MLP(sizes, mlp.init_params(sizes, 0))
    first = net.gradients(X, T)[0]
    for step in range(400):
        idx = rng.integers(0, len(X), 512)
        net.train_step(X[idx], T[idx], lr=2e-3)
    last = net.gradients(X, T)[0]
    assert last < 0.1 * first
