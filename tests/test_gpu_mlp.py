"""The warm-start network's GPU kernels (MFMA BF16 products, FP32 accumulate, Adam)
against the FP64 reference in oracle/mlp.py, entry by entry.

The reference gets the BF16-rounded weights and inputs the GPU uses and rounds the hidden
activations and the backward pass's gradients to BF16 at the same points (the network's
stated storage precision), so what separates the two is the summation order of the FP32
products. That order can push a value across a BF16 rounding boundary, which moves it by one
BF16 step (2^-8 of its size) and carries on through later layers; every entry must lie within
2^-6 (a few such steps) of the sum of the magnitudes of its terms (oracle.mlp.magnitudes). A
wrong tile, a dropped edge row or a transposed operand moves entries by their own size,
which is of the order of that sum (measured on a CPU model of the kernels: a zeroed 16 x 16
tile of dW sits at 0.7 to 1.0 of it, order effects at 2e-3 at most)."""
import numpy as np
import pytest

from oracle import mlp as ref
from paper_2510_10891_amd import mlp

pytestmark = pytest.mark.gpu

TOL = 2.0 ** -6


def bf16(a):
    """Round values to the nearest BF16 (ties to even) through float32, returned as float64."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


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


# widths and row counts off the 16-wide tiles on purpose (M, N and K of every product)
SHAPES = [([12, 256, 256, 4], 1000), ([9, 256, 256, 1], 333), ([16, 32, 5], 17), ([3, 7], 64),
          ([20, 48, 33, 7], 45), ([12, 70, 40, 3], 5000)]   # the last: dW products split over the depth


@pytest.mark.parametrize("sizes,rows", SHAPES)
def test_forward_matches_reference_entrywise(sizes, rows):
    params, X, T = problem(sizes, rows, 0)
    net = mlp.MLP(sizes, params)
    Y = net.forward(X)
    Ws, bs, Xb = reference(params, sizes, X)
    out, _, _ = ref.forward(Xb, Ws, bs, rnd=bf16)
    mo, _, _ = ref.magnitudes(Xb, Ws, bs, T.astype(np.float64), rnd=bf16)
    err = np.abs(Y - out)
    assert np.all(err <= TOL * mo), (err / mo).max()


@pytest.mark.parametrize("sizes,rows", SHAPES)
def test_gradients_match_reference_entrywise(sizes, rows):
    params, X, T = problem(sizes, rows, 1)
    net = mlp.MLP(sizes, params)
    loss, g = net.gradients(X, T)
    Ws, bs, Xb = reference(params, sizes, X)
    T64 = T.astype(np.float64)
    rloss, dWs, dbs = ref.backward(Xb, Ws, bs, T64, rnd=bf16)
    _, mW, mb = ref.magnitudes(Xb, Ws, bs, T64, rnd=bf16)
    assert abs(loss - rloss) <= 1e-3 * rloss
    gW, gb = mlp.unpack(g, sizes)
    for i in range(len(Ws)):
        eW = np.abs(gW[i] - dWs[i])
        assert np.all(eW <= TOL * mW[i] + 1e-12), (f"dW{i}", (eW / (mW[i] + 1e-300)).max())
        eb = np.abs(gb[i] - dbs[i])
        assert np.all(eb <= TOL * mb[i] + 1e-12), (f"db{i}", (eb / (mb[i] + 1e-300)).max())


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
