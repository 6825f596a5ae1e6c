"""Pins of the FP64 warm-start network reference (oracle/mlp.py)."""
import numpy as np
import pytest

from oracle import mlp


def _net(rng, sizes):
    Ws = [rng.standard_normal((a, b)) / np.sqrt(a) for a, b in zip(sizes[:-1], sizes[1:])]
    bs = [0.1 * rng.standard_normal(b) for b in sizes[1:]]
    return Ws, bs


@pytest.mark.parametrize("sizes", [(5, 7, 6, 3), (4, 2), (9, 16, 16, 1)])
def test_gradients_match_central_differences(sizes):
    rng = np.random.default_rng(len(sizes))
    Ws, bs = _net(rng, sizes)
    X = rng.standard_normal((11, sizes[0]))
    T = rng.standard_normal((11, sizes[-1]))
    L, dWs, dbs = mlp.backward(X, Ws, bs, T)
    h = 1e-6
    for i in range(len(Ws)):
        for idx in np.ndindex(Ws[i].shape):
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[i][idx] += h
            Wm[i][idx] -= h
            fd = (mlp.loss(mlp.forward(X, Wp, bs)[0], T) - mlp.loss(mlp.forward(X, Wm, bs)[0], T)) / (2 * h)
            assert abs(fd - dWs[i][idx]) <= 1e-6 * (1 + abs(fd))
        for j in range(len(bs[i])):
            bp = [b.copy() for b in bs]
            bm = [b.copy() for b in bs]
            bp[i][j] += h
            bm[i][j] -= h
            fd = (mlp.loss(mlp.forward(X, Ws, bp)[0], T) - mlp.loss(mlp.forward(X, Ws, bm)[0], T)) / (2 * h)
            assert abs(fd - dbs[i][j]) <= 1e-6 * (1 + abs(fd))


def test_relu_only_between_layers():
    rng = np.random.default_rng(3)
    Ws, bs = _net(rng, (3, 4, 2))
    X = rng.standard_normal((5, 3))
    out, hs, zs = mlp.forward(X, Ws, bs)
    assert np.allclose(hs[1], np.maximum(zs[0], 0))
    assert np.allclose(out, zs[1])            # the last layer is linear
    assert (out < 0).any()


def test_adam_first_step_moves_by_lr_against_the_sign():
    g = np.array([3.0, -0.5, 1e-3])
    w, m, v = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), t=1, lr=0.01)
    assert np.allclose(w, -0.01 * np.sign(g), rtol=1e-4)


def test_adam_minimises_a_quadratic():
    rng = np.random.default_rng(0)
    target = rng.standard_normal(6)
    w, m, v = np.zeros(6), np.zeros(6), np.zeros(6)
    for t in range(1, 3001):
        w, m, v = mlp.adam(w, w - target, m, v, t, lr=0.01)
    assert np.allclose(w, target, atol=1e-3)
