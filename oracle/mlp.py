"""FP64 reference of the warm-start network: a plain multilayer perceptron.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): the GPU training and inference
kernels are checked against these functions; the product never imports them.

Network: h_0 = X; z_i = h_i W_i + b_i; h_{i+1} = max(z_i, 0) for every layer but the
last, whose z is the output. Loss: L = 0.5 * mean over all output entries of
(out - target)^2. Gradients by the chain rule written out layer by layer; Adam as
published by Kingma and Ba (2015) with bias correction.

`rnd` (optional) is applied where the network's stated storage precision rounds a value: the
hidden activations h_1.. in the forward pass, and the gradient at the output and each
backpropagated gradient g W^T in the backward pass. Everything else is FP64. With rnd the
reference takes the same rounding decisions as a BF16-activation network, so only the
summation order of the products separates it from one.
"""
from __future__ import annotations

import numpy as np


def forward(X, Ws, bs, rnd=None):
    """Returns (output, [h_0, ..., h_{L-1}], [z_0, ..., z_{L-1}])."""
    h = np.asarray(X, np.float64)
    hs, zs = [], []
    for i, (W, b) in enumerate(zip(Ws, bs)):
        hs.append(h)
        z = h @ np.asarray(W, np.float64) + np.asarray(b, np.float64)
        zs.append(z)
        if i < len(Ws) - 1:
            h = np.maximum(z, 0.0)
            if rnd is not None:
                h = rnd(h)
        else:
            h = z
    return h, hs, zs


def magnitudes(X, Ws, bs, target, rnd=None):
    """The same passes on absolute values: per entry, the sum of the magnitudes of the terms
    each output, weight gradient and bias gradient is made of (|h| |W| + |b|, |h|^T |g|,
    sum |g|), the scale against which summation-order differences are measured."""
    out, hs, zs = forward(X, Ws, bs, rnd)
    mo = np.abs(hs[-1]) @ np.abs(np.asarray(Ws[-1], np.float64)) + np.abs(np.asarray(bs[-1], np.float64))
    g = (out - target) / out.size
    if rnd is not None:
        g = rnd(g)
    mW, mb = [None] * len(Ws), [None] * len(Ws)
    for i in reversed(range(len(Ws))):
        mW[i] = np.abs(hs[i]).T @ np.abs(g)
        mb[i] = np.abs(g).sum(axis=0)
        if i > 0:
            gh = g @ np.asarray(Ws[i], np.float64).T
            if rnd is not None:
                gh = rnd(gh)
            g = gh * (zs[i - 1] > 0)
    return mo, mW, mb


def loss(out, target):
    d = out - target
    return 0.5 * float(np.mean(d * d))


def backward(X, Ws, bs, target, rnd=None):
    """Loss and its gradients (dWs, dbs) with respect to every weight and bias."""
    out, hs, zs = forward(X, Ws, bs, rnd)
    N = out.size
    g = (out - target) / N              # d loss / d out
    if rnd is not None:
        g = rnd(g)
    dWs, dbs = [None] * len(Ws), [None] * len(Ws)
    for i in reversed(range(len(Ws))):
        dWs[i] = hs[i].T @ g
        dbs[i] = g.sum(axis=0)
        if i > 0:
            gh = g @ np.asarray(Ws[i], np.float64).T
            if rnd is not None:
                gh = rnd(gh)
            g = gh * (zs[i - 1] > 0)
    return loss(out, target), dWs, dbs


def adam(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns the new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
