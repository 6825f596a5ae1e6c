"""FP64 reference of the warm-start network: a plain multilayer perceptron.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): the GPU training and inference
kernels are checked against these functions; the product never imports them.

Network: h_0 = X; z_i = h_i W_i + b_i; h_{i+1} = max(z_i, 0) for every layer but the
last, whose z is the output. Loss: L = 0.5 * mean over all output entries of
(out - target)^2. Gradients by the chain rule written out layer by layer; Adam as
published by Kingma and Ba (2015) with bias correction.
"""
from __future__ import annotations

import numpy as np


def forward(X, Ws, bs):
    """Returns (output, [h_0, ..., h_{L-1}], [z_0, ..., z_{L-1}])."""
    h = np.asarray(X, np.float64)
    hs, zs = [], []
    for i, (W, b) in enumerate(zip(Ws, bs)):
        hs.append(h)
        z = h @ np.asarray(W, np.float64) + np.asarray(b, np.float64)
        zs.append(z)
        h = np.maximum(z, 0.0) if i < len(Ws) - 1 else z
    return h, hs, zs


def loss(out, target):
    d = out - target
    return 0.5 * float(np.mean(d * d))


def backward(X, Ws, bs, target):
    """Loss and its gradients (dWs, dbs) with respect to every weight and bias."""
    out, hs, zs = forward(X, Ws, bs)
    N = out.size
    g = (out - target) / N              # d loss / d out
    dWs, dbs = [None] * len(Ws), [None] * len(Ws)
    for i in reversed(range(len(Ws))):
        dWs[i] = hs[i].T @ g
        dbs[i] = g.sum(axis=0)
        if i > 0:
            g = (g @ np.asarray(Ws[i], np.float64).T) * (zs[i - 1] > 0)
    return loss(out, target), dWs, dbs


def adam(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns the new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
