"""Per-block precision selector network, plain FP64.

Test infrastructure only (see the package docstring).

A multilayer perceptron maps the 16 block features to three classes
(0 = FP64, 1 = FP32, 2 = FP16): standardised input -> 64 ReLU -> 64 ReLU -> 3
logits -> softmax. Training minimises the mean softmax cross-entropy with Adam.
The paper's Sec. 4.5 relates convergence delay to block features (multiscale
strength, diagonal dominance); the network learns that relation from labels
the method itself generates.

Parameter vector layout (float, 5443 entries), shared by name with the GPU
kernels' documentation but implemented independently:
  W1[64,16] b1[64] W2[64,64] b2[64] W3[3,64] b3[3]   (row-major, out x in)
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT = 16, 64, 3
SHAPES = (("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
          ("W3", (NOUT, NH)), ("b3", (NOUT,)))
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shp in SHAPES:
        sz = int(np.prod(shp))
        out[name] = theta[o:o + sz].reshape(shp)
        o += sz
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(rng):
    """He-uniform weights, zero biases."""
    d = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shp[1])
            d[name] = rng.uniform(-lim, lim, size=shp)
        else:
            d[name] = np.zeros(shp)
    return pack(d)


def forward(theta, X, mu, sigma):
    """Returns (logits (N,3), cache)."""
    p = unpack(theta)
    Xn = (np.asarray(X, dtype=np.float64) - mu) / sigma
    z1 = Xn @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    logits = h2 @ p["W3"].T + p["b3"]
    return logits, (Xn, z1, h1, z2, h2)


def softmax(logits):
    m = np.max(logits, axis=1, keepdims=True)
    e = np.exp(logits - m)
    return e / np.sum(e, axis=1, keepdims=True)


def loss(theta, X, y, mu, sigma):
    """Mean softmax cross-entropy."""
    logits, _ = forward(theta, X, mu, sigma)
    m = np.max(logits, axis=1, keepdims=True)
    lse = m[:, 0] + np.log(np.sum(np.exp(logits - m), axis=1))
    return float(np.mean(lse - logits[np.arange(len(y)), y]))


def backward(theta, X, y, mu, sigma):
    """Gradient of ``loss`` with respect to the parameter vector."""
    p = unpack(theta)
    logits, (Xn, z1, h1, z2, h2) = forward(theta, X, mu, sigma)
    N = len(y)
    g = softmax(logits)
    g[np.arange(N), y] -= 1.0
    g /= N                                   # dL/dlogits
    d = {}
    d["W3"] = g.T @ h2
    d["b3"] = g.sum(axis=0)
    gh2 = (g @ p["W3"]) * (z2 > 0)
    d["W2"] = gh2.T @ h1
    d["b2"] = gh2.sum(axis=0)
    gh1 = (gh2 @ p["W2"]) * (z1 > 0)
    d["W1"] = gh1.T @ Xn
    d["b1"] = gh1.sum(axis=0)
    return pack(d)


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), bias-corrected, step count t >= 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def predict(theta, X, mu, sigma):
    """Class with the largest logit; ties go to the higher precision (lower
    class index)."""
    logits, _ = forward(theta, X, mu, sigma)
    return np.argmax(logits, axis=1)
