"""FP64 reference of the edge-scoring MLP -- TEST INFRASTRUCTURE.

64 -> 256 -> 256 -> 1 with ReLU, binary cross-entropy with logits, and
Adam.  With ``bf16=True`` the values are rounded to BF16 (nearest, ties to
even) at exactly the points where the GPU path rounds them: the features,
W1, W2, H1 and H2 (after bias + ReLU), dH2 and dH1 (before they enter a
matrix product).  Everything else is float64.  With ``bf16=False`` it is
the plain float64 network, which the finite-difference pins check.

Flat parameter layout: W1[64][256] | b1 | W2[256][256] | b2 | w3 | b3.
"""
from __future__ import annotations

import numpy as np

IN, H = 64, 256
W1, B1 = slice(0, IN * H), slice(IN * H, IN * H + H)
_o = IN * H + H
W2, B2 = slice(_o, _o + H * H), slice(_o + H * H, _o + H * H + H)
_o = _o + H * H + H
W3, B3 = slice(_o, _o + H), slice(_o + H, _o + H + 1)
N_PARAMS = _o + H + 1          # 82,689


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return p[W1].reshape(IN, H), p[B1], p[W2].reshape(H, H), p[B2], p[W3], p[B3][0]


def forward(p, X, bf=True, shift=None, scale=None):
    """shift/scale: optional input standardisation x' = (x - shift) * scale."""
    w1, b1, w2, b2, w3, b3 = unpack(p)
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    if shift is not None:
        X = (X - shift) * scale
    Xb, w1b, w2b = r(X), r(w1), r(w2)
    H1 = r(np.maximum(Xb @ w1b + b1, 0.0))
    H2 = r(np.maximum(H1 @ w2b + b2, 0.0))
    z = H2 @ w3 + b3
    return z, (Xb, w1b, w2b, H1, H2)


def bce(z, y):
    """Mean binary cross-entropy with logits."""
    return float(np.mean(np.log1p(np.exp(-np.abs(z))) + np.maximum(z, 0.0) - z * y))


def grad(p, X, y, bf=True, shift=None, scale=None):
    """Gradient of the mean BCE with respect to the flat parameters, and the loss."""
    w1, b1, w2, b2, w3, b3 = unpack(p)
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    z, (Xb, w1b, w2b, H1, H2) = forward(p, X, bf, shift, scale)
    B = X.shape[0]
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / B
    g = np.zeros(N_PARAMS)
    g[W3] = H2.T @ dz
    g[B3] = dz.sum()
    dH2 = r(np.outer(dz, w3) * (H2 > 0))
    g[W2] = (H1.T @ dH2).ravel()
    g[B2] = dH2.sum(0)
    dH1 = r((dH2 @ w2b.T) * (H1 > 0))
    g[W1] = (Xb.T @ dH1).ravel()
    g[B1] = dH1.sum(0)
    return g, bce(z, y)


def adam(p, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    p = p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return p, m, v
