"""FP64 forward/backward of the shape-parameter regressor (test infrastructure).

Network: x (128) -> h1 = relu(W1 x + b1) (128) -> h2 = relu(W2 h1 + b2) (128)
-> y = w3 . h2 + b3, trained on the mean squared error against
y* = log(eps* rho), eps* from the bisection of Sec. 5.  Parameter vector
layout: W1 (128 x 128, out x in), b1, W2, b2, w3, b3.

With quantize=True the values are rounded to BF16 (round to nearest even,
from FP32) at the points where the GPU kernels hold them in BF16: inputs,
the W1 and W2 copies, h1, h2, dL/dh2 and dL/dh1.  Everything else is FP64.
With quantize=False this is the plain network, whose gradient is checked
against central differences.

Features: offsets x_j - x_1 (j = 2..n) in the tangent frame tau_1 ~ the
projection of x_2 - x_1 on the tangent plane at x_1, tau_2 = nu x tau_1,
divided by rho = max_j |x_j - x_1|, interleaved (s_2, t_2, s_3, t_3, ...) and
zero-padded to 128.
"""
from __future__ import annotations

import numpy as np

F = 128
H = 128
NPARAM = H * F + H + H * H + H + H + 1


def bf16(a):
    """Round to BF16 (via FP32, round to nearest even); returns float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * F].reshape(H, F); o += H * F
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def forward(p, X, quantize=True):
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = q(X)
    a1 = X @ q(W1).T + b1
    h1 = q(np.maximum(a1, 0.0))
    a2 = h1 @ q(W2).T + b2
    h2 = q(np.maximum(a2, 0.0))
    y = h2 @ w3 + b3
    return y, (X, a1, h1, a2, h2)


def loss_and_grad(p, X, t, quantize=True):
    """Mean squared error and its gradient (backpropagation written out)."""
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, w3, b3 = unpack(p)
    y, (Xq, a1, h1, a2, h2) = forward(p, X, quantize)
    B = len(t)
    e = y - t
    loss = float(np.mean(e * e))
    dy = 2.0 * e / B
    gw3 = h2.T @ dy
    gb3 = dy.sum()
    dh2 = q(np.outer(dy, w3) * (a2 > 0))
    gb2 = dh2.sum(axis=0)
    gW2 = dh2.T @ h1
    dh1 = q((dh2 @ q(W2)) * (a1 > 0))
    gb1 = dh1.sum(axis=0)
    gW1 = dh1.T @ Xq
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, [gb3]])
    return loss, g


def features(X, nrm, idx):
    """Tangent-frame offset features (N x 128, FP64, not rounded) and rho."""
    N, n = idx.shape
    out = np.zeros((N, F))
    rho = np.zeros(N)
    for s in range(N):
        c = idx[s, 0]
        d = X[idx[s]] - X[c]
        r = np.sqrt(np.max(np.sum(d * d, axis=1)))
        nu = nrm[c] / np.linalg.norm(nrm[c])
        t1 = d[1] - (d[1] @ nu) * nu
        if np.linalg.norm(t1) <= 1e-12 * r:
            t1 = np.array([0.0, nu[2], -nu[1]]) if abs(nu[0]) < 0.9 else np.array([-nu[2], 0.0, nu[0]])
        t1 = t1 / np.linalg.norm(t1)
        t2 = np.cross(nu, t1)
        out[s, 0:2 * (n - 1):2] = (d[1:] @ t1) / r
        out[s, 1:2 * (n - 1):2] = (d[1:] @ t2) / r
        rho[s] = r
    return out, rho
