"""Learned per-stencil shape parameter: labels, training and use.

Labels come from the library's own bisection (Sec. 5, eq. target_cond): for
every stencil of the training node sets, y = log(eps* rho) where eps* is the
bisection root for the target condition number.  The network (BF16 MFMA,
trained by the library's forward/backward/Adam kernels) then proposes eps for
new stencils; rbffd_build_weights in "learned" mode computes kappa_2 at the
proposal and keeps it only inside the acceptance band, bisecting otherwise.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import (MLP, build_weights, default_context, knn, mlp_features, mlp_init)


def label_node_set(X, nrm, n=50, kappa_target=1e12, ctx=None):
    """(features int16 N x 128, labels float32 N) for one node set, on the device."""
    ctx = ctx or default_context()
    Xd = torch.as_tensor(X).cuda() if not isinstance(X, torch.Tensor) else X
    Nd = torch.as_tensor(nrm).cuda() if not isinstance(nrm, torch.Tensor) else nrm
    idx, _ = knn(Xd, n, ctx=ctx)
    res = build_weights(Xd, Nd, n, idx=idx, ctx=ctx, eps_mode="bisect", kappa_target=kappa_target)
    feats, rho = mlp_features(Xd, Nd, idx, ctx=ctx)
    ok = res.status == 0
    y = torch.log(res.eps * rho).to(torch.float32)
    return feats[ok], y[ok]


def train(feats, labels, epochs=20, batch=4096, lr=1e-3, seed=1, ctx=None, verbose=True):
    """Train a fresh network on (feats, labels); returns (MLP, per-step losses, seconds)."""
    ctx = ctx or default_context()
    count = feats.shape[0]
    steps_per_epoch = max(1, count // batch)
    net = MLP(mlp_init(seed=seed, bias_out=float(labels.mean().item())), ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = []
    for e in range(epochs):
        lr_e = lr * (0.5 * (1.0 + math.cos(math.pi * e / epochs)))  # cosine decay per epoch
        l = net.train(feats, labels, steps=steps_per_epoch, batch=batch, lr=lr_e, seed=seed * 1000003 + e + 1)
        losses.append(l)
        if verbose:
            torch.cuda.synchronize()
            print(f"[learned] epoch {e}: batch loss {float(l[-50:].mean().item()):.3e}", flush=True)
    torch.cuda.synchronize()
    return net, torch.cat(losses), time.perf_counter() - t0


def learned_weights(net, Xd, Nd, n, idx, kappa_target=1e12, band=(1e11, 1e13), ctx=None):
    """Weights with eps proposed by `net`, kappa_2-checked, bisection fallback."""
    ctx = ctx or net.ctx
    eps_hat = net.predict_eps(Xd, Nd, idx)
    return build_weights(Xd, Nd, n, idx=idx, eps_in=eps_hat, ctx=ctx, eps_mode="learned",
                         kappa_target=kappa_target, band=band)


def constant_eps(Xd, Nd, idx, c, ctx=None):
    """The single-constant heuristic eps = c / rho (stencil radius rho)."""
    _, rho = mlp_features(Xd, Nd, idx, ctx=ctx)
    return c / rho
