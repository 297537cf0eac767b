"""The allocation-free operator application (rbffd_apply_noalloc) against
rbffd_apply through the C ABI: the same kernels, so the same bits, on two
calls in a row (the second on a smaller operator, which reuses the fixed
array the first left its values in), in FP64 and FP32; an operator larger
than the array is refused in FP64 and still fits in FP32."""
import ctypes

import numpy as np
import pytest
import torch

from oracle.knn import knn as oracle_knn
from oracle.weights import build_weights as oracle_weights
from synth import fibonacci_sphere, real_sph_harm

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def noalloc(lib, op, u, prec):
    ctx = op.ctx
    out = torch.empty_like(u)
    ctx.enter(u, out)
    rc = ctx.lib.rbffd_apply_noalloc(ctx.h, op.h, lib.PRECS[prec], ctypes.c_void_p(u.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()))
    ctx.leave()
    return rc, out


def test_noalloc_apply_matches_apply(lib):
    ops = []
    for N, n in ((2500, 31), (700, 20)):  # second call: a smaller operator
        X, nrm = fibonacci_sphere(N)
        idx = oracle_knn(X, n)
        W = oracle_weights(X, nrm, idx, 3.0)
        _, perm = lib.knn(dev(X), n)
        ops.append((lib.Operator(dev(idx, torch.int32), dev(W), perm=perm), X))
    for prec in ("f64", "f32"):
        for op, X in ops:
            u = dev(real_sph_harm(3, 1, X) + 0.1 * np.cos(3 * X[:, 0]))
            rc, got = noalloc(lib, op, u, prec)
            assert rc == 0, op.ctx.lib.rbffd_last_error(op.ctx.h)
            ref = op.apply(u, prec)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), prec


def test_noalloc_refuses_operators_beyond_the_array(lib):
    N = 4194305  # padded to 4194368 rows: 2 x 8 B x rows > 64 MiB in FP64
    i = np.arange(N, dtype=np.int32)
    idx = np.stack([i, (i + 1) % N], axis=1).astype(np.int32)
    w = np.stack([-np.ones(N), np.ones(N)], axis=1)
    op = lib.Operator(dev(idx, torch.int32), dev(w))
    u = dev(np.sin(np.arange(N) * 1e-3))
    rc, _ = noalloc(lib, op, u, "f64")
    assert rc == lib.RBFFD_E_UNSUPPORTED
    rc, got = noalloc(lib, op, u, "f32")  # 2 x 4 B x rows fits
    assert rc == 0
    ref = op.apply(u, "f32")
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
