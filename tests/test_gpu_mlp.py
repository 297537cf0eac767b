"""BF16-MFMA network kernels vs the FP64 oracle with the same BF16 rounding points.

Tolerances: features within one BF16 ulp (both sides round an FP64 value);
forward outputs and per-tensor gradients within 1e-2 relative (FP32
accumulation on the GPU vs FP64 in the oracle, plus rare one-ulp BF16
flips of activations near a rounding boundary).
"""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from oracle.knn import knn as oracle_knn
from synth import blob, jittered_torus

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def bf16_to_f64(t):
    torch.cuda.synchronize()
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def bf16_bits(a):
    return (np.asarray(omlp.bf16(a), dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)


# N = 2999 and 1001 leave the last wavefront of four stencils partly empty;
# n = 64 uses every lane of the wavefront (its largest stencil)
@pytest.mark.parametrize("N,n", [(3000, 50), (2999, 50), (1001, 64)])
def test_features_match_oracle(lib, N, n):
    X, nrm = blob(3000, oversample=2.0)
    X, nrm = X[:N], nrm[:N]
    idx = oracle_knn(X, n)
    f, rho = lib.mlp_features(dev(X), dev(nrm), dev(idx, torch.int32))
    got = bf16_to_f64(f)
    ref, rref = omlp.features(X, nrm, idx)
    refq = omlp.bf16(ref)
    # one BF16 ulp, with an absolute floor for entries that vanish by construction
    # (the second coordinate of the nearest neighbour is 0 up to FP64 rounding)
    ulp = np.maximum(np.abs(refq) * 2.0 ** -7, 1e-12)
    assert np.all(np.abs(got - refq) <= ulp)
    big = np.abs(refq) > 1e-12
    assert np.mean(got[big] != refq[big]) < 1e-3
    assert np.allclose(rho.cpu().numpy(), rref, rtol=1e-15)


def test_features_reject_stencils_wider_than_a_wavefront(lib):
    X, nrm = blob(3000, oversample=2.0)
    idx = oracle_knn(X[:500], 65)
    with pytest.raises(lib.RbffdError, match="n <= 64"):
        lib.mlp_features(dev(X[:500]), dev(nrm[:500]), dev(idx, torch.int32))


@pytest.fixture(scope="module")
def batch():
    rng = np.random.default_rng(5)
    B = 320  # five 64-sample tiles
    X = omlp.bf16(rng.uniform(-1, 1, size=(B, omlp.F)))
    X[:, 98:] = 0.0
    t = rng.normal(-0.6, 0.2, size=B)
    p = rng.standard_normal(omlp.NPARAM) * 0.08
    p = p.astype(np.float32).astype(np.float64)
    return X, t, p


def to_bits(X):
    return torch.as_tensor(bf16_bits(X).view(np.int16)).cuda()


def test_forward_matches_oracle(lib, batch):
    X, t, p = batch
    y = lib.mlp_forward(dev(p, torch.float32), to_bits(X))
    torch.cuda.synchronize()
    yg = y.cpu().numpy().astype(np.float64)
    yo, _ = omlp.forward(p, X, quantize=True)
    assert np.linalg.norm(yg - yo) / np.linalg.norm(yo) < 1e-3


def test_ragged_batch_forward(lib, batch):
    X, t, p = batch
    Xr = X[:77]
    y = lib.mlp_forward(dev(p, torch.float32), to_bits(Xr))
    torch.cuda.synchronize()
    yo, _ = omlp.forward(p, Xr, quantize=True)
    assert np.linalg.norm(y.cpu().numpy() - yo) / np.linalg.norm(yo) < 1e-3


def test_gradient_matches_oracle(lib, batch):
    X, t, p = batch
    g, loss = lib.mlp_grad(dev(p, torch.float32), to_bits(X), dev(t, torch.float32))
    torch.cuda.synchronize()
    gg = g.cpu().numpy().astype(np.float64)
    lo, go = omlp.loss_and_grad(p, X, t, quantize=True)
    assert abs(loss.item() - lo) / lo < 1e-3
    H, F = omlp.H, omlp.F
    parts = {"W1": slice(0, H * F), "b1": slice(H * F, H * F + H), "W2": slice(H * F + H, H * F + H + H * H),
             "b2": slice(H * F + H + H * H, H * F + 2 * H + H * H), "w3": slice(H * F + 2 * H + H * H, -1),
             "b3": slice(-1, None)}
    for name, sl in parts.items():
        ref = go[sl]
        err = np.linalg.norm(gg[sl] - ref) / max(np.linalg.norm(ref), 1e-30)
        assert err < 1e-2, (name, err)


def test_training_reduces_loss(lib, batch):
    X, t, p0 = batch
    rng = np.random.default_rng(9)
    Xs = omlp.bf16(rng.uniform(-1, 1, size=(4096, omlp.F)))
    Xs[:, 98:] = 0
    w = rng.standard_normal(98) / 10
    ts = np.tanh(Xs[:, :98] @ w) - 0.6  # a smooth target the network can fit
    net = lib.MLP(lib.mlp_init(seed=3, bias_out=-0.6))
    feats = to_bits(Xs)
    tgt = dev(ts, torch.float32)
    y0 = net.forward(feats).cpu().numpy()
    losses = net.train(feats, tgt, steps=300, batch=512, lr=2e-3, seed=11)
    torch.cuda.synchronize()
    l = losses.cpu().numpy()
    y1 = net.forward(feats).cpu().numpy()
    m0 = np.mean((y0 - ts) ** 2)
    m1 = np.mean((y1 - ts) ** 2)
    assert np.all(np.isfinite(l))
    assert m1 < 0.2 * m0, (m0, m1)
    assert l[-20:].mean() < l[:20].mean()
