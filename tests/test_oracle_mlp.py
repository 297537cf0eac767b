"""Pins of the FP64 MLP oracle: finite differences, BF16 rounding, feature geometry."""
import numpy as np

from oracle import mlp


def rand_params(seed=0):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(mlp.NPARAM) * 0.1
    return p


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = rand_params(1)
    X = rng.uniform(-1, 1, size=(16, mlp.F))
    t = rng.standard_normal(16)
    _, g = mlp.loss_and_grad(p, X, t, quantize=False)
    h = 1e-6
    W1o, b1o, W2o = 0, mlp.H * mlp.F, mlp.H * mlp.F + mlp.H
    picks = list(rng.choice(mlp.NPARAM, 60, replace=False)) + [W1o + 5, b1o + 3, W2o + 77, mlp.NPARAM - 1,
                                                               mlp.NPARAM - 2]
    for k in picks:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        lp, _ = mlp.loss_and_grad(pp, X, t, quantize=False)
        lm, _ = mlp.loss_and_grad(pm, X, t, quantize=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_bf16_round_to_nearest_even():
    one = 1.0
    ulp = 2.0 ** -7
    assert mlp.bf16(one) == one
    assert mlp.bf16(one + ulp / 2) == one                 # tie -> even (1.0)
    assert mlp.bf16(one + 3 * ulp / 2) == one + 2 * ulp   # tie -> even (1 + 2 ulp)
    assert mlp.bf16(one + 0.6 * ulp) == one + ulp
    assert mlp.bf16(-3.0) == -3.0
    assert mlp.bf16(0.0) == 0.0


def test_features_on_a_lattice_and_invariance():
    # planar lattice, normal +z: the nearest neighbour of the centre defines tau_1
    g = np.arange(-2, 3) * 0.5
    P = np.array([[x, y, 0.0] for x in g for y in g])
    c = 12  # (0, 0)
    d2 = np.sum((P - P[c]) ** 2, axis=1)
    order = np.lexsort((np.arange(len(P)), d2))
    idx = order[:9][None, :]
    nrm = np.tile([0.0, 0.0, 1.0], (len(P), 1))
    f, rho = mlp.features(P, nrm, idx)
    assert np.isclose(rho[0], np.sqrt(0.5))
    # first neighbour lies on tau_1: (s, t) = (0.5/rho, 0)
    assert np.isclose(f[0, 0], 0.5 / rho[0]) and abs(f[0, 1]) < 1e-15
    # every offset keeps its length in the tangent plane
    s, t = f[0, 0:16:2], f[0, 1:16:2]
    assert np.allclose(np.hypot(s, t) * rho[0], np.sqrt(d2[idx[0, 1:]]))
    assert np.all(f[0, 16:] == 0.0)
    # rotation + translation + scaling of the cloud leaves the features unchanged
    Q, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((3, 3)))
    f2, rho2 = mlp.features(3.0 * P @ Q.T + 1.0, nrm @ Q.T, idx)
    assert np.allclose(f2, f, atol=1e-12) and np.isclose(rho2[0], 3 * rho[0])
