"""Learned-eps path: kappa_2 check and bisection fallback against the oracle,
and what a trained network gains over a constant eps * rho."""
import math

import numpy as np
import pytest
import torch

from oracle.knn import knn as oracle_knn
from oracle.shape import bisect_eps, stencil_kappa
from oracle.weights import build_weights as oracle_weights
from synth import ellipsoid, jittered_torus, torus_grid_for_count

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


@pytest.fixture(scope="module")
def torus():
    X, nrm = jittered_torus(40, 120)
    idx = oracle_knn(X, 50)
    return X, nrm, idx


def test_learned_mode_band_check_and_fallback(lib, torus):
    """Proposals inside [1e11, 1e13] are kept; the others fall back to bisection."""
    X, nrm, idx = torus
    rho = np.sqrt(np.max(np.sum((X[idx] - X[idx[:, :1]]) ** 2, axis=2), axis=1))
    rng = np.random.default_rng(4)
    prop = rng.uniform(0.45, 0.7, size=len(X)) / rho
    res = lib.build_weights(dev(X), dev(nrm), 50, idx=dev(idx, torch.int32), eps_in=dev(prop),
                            eps_mode="learned", kappa_target=1e12, band=(1e11, 1e13))
    torch.cuda.synchronize()
    st, eg, ne = res.status.cpu().numpy(), res.eps.cpu().numpy(), res.nevals.cpu().numpy()
    kg = res.kappa.cpu().numpy()
    assert set(np.unique(st)) <= {0, 1}
    assert 0 < np.mean(st == 1) < 1
    for i in rng.choice(len(X), 80, replace=False):
        k = stencil_kappa(X[idx[i]], prop[i])
        near = min(abs(math.log(k / 1e11)), abs(math.log(k / 1e13))) < 1e-3
        inside = 1e11 < k <= 1e13
        if near:
            continue
        if inside:
            assert st[i] == 0 and eg[i] == prop[i] and ne[i] == 1
            # the kept proposal's kappa_2, searched inside the band's bracket
            assert abs(kg[i] / k - 1.0) <= 20 * k * 2.0 ** -53
        else:
            assert st[i] == 1
            eo, _, _, _ = bisect_eps(X[idx[i]], 1e12)
            assert abs(eg[i] - eo) <= 2e-4


def test_band_stopped_fallback(lib, torus):
    """With band_stop the fallback bisection ends as soon as kappa_2 is inside
    the band: kept proposals are untouched (bit for bit), fallback stencils end
    inside [1e11, 1e13] (oracle kappa_2 at the GPU's eps) after fewer kappa_2
    evaluations than the bisection to the paper's tolerance."""
    X, nrm, idx = torus
    rho = np.sqrt(np.max(np.sum((X[idx] - X[idx[:, :1]]) ** 2, axis=2), axis=1))
    rng = np.random.default_rng(4)
    prop = rng.uniform(0.45, 0.7, size=len(X)) / rho
    args = (dev(X), dev(nrm), 50)
    kw = dict(idx=dev(idx, torch.int32), eps_in=dev(prop), eps_mode="learned", kappa_target=1e12, band=(1e11, 1e13))
    full = lib.build_weights(*args, **kw)
    stop = lib.build_weights(*args, band_stop=True, **kw)
    torch.cuda.synchronize()
    st = stop.status.cpu().numpy()
    assert np.array_equal(st, full.status.cpu().numpy())
    kept, fb = st == 0, st == 1
    assert kept.any() and fb.any()
    for name in ("w", "eps", "kappa", "nevals"):
        a, b = getattr(full, name).cpu().numpy(), getattr(stop, name).cpu().numpy()
        assert np.array_equal(a[kept], b[kept]), name
    ks, ns, nf = stop.kappa.cpu().numpy(), stop.nevals.cpu().numpy(), full.nevals.cpu().numpy()
    assert np.all((ks[fb] > 1e11) & (ks[fb] <= 1e13))
    assert np.mean(ns[fb]) < np.mean(nf[fb])
    es = stop.eps.cpu().numpy()
    rows = rng.choice(np.flatnonzero(fb), min(20, int(fb.sum())), replace=False)
    kap = np.array([stencil_kappa(X[idx[i]], es[i]) for i in rows])
    assert np.all((kap > 1e11 * (1 - 1e-3)) & (kap <= 1e13 * (1 + 1e-3)))
    # the weights are those of the stopping eps (oracle at the GPU's eps,
    # per row within 0.5 kappa u as in the other weight parity tests)
    wo = oracle_weights(X, nrm, idx, es, rows=rows)
    wg = stop.w.cpu().numpy()[rows]
    err = np.linalg.norm(wg - wo, axis=1) / np.linalg.norm(wo, axis=1)
    print(f"[band-stop] max err/(kappa u) = {np.max(err / (kap * 2.0 ** -53)):.4f}", flush=True)
    assert np.all(err <= np.maximum(1e-9, 0.5 * kap * 2.0 ** -53))


def test_kept_proposals_report_kappa_low_band(lib, torus):
    """Well-conditioned band [1e5, 1e7]: proposals at the bisected eps for
    kappa_T = 1e6 are all kept, and their kappa_2 (eigenvalue search stopped at
    band_lo u) matches the oracle's to 20 kappa u."""
    X, nrm, idx = torus
    Xd, Nd, I = dev(X), dev(nrm), dev(idx, torch.int32)
    b = lib.build_weights(Xd, Nd, 50, idx=I, eps_mode="bisect", kappa_target=1e6)
    res = lib.build_weights(Xd, Nd, 50, idx=I, eps_in=b.eps, eps_mode="learned", kappa_target=1e6,
                            band=(1e5, 1e7))
    torch.cuda.synchronize()
    st, kg, eps = res.status.cpu().numpy(), res.kappa.cpu().numpy(), res.eps.cpu().numpy()
    ok = b.status.cpu().numpy() == 0
    assert ok.mean() > 0.99 and np.all(st[ok] == 0)
    assert torch.equal(res.w[torch.as_tensor(ok).cuda()], b.w[torch.as_tensor(ok).cuda()])  # same eps, same weights
    for i in np.random.default_rng(6).choice(np.flatnonzero(ok), 40, replace=False):
        k = stencil_kappa(X[idx[i]], eps[i])
        assert abs(kg[i] / k - 1.0) <= 20 * k * 2.0 ** -53


def test_unusable_predictions_reproduce_bisection_bitwise(lib, torus):
    """Non-finite proposals (a corrupted network) send every stencil to the
    fallback, whose results are bit-identical to plain bisection."""
    X, nrm, idx = torus
    bad = np.full(len(X), np.nan)
    a = lib.build_weights(dev(X), dev(nrm), 50, idx=dev(idx, torch.int32), eps_in=dev(bad), eps_mode="learned")
    b = lib.build_weights(dev(X), dev(nrm), 50, idx=dev(idx, torch.int32), eps_mode="bisect")
    torch.cuda.synchronize()
    assert np.all(a.status.cpu().numpy() == 1)
    assert torch.equal(a.w, b.w) and torch.equal(a.eps, b.eps) and torch.equal(a.kappa, b.kappa)


def test_trained_network_beats_constant_heuristic(lib):
    """Train on blobs and a torus, evaluate on a held-out blob point cloud: the
    network's proposals sit closer to the target condition number than the
    best single eps*rho constant and fall back less often (measured: mean
    |log10 kappa/kappa_T| 0.318 vs 0.342, fallback 1.5% vs 2.7%)."""
    from paper_1404_0812_amd import learned
    from synth import blob

    kT, band = 1e10, (1e9, 1e11)
    feats, labels = [], []
    sets = [blob(30000, seed=41, oversample=2.0), blob(30000, seed=42, oversample=2.0),
            jittered_torus(*torus_grid_for_count(20000, 1.0, 0.3), 1.0, 0.3, seed=7)]
    for X, nrm in sets:
        f, y = learned.label_node_set(X, nrm, 50, kT)
        feats.append(f)
        labels.append(y)
    feats = torch.cat(feats)
    labels = torch.cat(labels)
    net, losses, _ = learned.train(feats, labels, epochs=40, batch=1024, lr=2e-3, seed=3, verbose=False)
    assert torch.isfinite(losses).all()
    Xh, nh = blob(30000, seed=43, oversample=2.0)
    Xd, Nd = dev(Xh), dev(nh)
    idx, _ = lib.knn(Xd, 50)
    eps_l = net.predict_eps(Xd, Nd, idx)
    c = float(torch.exp(labels.mean()).item())
    eps_c = learned.constant_eps(Xd, Nd, idx, c)
    k_l = lib.kappa(Xd, idx, eps_l).cpu().numpy()
    k_c = lib.kappa(Xd, idx, eps_c).cpu().numpy()
    dev_l = np.mean(np.abs(np.log10(k_l / kT)))
    dev_c = np.mean(np.abs(np.log10(k_c / kT)))
    res_l = lib.build_weights(Xd, Nd, 50, idx=idx, eps_in=eps_l, eps_mode="learned", kappa_target=kT, band=band)
    res_c = lib.build_weights(Xd, Nd, 50, idx=idx, eps_in=eps_c, eps_mode="learned", kappa_target=kT, band=band)
    torch.cuda.synchronize()
    fb_l = float((res_l.status == 1).float().mean().item())
    fb_c = float((res_c.status == 1).float().mean().item())
    print(f"mean |log10 kappa/kT|: learned {dev_l:.3f} constant {dev_c:.3f}; fallback {fb_l:.4f} vs {fb_c:.4f}")
    # bars from the recorded measurement (mean deviation 0.318 vs 0.342, ratio
    # 0.93; fallback 1.5% vs 2.7%) with a margin for the run-to-run spread:
    # the tangent-plane inputs leave the curvature of the stencil out, which
    # caps what a network of them can add over one constant eps * rho
    assert dev_l <= 0.97 * dev_c
    assert fb_l < 0.75 * fb_c
    k = res_l.kappa.cpu().numpy()
    assert np.all((k > 0.99 * band[0]) & (k < 1.01 * band[1]))
