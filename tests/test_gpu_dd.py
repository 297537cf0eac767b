"""Double-double weights (extended precision, the quad-precision weights of
Sec. 6.2) against 60-digit truth and high-precision kappa_2 / bisection.

Bars, set from the arithmetic: the double-double path carries about
2^-104 relative rounding per operation, amplified by the conditioning, so
weights must sit within max(1e-14, 100 kappa 2^-104) of the 60-digit
weights (relative, per row; the 1e-14 floor covers the final rounding to
FP64); kappa_2 within max(1e-10, 100 kappa 2^-104) relative of the
high-precision eigenvalue kappa_2; eps from the bisection within the paper's
tolerance of the high-precision bisection's (or, where a decision differs,
kappa_2 on the right side of kappa_T at eps -/+ the tolerance).
"""
import time

import numpy as np
import pytest
import torch

from oracle.knn import knn as oracle_knn
from oracle.truth import bisect_eps_mp, stencil_kappa_mp, stencil_weights_mp
from synth import icosahedral_sphere

pytestmark = pytest.mark.gpu
UDD = 2.0 ** -104
KW = dict(kernel="imq", degree=0)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def ico642():
    X, nrm = icosahedral_sphere(3)
    return X, nrm, oracle_knn(X, 17)


@pytest.mark.parametrize("eps", [1.0, 0.08])
def test_dd_weights_fixed_eps_against_truth(lib, ico642, eps):
    """Fixed eps: kappa ~ 1e7 (FP64 resolves it) and ~ 1e16..1e17 (it does not)."""
    X, nrm, idx = ico642
    res = lib.build_weights_dd(dev(X), dev(nrm), 17, idx=dev(idx, torch.int32), eps_mode="fixed", eps=eps, **KW)
    w, k, st = host(res.w), host(res.kappa), host(res.status)
    assert np.all(st == 0)
    worst = 0.0
    for i in (0, 101, 377, 641):
        wt = stencil_weights_mp(X[idx[i]], nrm[idx[i]], eps, degree=0, kernel="imq")
        km = stencil_kappa_mp(X[idx[i]], eps, **KW)
        err = np.linalg.norm(w[i] - wt) / np.linalg.norm(wt)
        worst = max(worst, err)
        assert err <= max(1e-14, 100 * km * UDD), (i, err, km)
        assert abs(k[i] / km - 1.0) <= max(1e-10, 100 * km * UDD), (i, k[i], km)
    print(f"[dd] eps={eps}: kappa ~ {np.median(k):.2e}, max weight error vs 60 digits {worst:.2e}", flush=True)
    if eps == 1.0:  # where FP64 resolves kappa, the FP64 path agrees to its own bar
        r64 = lib.build_weights(dev(X), dev(nrm), 17, idx=dev(idx, torch.int32), eps_mode="fixed", eps=eps, **KW)
        w64 = host(r64.w)
        e64 = np.linalg.norm(w64 - w, axis=1) / np.linalg.norm(w, axis=1)
        assert np.all(e64 <= 0.5 * k * 2.0 ** -53 + 1e-15)


def test_dd_bisection_beyond_fp64(lib, ico642):
    """Bisection to kappa_T = 1e18 (the top of the Sec. 6.1 schedule)."""
    X, nrm, idx = ico642
    kT = 1e18
    t0 = time.perf_counter()
    res = lib.build_weights_dd(dev(X), dev(nrm), 17, idx=dev(idx, torch.int32), eps_mode="bisect", kappa_target=kT,
                               **KW)
    eg, kg, st, w = host(res.eps), host(res.kappa), host(res.status), host(res.w)
    print(f"[dd] N=642 n=17 bisection to 1e18: {time.perf_counter() - t0:.3f} s, kappa median {np.median(kg):.3e}, "
          f"evals {np.median(host(res.nevals))}", flush=True)
    assert np.all(st == 0)
    for i in (5, 300):
        eo, sto = bisect_eps_mp(X[idx[i]], kT, **KW)
        assert sto == 0
        if abs(eg[i] - eo) > 2e-4:
            assert stencil_kappa_mp(X[idx[i]], eg[i] - 1e-4, **KW) > kT > stencil_kappa_mp(X[idx[i]], eg[i] + 1e-4, **KW)
    for i in (5, 300, 600):
        km = stencil_kappa_mp(X[idx[i]], eg[i], **KW)
        assert abs(kg[i] / km - 1.0) <= max(1e-10, 100 * km * UDD)
        assert abs(np.log(km / kT)) < 0.05
        wt = stencil_weights_mp(X[idx[i]], nrm[idx[i]], eg[i], degree=0, kernel="imq")
        err = np.linalg.norm(w[i] - wt) / np.linalg.norm(wt)
        assert err <= max(1e-14, 100 * km * UDD), (i, err, km)


def test_dd_rejects_what_it_does_not_cover(lib, ico642):
    X, nrm, idx = ico642
    with pytest.raises(lib.RbffdError):
        lib.build_weights_dd(dev(X), dev(nrm), 17, idx=dev(idx, torch.int32), eps_mode="fixed", eps=1.0)  # degree 2
    with pytest.raises(lib.RbffdError):
        lib.build_weights_dd(dev(X), dev(nrm), 48, eps_mode="fixed", eps=1.0, **KW)  # n + 1 > 48
