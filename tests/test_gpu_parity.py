"""HIP path vs the CPU oracle, element by element on seeded inputs.

Tolerances:
  kNN            bit-exact (stencil lists in (d^2, index) order).
  weights        per row: ||w_gpu - w_ora|| / ||w_ora|| <= max(1e-9, 0.5 kappa u),
                 u = 2^-53, kappa = the oracle's kappa_2 of that stencil.  Two FP64
                 codes of the same weights differ by the conditioning: against a
                 60-digit truth the oracle sits at 0.01-0.06 kappa u (measured),
                 so 0.5 kappa u bounds the sum of both errors.  Well-conditioned
                 stencils (kappa <= 1.8e7) meet the literal 1e-9.
  kappa_2        relative 20 kappa u + 1e-12: the smallest eigenvalue carries an
                 absolute error of a few u ||A~|| in any backward-stable method.
  eps (bisection) |eps_gpu - eps_ora| <= 2 eps_tol: a decision that differs where
                 kappa(mid) ~ kappa_T lands both runs within tol of that mid.
  SpMV FP64      1e-13 relative to sum_j |w_ij u_j| (row-wise).
  RK4 FP64       1e-12 relative L2 of the trajectory end point.
  RK4 FP32       1e-5 relative L2 against the FP64 oracle at the final time.
"""
import math

import numpy as np
import pytest
import torch

from oracle.knn import knn as oracle_knn
from oracle.shape import bisect_eps, stencil_kappa
from oracle.shape import STATUS_NO_BRACKET
from oracle.stepper import assemble, laplacian_apply, rk4
from oracle.weights import build_weights as oracle_weights
from synth import (blob, cached, fibonacci_sphere, jittered_torus, planar_patch, real_sph_harm,
                   random_sph_harm_ic, schnakenberg_ic)

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


WEIGHT_KU = 0.5  # per-row bound in units of kappa u (see the module docstring)


def weight_rule(wg, wo, kap, ku=None):
    err = np.linalg.norm(wg - wo, axis=1) / np.linalg.norm(wo, axis=1)
    tol = np.maximum(1e-9, (WEIGHT_KU if ku is None else ku) * kap * U64)
    print(f"[weights] max err/(kappa u) = {np.max(err / (kap * U64)):.4f} over {len(err)} rows "
          f"(kappa {kap.min():.1e}..{kap.max():.1e})", flush=True)
    return err, tol


def oracle_kappas(X, idx, eps, rows, **kw):
    eps = np.broadcast_to(np.asarray(eps, dtype=float), (len(idx),))
    return np.array([stencil_kappa(X[idx[i]], eps[i], **kw) for i in rows])


# ------------------------------------------------------------------ kNN ----

@pytest.mark.parametrize("case", ["sphere2500_n31", "torus_n50", "blob_n50", "lattice_ties", "all_nodes",
                                  "ellipsoid_n70", "blob_n101", "sphere_n128"])
def test_knn_exact(lib, case):
    if case == "sphere2500_n31":
        X, _ = fibonacci_sphere(2500); n = 31
    elif case == "ellipsoid_n70":
        from synth import ellipsoid
        X, _ = ellipsoid(4000, 1.5, 1.0, 0.6); n = 70
    elif case == "blob_n101":
        X, _ = blob(6000, oversample=2.0); n = 101
    elif case == "sphere_n128":
        X, _ = fibonacci_sphere(3000); n = 128
    elif case == "torus_n50":
        X, _ = jittered_torus(40, 120); n = 50
    elif case == "blob_n50":
        X, _ = blob(3000, oversample=2.0); n = 50
    elif case == "lattice_ties":
        X, _ = planar_patch(23, spacing=0.125); n = 21      # many exact distance ties
    else:
        X, _ = fibonacci_sphere(37); n = 37                   # n = N
    print(f"[knn] case={case} N={len(X)} n={n}", flush=True)
    idx, perm = lib.knn(dev(X), n)
    got = host(idx)
    ref = oracle_knn(X, n)
    assert np.array_equal(got, ref)
    p = host(perm)
    assert np.array_equal(np.sort(p), np.arange(len(X)))


def test_knn_full_size_sampled(lib):
    """N = 1e6 blob, n = 50 (the benchmark workload): sampled rows vs the oracle."""
    X, _ = cached(blob, 1_000_000)
    print("[knn] blob N=1e6 n=50", flush=True)
    idx, _ = lib.knn(dev(X), 50)
    got = host(idx)
    rows = np.random.default_rng(7).choice(len(X), 300, replace=False)
    ref = oracle_knn(X, 50, rows=rows)
    assert np.array_equal(got[rows], ref)
    assert np.all(got[:, 0] == np.arange(len(X)))


# -------------------------------------------------------------- weights ----

@pytest.fixture(scope="module")
def sphere():
    X, nrm = fibonacci_sphere(2500)
    idx = oracle_knn(X, 31)
    return X, nrm, idx


@pytest.mark.parametrize("eps,literal", [(4.0, True), (2.0, False)])
def test_weights_fixed_eps_sphere(lib, sphere, eps, literal):
    X, nrm, idx = sphere
    print(f"[weights] sphere N=2500 n=31 MQ deg2 eps={eps}", flush=True)
    res = lib.build_weights(dev(X), dev(nrm), 31, idx=dev(idx, torch.int32), eps_mode="fixed", eps=eps)
    wg = host(res.w)
    rows = np.arange(0, 2500, 5)
    wo = oracle_weights(X, nrm, idx, eps, rows=rows)
    kap = oracle_kappas(X, idx, eps, rows)
    err, tol = weight_rule(wg[rows], wo, kap)
    if literal:
        assert kap.max() < 1.8e7
        assert err.max() <= 1e-9, err.max()
    assert np.all(err <= tol), (err / tol).max()
    assert np.all(host(res.status) == 0)
    # kappa_2 parity
    kg = host(res.kappa)[rows]
    assert np.all(np.abs(kg / kap - 1.0) <= 20 * kap * U64 + 1e-12), np.abs(kg / kap - 1).max()


@pytest.mark.parametrize("kernel,degree", [("imq", 0), ("mq", 1), ("ga", 2)])
def test_weights_kernels_and_borders(lib, sphere, kernel, degree):
    X, nrm, idx = sphere
    eps = {"imq": 3.0, "mq": 3.0, "ga": 4.0}[kernel]
    print(f"[weights] kernel={kernel} degree={degree} eps={eps}", flush=True)
    res = lib.build_weights(dev(X), dev(nrm), 31, idx=dev(idx, torch.int32), eps_mode="fixed", eps=eps,
                            kernel=kernel, degree=degree)
    wg = host(res.w)
    rows = np.arange(3, 2500, 17)
    wo = oracle_weights(X, nrm, idx, eps, kernel=kernel, degree=degree, rows=rows)
    kap = oracle_kappas(X, idx, eps, rows, kernel=kernel, degree=degree)
    err, tol = weight_rule(wg[rows], wo, kap)
    assert np.all(err <= tol), (err / tol).max()


def test_weights_torus_given_eps_and_ragged(lib):
    """Ragged N (not a multiple of anything), n = 50, per-stencil eps."""
    X, nrm = jittered_torus(37, 111)  # N = 4107
    n = 50
    idx = oracle_knn(X, n)
    rng = np.random.default_rng(11)
    rho = np.sqrt(np.max(np.sum((X[idx] - X[idx[:, :1]]) ** 2, axis=2), axis=1))
    eps = rng.uniform(0.6, 1.0, size=len(X)) / rho
    print(f"[weights] torus N={len(X)} n=50 given eps", flush=True)
    res = lib.build_weights(dev(X), dev(nrm), n, idx=dev(idx, torch.int32), eps_in=dev(eps), eps_mode="given")
    wg = host(res.w)
    rows = np.arange(0, len(X), 13)
    wo = oracle_weights(X, nrm, idx, eps, rows=rows)
    kap = oracle_kappas(X, idx, eps, rows)
    err, tol = weight_rule(wg[rows], wo, kap)
    assert np.all(err <= tol), (err / tol).max()
    assert np.allclose(host(res.eps), eps, rtol=0, atol=0)


def test_bisection_parity_torus(lib):
    X, nrm = jittered_torus(40, 120)
    n = 50
    idx = oracle_knn(X, n)
    print(f"[bisect] torus N={len(X)} n=50 kappa_T=1e12", flush=True)
    res = lib.build_weights(dev(X), dev(nrm), n, idx=dev(idx, torch.int32), eps_mode="bisect", kappa_target=1e12)
    eg, kg, st, ne = host(res.eps), host(res.kappa), host(res.status), host(res.nevals)
    rows = np.random.default_rng(3).choice(len(X), 120, replace=False)
    for i in rows:
        eo, ko, evo, sto = bisect_eps(X[idx[i]], 1e12)
        assert st[i] == sto == 0
        assert abs(eg[i] - eo) <= 2e-4, (i, eg[i], eo)
        assert abs(ne[i] - evo) <= 2
    assert np.all(np.abs(np.log(kg / 1e12)) < 0.05)
    # weights at the GPU's eps vs the oracle at that eps
    wg = host(res.w)
    sub = rows[:40]
    wo = oracle_weights(X, nrm, idx, eg, rows=sub)
    kap = oracle_kappas(X, idx, eg, sub)
    err, tol = weight_rule(wg[sub], wo, kap)
    assert np.all(err <= tol), (err / tol).max()


@pytest.mark.parametrize("n,kernel,degree", [(70, "mq", 2), (101, "mq", 2), (118, "mq", 2), (101, "imq", 0),
                                             (70, "ga", 1)])
def test_large_stencils_four_waves(lib, n, kernel, degree):
    """m = n + border in (64, 128]: four wavefronts per stencil (n = 118 with
    the degree-2 border is the largest system, m = 128).  Bisection to
    kappa_T = 1e10 against the oracle's, then weights at the GPU's eps."""
    X, nrm = fibonacci_sphere(2117)
    idx = oracle_knn(X, n)
    kT = 1e10
    print(f"[weights4] sphere N=2117 n={n} {kernel} degree={degree} bisect kT={kT:g}", flush=True)
    res = lib.build_weights(dev(X), dev(nrm), n, idx=dev(idx, torch.int32), eps_mode="bisect", kappa_target=kT,
                            kernel=kernel, degree=degree)
    eg, kg, st, ne, wg = host(res.eps), host(res.kappa), host(res.status), host(res.nevals), host(res.w)
    rows = np.random.default_rng(n).choice(len(X), 24, replace=False)
    rows[0] = len(X) - 1
    for i in rows:
        eo, ko, evo, sto = bisect_eps(X[idx[i]], kT, kernel=kernel, degree=degree)
        assert st[i] == sto == 0, (i, st[i], sto)
        assert abs(eg[i] - eo) <= 2e-4, (i, eg[i], eo)
        assert abs(ne[i] - evo) <= 2
    wo = oracle_weights(X, nrm, idx, eg, kernel=kernel, degree=degree, rows=rows)
    kap = oracle_kappas(X, idx, eg, rows, kernel=kernel, degree=degree)
    err, tol = weight_rule(wg[rows], wo, kap)
    assert np.all(err <= tol), (err / tol).max()
    assert np.all(np.abs(kg[rows] / kap - 1.0) <= 20 * kap * U64 + 1e-12), np.abs(kg[rows] / kap - 1).max()
    # zero row sums (constants are reproduced) over every stencil
    assert np.all(np.abs(wg.sum(axis=1)) <= 1e-6 * np.abs(wg).sum(axis=1))


def test_weights_without_given_stencils_runs_knn(lib, sphere):
    X, nrm, idx = sphere
    res = lib.build_weights(dev(X), dev(nrm), 31, eps_mode="fixed", eps=4.0)
    assert np.array_equal(host(res.idx), idx)


def test_duplicate_node_flagged(lib):
    X, nrm = fibonacci_sphere(500)
    X = X.copy()
    X[10] = X[11]
    res = lib.build_weights(dev(X), dev(nrm), 20, eps_mode="fixed", eps=3.0)
    st = host(res.status)
    assert st[10] == lib.ST_DUPLICATE and st[11] == lib.ST_DUPLICATE


def test_argument_errors(lib):
    X, nrm = fibonacci_sphere(40)
    with pytest.raises(lib.RbffdError):
        lib.build_weights(dev(X), dev(nrm), 41)          # n > N
    with pytest.raises(lib.RbffdError):
        lib.build_weights(dev(X), dev(nrm), 31, degree=3)
    X2, nrm2 = fibonacci_sphere(200)
    with pytest.raises(lib.RbffdError):
        lib.build_weights(dev(X2), dev(nrm2), 119)       # n + border = 129 > 128
    with pytest.raises(lib.RbffdError):
        lib.build_weights(dev(X2), dev(nrm2), 31, eps_mode="given")   # eps_in missing
    Xe = np.zeros((0, 3))
    r = lib.build_weights(dev(Xe), dev(Xe), 31)          # empty input: nothing to do
    assert r.w.shape == (0, 31)


# -------------------------------------------------------- operator/step ----

@pytest.fixture(scope="module")
def sphere_op(lib, sphere):
    X, nrm, idx = sphere
    W = oracle_weights(X, nrm, idx, 2.0)
    idx_d = dev(idx, torch.int32)
    _, perm = lib.knn(dev(X), 31)
    op = lib.Operator(idx_d, dev(W), perm=perm)
    return X, idx, W, op


def test_spmv_f64(lib, sphere_op):
    X, idx, W, op = sphere_op
    u = np.random.default_rng(1).standard_normal(len(X))
    got = host(op.apply(dev(u), "f64"))
    ref = laplacian_apply(idx, W, u)
    scale = np.sum(np.abs(W * u[idx]), axis=1)
    assert np.all(np.abs(got - ref) <= 1e-13 * scale)


def test_spmv_f32_difference_form(lib, sphere_op):
    X, idx, W, op = sphere_op
    u = real_sph_harm(3, 1, X)
    got = host(op.apply(dev(u), "f32"))
    ref = laplacian_apply(idx, W, u)
    scale = np.sum(np.abs(W), axis=1) * np.abs(u).max()
    assert np.all(np.abs(got - ref) <= 2e-6 * scale)
    # L 1 = 0 exactly in the difference form
    one = host(op.apply(dev(np.ones(len(X))), "f32"))
    assert np.all(one == 0.0)


def test_spmv_f32_halo_and_direct_paths(lib, sphere_op):
    """Spatial order: every slice's neighbourhood fits the LDS halo; a random
    row order: slices read > 640 distinct rows and gather directly.  Both paths
    against the oracle, and bit-equal to each other (same slot order)."""
    X, idx, W, op = sphere_op
    shuffled = np.random.default_rng(8).permutation(len(X))
    op_plain = lib.Operator(dev(idx, torch.int32), dev(W), perm=dev(shuffled, torch.int32))
    ns, hs, _, he = op.stats()
    ns2, hs2, _, _ = op_plain.stats()
    print(f"[halo] spatial order {hs}/{ns} slices staged, mean halo {he / max(hs, 1):.0f}; random order {hs2}/{ns2}",
          flush=True)
    assert hs == ns and hs2 <= 1  # at most the 4-row tail slice fits
    u, _ = random_sph_harm_ic(X, seed=4)
    ref = laplacian_apply(idx, W, u)
    scale = np.sum(np.abs(W), axis=1) * np.abs(u).max()
    a = host(op.apply(dev(u), "f32"))
    b = host(op_plain.apply(dev(u), "f32"))
    assert np.all(np.abs(a - ref) <= 2e-6 * scale)
    assert np.array_equal(a, b)


def test_rk4_f64_heat_sphere(lib, sphere_op):
    """The unit-sphere heat workload: u0 = Y_6^3 + 0.1 Y_2^1, dt = 1e-4, 1000 steps."""
    X, idx, W, op = sphere_op
    u0 = real_sph_harm(6, 3, X) + 0.1 * real_sph_harm(2, 1, X)
    print("[rk4] f64 heat sphere 1000 steps", flush=True)
    got = host(op.step(dev(u0), 1e-4, 1000, prec="f64", graph_steps=50))[0]
    (ref,) = rk4(assemble(idx, W), [u0], [1.0], dt=1e-4, nsteps=1000)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-12
    ue = math.exp(-4.2) * real_sph_harm(6, 3, X) + 0.1 * math.exp(-0.6) * real_sph_harm(2, 1, X)
    assert np.linalg.norm(got - ue) / np.linalg.norm(ue) < 3e-3


def test_rk4_f32_vs_f64_oracle(lib):
    """FP32 state (difference form) against the FP64 oracle at t_final, N = 1e4."""
    X, nrm = fibonacci_sphere(10000)
    idx = oracle_knn(X, 31)
    W = oracle_weights(X, nrm, idx, 4.0)
    u0, _ = random_sph_harm_ic(X)
    u0 = u0.astype(np.float32).astype(np.float64)
    print("[rk4] f32 sphere N=1e4 200 steps", flush=True)
    op = lib.Operator(dev(idx, torch.int32), dev(W))
    dt = 2e-5
    got = host(op.step(dev(u0), dt, 200, prec="f32", graph_steps=40))[0]
    (ref,) = rk4(assemble(idx, W), [u0], [1.0], dt=dt, nsteps=200)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-5


def test_schnakenberg_two_species_f64_and_f32(lib, sphere_op):
    X, idx, W, op = sphere_op
    u0, v0 = schnakenberg_ic(len(X))
    u0 = u0.astype(np.float32).astype(np.float64)
    v0 = v0.astype(np.float32).astype(np.float64)
    prm = {"a": 0.1, "b": 0.9, "gamma": 50.0}
    D = [1.0, 10.0]
    dt, steps = 5e-6, 100
    (ru, rv) = rk4(assemble(idx, W), [u0, v0], D, "schnakenberg", prm, dt=dt, nsteps=steps)
    st = dev(np.stack([u0, v0]))
    g64 = host(op.step(st, dt, steps, prec="f64", D=D, reaction="schnakenberg", params=(0.1, 0.9, 50.0)))
    assert np.linalg.norm(g64[0] - ru) / np.linalg.norm(ru) <= 1e-12
    assert np.linalg.norm(g64[1] - rv) / np.linalg.norm(rv) <= 1e-12
    g32 = host(op.step(st, dt, steps, prec="f32", D=D, reaction="schnakenberg", params=(0.1, 0.9, 50.0)))
    assert np.linalg.norm(g32[0] - ru) / np.linalg.norm(ru) <= 1e-5
    assert np.linalg.norm(g32[1] - rv) / np.linalg.norm(rv) <= 1e-5


def test_turing_two_species_f64_and_f32(lib, sphere_op):
    """The activator-inhibitor kinetics of Sec. 7 (eqs. turing1-2) with the
    spots parameters of Table 1 and delta_u = 0.516 delta_v, from small noise
    around the equilibrium (0, 0)."""
    X, idx, W, op = sphere_op
    rng = np.random.default_rng(12)
    u0 = rng.uniform(-0.01, 0.01, len(X)).astype(np.float32).astype(np.float64)
    v0 = rng.uniform(-0.01, 0.01, len(X)).astype(np.float32).astype(np.float64)
    prm = {"alpha": 0.899, "beta": -0.91, "gamma": -0.899, "tau1": 0.02, "tau2": 0.2}
    params = (0.899, -0.91, -0.899, 0.02, 0.2)
    D = [0.516 * 0.01, 0.01]
    dt, steps = 1e-3, 200
    (ru, rv) = rk4(assemble(idx, W), [u0, v0], D, "turing", prm, dt=dt, nsteps=steps)
    st = dev(np.stack([u0, v0]))
    g64 = host(op.step(st, dt, steps, prec="f64", D=D, reaction="turing", params=params))
    assert np.linalg.norm(g64[0] - ru) / np.linalg.norm(ru) <= 1e-12
    assert np.linalg.norm(g64[1] - rv) / np.linalg.norm(rv) <= 1e-12
    g32 = host(op.step(st, dt, steps, prec="f32", D=D, reaction="turing", params=params))
    assert np.linalg.norm(g32[0] - ru) / np.linalg.norm(ru) <= 1e-5
    assert np.linalg.norm(g32[1] - rv) / np.linalg.norm(rv) <= 1e-5


def test_graph_replay_matches_eager(lib, sphere_op):
    X, idx, W, op = sphere_op
    u0 = real_sph_harm(4, 2, X)
    a = host(op.step(dev(u0), 1e-4, 120, prec="f64", graph_steps=1000))   # 120 < 1000: all eager
    b = host(op.step(dev(u0), 1e-4, 120, prec="f64", graph_steps=30))     # 4 graph replays
    c = host(op.step(dev(u0), 1e-4, 120, prec="f64", graph_steps=30))     # cached graph
    assert np.array_equal(a, b) and np.array_equal(b, c)


@pytest.mark.slow
def test_weights_against_60_digit_truth(lib, sphere):
    """GPU and oracle against 60-digit weights of the same stencils (kappa ~ 1e10):
    the GPU error stays within max(2x the oracle's error, 0.1 kappa u)."""
    from oracle.truth import stencil_weights_mp

    X, nrm, idx = sphere
    eps = 2.0
    res = lib.build_weights(dev(X), dev(nrm), 31, idx=dev(idx, torch.int32), eps_mode="fixed", eps=eps)
    wg = host(res.w)
    for i in (0, 70, 1325, 1680, 2030, 2499):
        s = idx[i]
        wt = stencil_weights_mp(X[s], nrm[s], eps)
        wo = oracle_weights(X, nrm, idx, eps, rows=[i])[0]
        k = stencil_kappa(X[s], eps)
        nt = np.linalg.norm(wt)
        eg = np.linalg.norm(wg[i] - wt) / nt
        eo = np.linalg.norm(wo - wt) / nt
        assert eg <= max(2 * eo, 0.1 * k * U64) + 1e-12, (i, eg / (k * U64), eo / (k * U64))


def test_out_of_range_indices_are_flagged(lib, sphere):
    """Stencil entries outside [0, N) are caught on the device: the weights
    call marks that stencil (status 6, NaN weights) and leaves the others
    alone; the operator build refuses the stencils and a non-permutation."""
    X, nrm, idx = sphere
    bad = idx.copy()
    bad[7, 3] = len(X) + 5
    bad[9, 0] = -1
    ref = lib.build_weights(dev(X), dev(nrm), 31, idx=dev(idx, torch.int32), eps_mode="fixed", eps=4.0)
    got = lib.build_weights(dev(X), dev(nrm), 31, idx=dev(bad, torch.int32), eps_mode="fixed", eps=4.0)
    st = host(got.status)
    assert st[7] == lib.ST_BAD_INDEX and st[9] == lib.ST_BAD_INDEX
    w = host(got.w)
    assert np.all(np.isnan(w[7])) and np.all(np.isnan(w[9]))
    keep = np.setdiff1d(np.arange(len(X)), [7, 9])
    assert np.array_equal(w[keep], host(ref.w)[keep]) and np.all(st[keep] == 0)
    with pytest.raises(lib.RbffdError):
        lib.Operator(dev(bad, torch.int32), ref.w)
    perm = np.arange(len(X), dtype=np.int32)
    perm[5] = 6  # 5 is never reached
    with pytest.raises(lib.RbffdError):
        lib.Operator(dev(idx, torch.int32), ref.w, perm=dev(perm, torch.int32))


def test_zero_normal_flagged(lib, sphere):
    """A zero or non-finite normal leaves Pi_i = I - nu nu^T undefined
    (Sec. 3): every stencil holding that node gets status 7 and NaN outputs;
    all other stencils are unchanged bit for bit."""
    X, nrm, idx = sphere
    bad = nrm.copy()
    bad[100] = 0.0
    bad[200, 1] = np.nan
    ref = lib.build_weights(dev(X), dev(nrm), 31, idx=dev(idx, torch.int32), eps_mode="fixed", eps=4.0)
    got = lib.build_weights(dev(X), dev(bad), 31, idx=dev(idx, torch.int32), eps_mode="fixed", eps=4.0)
    st = host(got.status)
    hit = np.any((idx == 100) | (idx == 200), axis=1)
    assert hit.sum() >= 60
    assert np.all(st[hit] == lib.ST_BAD_NORMAL) and np.all(st[~hit] == 0)
    w = host(got.w)
    assert np.all(np.isnan(w[hit])) and np.all(np.isnan(host(got.eps)[hit]))
    assert np.array_equal(w[~hit], host(ref.w)[~hit])


def test_unreachable_target_gives_no_bracket(lib):
    """kappa_T below what any eps reaches on the stencil: the bracket cannot
    be formed (status 2, as the oracle's bisection reports), weights still finite."""
    X, nrm = fibonacci_sphere(800)
    idx = oracle_knn(X, 31)
    res = lib.build_weights(dev(X), dev(nrm), 31, idx=dev(idx, torch.int32), eps_mode="bisect",
                            kappa_target=2.0, max_expand=2)
    st = host(res.status)
    assert np.all(st == lib.ST_NO_BRACKET)
    for i in (0, 400, 799):
        _, _, _, sto = bisect_eps(X[idx[i]], 2.0, max_expand=2)
        assert sto == STATUS_NO_BRACKET
    assert np.all(np.isfinite(host(res.w)))


def test_step_reports_nonfinite_state(lib, sphere_op):
    """A step far beyond the RK4 stability limit overflows the state: the call
    fails with the non-finite error instead of returning Inf/NaN silently; a
    stable call on the same operator afterwards succeeds."""
    X, idx, W, op = sphere_op
    u0 = real_sph_harm(4, 2, X)
    for prec in ("f64", "f32"):
        with pytest.raises(lib.RbffdError, match="non-finite"):
            op.step(dev(u0), 1.0, 400, prec=prec, graph_steps=20)
    nan0 = u0.copy()
    nan0[5] = np.nan
    with pytest.raises(lib.RbffdError, match="non-finite"):
        op.step(dev(nan0), 1e-4, 3, prec="f64", graph_steps=50)  # eager steps only
    ok = host(op.step(dev(u0), 1e-4, 100, prec="f64", graph_steps=20))
    assert np.all(np.isfinite(ok))


def test_operator_requires_centre_in_slot0(lib, sphere_op):
    """The FP32 difference form drops slot 0, so a row whose slot 0 is not
    the row itself is refused at build time."""
    X, idx, W, _ = sphere_op
    sw = idx.copy()
    sw[17, [0, 1]] = sw[17, [1, 0]]
    with pytest.raises(lib.RbffdError):
        lib.Operator(dev(sw, torch.int32), dev(W))
    lib.Operator(dev(idx, torch.int32), dev(W))  # the unswapped rows build


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_forced_step_matches_oracle(lib, sphere_op, prec, tol):
    """du/dt = L u + exp(lam t) F (eq. diffusion_scalar with the separable
    forcing of Sec. 6) from t0 = 0.3: the GPU run against the oracle's forced
    RK4, graph replays plus an eager tail."""
    X, idx, W, op = sphere_op
    rng = np.random.default_rng(21)
    u0 = real_sph_harm(5, -2, X).astype(np.float32).astype(np.float64)
    F = rng.standard_normal(len(X))
    dt, steps, t0, lam = 1e-4, 130, 0.3, -5.0
    (ref,) = rk4(assemble(idx, W), [u0], [1.0], dt=dt, nsteps=steps, t0=t0, forcing=(lam, [F]))
    got = host(op.step(dev(u0), dt, steps, prec=prec, graph_steps=40, forcing=dev(F[None, :]), t0=t0, lam=lam))[0]
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= tol
    # the forcing matters at this size: the unforced run is far away
    (free,) = rk4(assemble(idx, W), [u0], [1.0], dt=dt, nsteps=steps)
    assert np.linalg.norm(free - ref) / np.linalg.norm(ref) > 100 * tol
    # two species with kinetics and forcing on both
    v0 = schnakenberg_ic(len(X))
    s0 = np.stack(v0).astype(np.float32).astype(np.float64)
    F2 = 0.1 * rng.standard_normal((2, len(X)))
    prm = {"a": 0.1, "b": 0.9, "gamma": 50.0}
    (ru, rv) = rk4(assemble(idx, W), [s0[0], s0[1]], [1.0, 10.0], "schnakenberg", prm, dt=5e-6, nsteps=90, t0=t0,
                   forcing=(lam, [F2[0], F2[1]]))
    g = host(op.step(dev(s0), 5e-6, 90, prec=prec, D=(1.0, 10.0), reaction="schnakenberg", params=(0.1, 0.9, 50.0),
                     graph_steps=40, forcing=dev(F2), t0=t0, lam=lam))
    assert np.linalg.norm(g[0] - ru) / np.linalg.norm(ru) <= tol
    assert np.linalg.norm(g[1] - rv) / np.linalg.norm(rv) <= tol
