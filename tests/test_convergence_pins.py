"""CPU pins of the pieces of the paper's convergence suite (Sec. 6.1):
the node sets, the manufactured solutions and their forcing, and the forced
RK4 of the oracle.

None of these re-types a formula under test: the analytic surface Laplacians
of the manufactured solutions are checked against finite differences of the
Laplace-Beltrami operator built numerically from each surface's
parametrisation, and the forced RK4 against the exact solution of a scalar
linear ODE.
"""
import math

import numpy as np
import pytest

from oracle.knn import knn
from oracle.stepper import assemble, rk4
from oracle.weights import build_weights
from synth import (bump_centres, icosahedral_sphere, real_sph_harm, sphere_forced, sphere_heat_series,
                   staggered_torus, torus_angles, torus_forced)


# ---------------------------------------------------------------- nodes ----

@pytest.mark.parametrize("level,N", [(0, 12), (1, 42), (3, 642), (4, 2562)])
def test_icosahedral_counts_and_spacing(level, N):
    """Sec. 6.1 uses N = 642, 2562, 10242, 40962 icosahedral nodes: 10 4^k + 2."""
    X, nrm = icosahedral_sphere(level)
    assert len(X) == N == 10 * 4 ** level + 2
    assert np.allclose(np.linalg.norm(X, axis=1), 1.0, atol=1e-15)
    assert np.array_equal(X, nrm)
    idx = knn(X, 2)
    d = np.linalg.norm(X[idx[:, 1]] - X, axis=1)
    assert d.min() > 0.0                 # no duplicates
    assert d.max() / d.min() < 1.3       # quasi-uniform (nearest-neighbour spacing)


@pytest.mark.parametrize("m", [10, 20])
def test_staggered_torus(m):
    """Sec. 6.1: N = 6 m^2 nodes on (1 - sqrt(x^2 + y^2))^2 + z^2 = 1/9,
    the second grid at the cell midpoints of the first."""
    X, nrm = staggered_torus(m)
    assert len(X) == 6 * m * m
    f = (1.0 - np.hypot(X[:, 0], X[:, 1])) ** 2 + X[:, 2] ** 2 - 1.0 / 9.0
    assert np.max(np.abs(f)) < 1e-15
    assert np.allclose(np.linalg.norm(nrm, axis=1), 1.0)
    # the normal is the normalised gradient of the implicit function
    s = np.hypot(X[:, 0], X[:, 1])
    grad = np.stack([-2 * (1 - s) * X[:, 0] / s, -2 * (1 - s) * X[:, 1] / s, 2 * X[:, 2]], axis=1)
    grad /= np.linalg.norm(grad, axis=1, keepdims=True)
    assert np.allclose(grad, nrm, atol=1e-12)
    phi, lam = torus_angles(X)
    half = 3 * m * m
    assert np.allclose(phi[half:] - phi[:half], math.pi / m, atol=1e-12) or \
        np.allclose(np.mod(phi[half:] - phi[:half] + math.pi, 2 * math.pi) - math.pi, math.pi / m, atol=1e-12)
    assert len(np.unique(np.round(X, 12), axis=0)) == len(X)


# ---------------------------------------------- manufactured solutions ----

def _lb_fd(embed, fun, p, q, h=1e-4):
    """Laplace-Beltrami of fun(embed(p, q)) at coordinates (p, q) by central
    differences, with the metric of the parametrisation `embed` also taken by
    central differences: (1/sqrt g) d_i (sqrt g g^{ij} d_j f)."""
    def metric(p, q):
        xp = (embed(p + h, q) - embed(p - h, q)) / (2 * h)
        xq = (embed(p, q + h) - embed(p, q - h)) / (2 * h)
        G = np.array([[xp @ xp, xp @ xq], [xq @ xp, xq @ xq]])
        return G

    def flux(p, q, i):
        G = metric(p, q)
        sg = math.sqrt(np.linalg.det(G))
        Gi = np.linalg.inv(G)
        fp = (fun(embed(p + h, q)) - fun(embed(p - h, q))) / (2 * h)
        fq = (fun(embed(p, q + h)) - fun(embed(p, q - h))) / (2 * h)
        return sg * (Gi[i, 0] * fp + Gi[i, 1] * fq)

    H = 1e-3
    d = ((flux(p + H, q, 0) - flux(p - H, q, 0)) / (2 * H) + (flux(p, q + H, 1) - flux(p, q - H, 1)) / (2 * H))
    return d / math.sqrt(np.linalg.det(metric(p, q)))


def test_sphere_forcing_is_the_manufactured_laplacian():
    """F = -5 g - Lap_S g for eq. sph_forced (reading: bumps exp(-10 (1 - xi.x)))."""
    cen = bump_centres("sphere")
    assert cen.shape == (23, 3)

    def embed(th, ph):
        return np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])

    rng = np.random.default_rng(3)
    for _ in range(12):
        th, ph = rng.uniform(0.3, 2.8), rng.uniform(-3, 3)
        x = embed(th, ph)
        g, F = sphere_forced(x[None, :], cen)
        lap = _lb_fd(embed, lambda y: sphere_forced(y[None, :], cen)[0][0], th, ph)
        assert abs((-5 * g[0] - F[0]) - lap) < 2e-4 * (1 + abs(lap)), (lap, -5 * g[0] - F[0])


def test_torus_forcing_is_the_manufactured_laplacian():
    """F = -5 g - Lap g for eq. torus_forced on the torus of eq. torus; the
    Laplacian is checked against the metric of the parametrisation itself."""
    cen = bump_centres("torus")
    assert cen.shape == (23, 2)

    def embed(p, l):
        c = 1.0 + math.cos(p) / 3.0
        return np.array([c * math.cos(l), c * math.sin(l), math.sin(p) / 3.0])

    def g_of(y):
        ph, la = torus_angles(y[None, :])
        return torus_forced(ph, la, cen)[0][0]

    rng = np.random.default_rng(4)
    for _ in range(12):
        p, l = rng.uniform(-3, 3), rng.uniform(-3, 3)
        x = embed(p, l)
        ph, la = torus_angles(x[None, :])
        assert abs(ph[0] - p) < 1e-12 and abs(la[0] - l) < 1e-12
        g, F = torus_forced(ph, la, cen)
        lap = _lb_fd(embed, g_of, p, l)
        assert abs((-5 * g[0] - F[0]) - lap) < 2e-4 * (1 + abs(lap)), (lap, -5 * g[0] - F[0])


def test_heat_series_solves_the_heat_equation():
    """Sec. 6.1 heat series: u_t = Lap_S u, checked by differences in t and
    on the sphere's parametrisation; at t -> infinity the l = 1 term leads."""
    def embed(th, ph):
        return np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])

    rng = np.random.default_rng(5)
    t, dt = 0.05, 1e-5
    for _ in range(6):
        th, ph = rng.uniform(0.4, 2.7), rng.uniform(-3, 3)
        x = embed(th, ph)[None, :]
        ut = (sphere_heat_series(x, t + dt)[0] - sphere_heat_series(x, t - dt)[0]) / (2 * dt)
        lap = _lb_fd(embed, lambda y: sphere_heat_series(y[None, :], t)[0], th, ph)
        assert abs(ut - lap) < 2e-4 * (1 + abs(ut)), (ut, lap)
    x = embed(1.0, 0.5)[None, :]
    lead = 20 / (3 * math.pi) * math.exp(-1 / 9) * math.exp(-2 * 3.0) * real_sph_harm(1, 1, x)[0]
    assert abs(sphere_heat_series(x, 3.0)[0] - lead) < 1e-5 * abs(lead)  # next term ~ e^{-12} smaller


# ---------------------------------------------------------- forced RK4 ----

def test_forced_rk4_matches_scalar_ode():
    """u' = a u + exp(lam t) F from t0: exact u(t) = e^{a (t - t0)} u0 +
    F (e^{lam t} - e^{a (t - t0) + lam t0}) / (lam - a).  RK4's global error
    is O(dt^4); a forcing taken at the wrong stage time leaves O(dt^2)."""
    a, lam, F, u0, t0 = -3.0, -5.0, 2.0, 0.7, 0.3
    L = assemble(np.array([[0]]), np.array([[a]]))
    for dt, tol in ((1e-2, 2e-9), (1e-3, 2e-13)):
        n = int(round(1.0 / dt))
        (u,) = rk4(L, [np.array([u0])], [1.0], dt=dt, nsteps=n, t0=t0, forcing=(lam, [np.array([F])]))
        t = t0 + n * dt
        ex = math.exp(a * (t - t0)) * u0 + F * (math.exp(lam * t) - math.exp(a * (t - t0) + lam * t0)) / (lam - a)
        assert abs(u[0] - ex) < tol, (dt, u[0] - ex)


def test_forced_sphere_tracks_manufactured_harmonic():
    """u = exp(-5t) Y_3^2 solves u_t = Lap_S u + f with f = exp(-5t) (12 - 5) Y_3^2
    (Lap_S Y_3^2 = -12 Y_3^2): the oracle's forced run stays on it to the
    discretisation error, and drifts off by far more without the forcing."""
    errs = []
    for level, eps in ((3, 3.0), (4, 6.0)):  # eps ~ sqrt(N): the same eps h on both
        X, nrm = icosahedral_sphere(level)
        idx = knn(X, 31)
        L = assemble(idx, build_weights(X, nrm, idx, eps))
        Y = real_sph_harm(3, 2, X)
        (u,) = rk4(L, [Y], [1.0], dt=1e-4, nsteps=500, forcing=(-5.0, [7.0 * Y]))
        ex = math.exp(-0.25) * Y
        errs.append(np.linalg.norm(u - ex) / np.linalg.norm(ex))
    (v,) = rk4(L, [Y], [1.0], dt=1e-4, nsteps=500)
    e_free = np.linalg.norm(v - ex) / np.linalg.norm(ex)
    assert errs[0] < 1e-2 and errs[1] < 0.5 * errs[0] and e_free > 0.2, (errs, e_free)


# ------------------------------------------------------------ IMEX BDF ----

from oracle.stepper import BDF_COEFFS, imex_bdf  # noqa: E402


def test_bdf_coefficients_are_consistent():
    """Each BDF row annihilates polynomials of degree <= k on the unit grid
    (order k) and each extrapolation row reproduces them at the new point."""
    for k, (a, b) in BDF_COEFFS.items():
        for p in range(k + 1):
            # sum_j a_j (1 - j)^p = d/dt t^p at t = 1 (times dt = 1) = p
            lhs = sum(a[j] * (1.0 - j) ** p for j in range(k + 1))
            assert abs(lhs - (p if p > 0 else 0.0)) < 1e-12, (k, p)
        for p in range(k):  # k past values extrapolate degree k - 1 exactly
            ext = sum(b[j - 1] * (1.0 - j) ** p for j in range(1, k + 1))
            assert abs(ext - 1.0) < 1e-12, (k, p)
        # and not degree k (the row is not padded with spurious accuracy)
        assert abs(sum(b[j - 1] * (1.0 - j) ** k for j in range(1, k + 1)) - 1.0) > 1e-3


def _forced_exact(t, a=-3.0, lam=-5.0, F=2.0, u0=0.7, t0=0.3):
    return math.exp(a * (t - t0)) * u0 + F * (math.exp(lam * t) - math.exp(a * (t - t0) + lam * t0)) / (lam - a)


@pytest.mark.parametrize("order", [1, 2, 3, 4])
@pytest.mark.parametrize("start", ["exact", "lower"])
def test_imex_bdf_order_on_forced_linear_ode(order, start):
    """u' = a u + exp(lam t) F (diffusion-like implicit term, implicit forcing):
    the global error at t0 + 1 falls as dt^order when the history comes from
    the exact solution (as the paper starts BDF4).  Started with the lower
    orders instead, the BDF1 first step's O(dt^2) error caps the order at 2."""
    a, lam, F, u0, t0 = -3.0, -5.0, 2.0, 0.7, 0.3
    L = assemble(np.array([[0]]), np.array([[a]]))
    errs = []
    for n in (40, 80, 160):
        dt = 1.0 / n
        hist = [[np.array([_forced_exact(t0 - j * dt)])] for j in range(1, order)] if start == "exact" else None
        (u,) = imex_bdf(L, [np.array([u0])], [1.0], dt=dt, nsteps=n, order=order, t0=t0,
                        forcing=(lam, [np.array([F])]), history=hist)
        errs.append(abs(u[0] - _forced_exact(t0 + 1.0)))
    rates = [math.log2(errs[j] / errs[j + 1]) for j in range(2)]
    want = order if start == "exact" else min(order, 2)
    assert min(rates) > want - 0.35, (order, errs, rates)


@pytest.mark.parametrize("order", [1, 2])
def test_imex_bdf_order_on_explicit_reaction(order):
    """u' = -u^2 (explicit, extrapolated reaction only): exact u = u0 / (1 + u0 t)."""
    L = assemble(np.array([[0, 1]]), np.array([[0.0, 0.0]]), N=2)[:1, :1]
    prm = None
    errs = []
    for n in (50, 100, 200):
        dt = 1.0 / n
        # the Schnakenberg kinetics with a = b = 0 and gamma = 1 give R_u = -u + u^2 v;
        # with v = 0 frozen (R_v = -u^2 v = 0) this is u' = -u
        (u, v) = imex_bdf(L, [np.array([0.8]), np.array([0.0])], [0.0, 0.0], "schnakenberg",
                          {"a": 0.0, "b": 0.0, "gamma": 1.0}, dt=dt, nsteps=n, order=order)
        errs.append(abs(u[0] - 0.8 * math.exp(-1.0)))
        assert v[0] == 0.0
    rates = [math.log2(errs[j] / errs[j + 1]) for j in range(2)]
    assert min(rates) > order - 0.2, (order, errs, rates)


def _turing_linear_case(l, m):
    """Small Y_l^m perturbation of (0, 0) on the unit sphere (icosahedral
    nodes, N = 2562, n = 31, MQ with the degree-2 border at eps = 2) for the
    Turing system with Table 1's spots kinetics and delta_v = 4.5e-3
    (delta_u = 0.516 delta_v), and its exact linear evolution."""
    import os

    from scipy.linalg import expm

    g = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.txt")):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split()
            g[k] = float(v)
    prm = {"alpha": g["turing_alpha"], "beta": g["turing_beta"], "gamma": g["turing_gamma"],
           "tau1": g["turing_spots_tau1"], "tau2": g["turing_spots_tau2"]}
    dv = 4.5e-3
    D = [g["turing_delta_u_over_delta_v"] * dv, dv]
    X, nrm = icosahedral_sphere(4)
    idx = knn(X, 31)
    W = build_weights(X, nrm, idx, 2.0)
    Y = real_sph_harm(l, m, X)
    k2 = l * (l + 1)
    J = np.array([[prm["alpha"] - D[0] * k2, 1.0], [prm["gamma"], prm["beta"] - D[1] * k2]])
    return X, idx, W, Y, prm, D, J, expm


@pytest.mark.parametrize("l,m", [(5, 2), (9, 3)])
def test_turing_linear_modes_follow_the_dispersion_relation(l, m):
    """Linearised about (0, 0), eqs. turing1-turing2 read u_t = delta_u Lap u +
    alpha u + v and v_t = delta_v Lap v + gamma u + beta v (the tau terms are
    quadratic and cubic in the perturbation).  With Lap_S Y_l^m = -l(l+1) Y_l^m
    the pair (u, v) = (a(t), b(t)) Y_l^m evolves as exp(J t) with
    J = [[alpha - delta_u k^2, 1], [gamma, beta - delta_v k^2]], k^2 = l(l+1):
    l = 5 decays (rate -0.108), l = 9 lies in the Turing band and grows
    (+0.013).  The oracle's RK4 on its weights follows exp(J t) to the
    operator's discretisation error over t = 20 from an amplitude of 1e-6."""
    X, idx, W, Y, prm, D, J, expm = _turing_linear_case(l, m)
    amp, T, dt = 1e-6, 20.0, 0.05
    u, v = rk4(assemble(idx, W), [amp * Y, np.zeros_like(Y)], D, "turing", prm, dt=dt, nsteps=int(round(T / dt)))
    E = expm(J * T)
    ue, ve = E[0, 0] * amp * Y, E[1, 0] * amp * Y
    eu = np.linalg.norm(u - ue) / np.linalg.norm(ue)
    ev = np.linalg.norm(v - ve) / np.linalg.norm(ve)
    assert eu < 2e-2 and ev < 2e-2, (l, eu, ev)
