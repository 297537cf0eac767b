"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each check is chosen so that a plausible mistake in the oracle (a dropped
projection, a wrong sign, a transposed operand, a lost border column) fails
at least one of them.  None of them re-types the oracle's own formulas.
"""
import math
import os

import numpy as np
import pytest

from oracle.knn import knn, knn_bruteforce
from oracle.shape import bisect_eps, kappa2, stencil_kappa
from oracle.stepper import assemble, laplacian_apply, reaction, rk4
from oracle.truth import stencil_weights_mp
from oracle.weights import (build_weights, phi, poly_border, psi, stencil_weights,
                            stencil_weights_row1)
from synth import (fibonacci_sphere, jittered_torus, planar_patch, real_sph_harm,
                   schnakenberg_ic)

U64 = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_facts.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split()
            out[k] = float(v)
    return out


@pytest.fixture(scope="module")
def sphere2500():
    X, nrm = fibonacci_sphere(2500)
    idx = knn(X, 31)
    return X, nrm, idx


# ----------------------------------------------------------------- kNN ----

def test_knn_lattice_shells():
    """Square lattice, spacing 1/8 (exact squared distances): the n nearest of
    the centre node are whole distance shells, ordered by (d^2, index)."""
    X, _ = planar_patch(9, spacing=0.125)
    c = 40  # centre of the 9 x 9 lattice
    # shells around the centre: d^2/h^2 = 0 (1), 1 (4), 2 (4), 4 (4), 5 (8)
    for n, shell in [(1, 0), (5, 1), (9, 2), (13, 4), (21, 5)]:
        idx = knn_bruteforce(X, n)[c]
        assert idx[0] == c
        d2 = np.sum((X[idx] - X[c]) ** 2, axis=1) / 0.125 ** 2
        assert np.all(np.diff(d2) >= 0)
        assert d2.max() == shell
        # within a shell, indices ascend
        for s in np.unique(d2):
            sel = idx[d2 == s]
            assert np.all(np.diff(sel) > 0)
    # a tie at the cut: n = 7 takes the two lowest-index nodes of the d^2 = 2 shell
    idx = knn_bruteforce(X, 7)[c]
    diag = sorted([c - 10, c - 8, c + 8, c + 10])
    assert list(idx[5:]) == diag[:2]


def test_knn_tree_path_equals_bruteforce():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((5000, 3))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    rows = rng.choice(5000, 200, replace=False)
    a = knn(X, 40, rows=rows)
    b = knn_bruteforce(X, 40)[rows]
    assert np.array_equal(a, b)


# ------------------------------------------------------- radial kernels ----

@pytest.mark.parametrize("kernel", ["mq", "imq", "ga"])
def test_psi_is_phi_prime_over_r(kernel):
    eps = 1.7
    r = np.linspace(0.05, 2.0, 40)
    h = 1e-6
    fd = (phi(kernel, eps, (r + h) ** 2) - phi(kernel, eps, (r - h) ** 2)) / (2 * h)
    assert np.allclose(psi(kernel, eps, r * r) * r, fd, rtol=1e-7, atol=1e-9)


def test_kernel_values_at_known_points():
    # phi(0) = 1 for all three; mq(r=1, eps=1) = sqrt 2
    for k in ("mq", "imq", "ga"):
        assert phi(k, 3.0, 0.0) == 1.0
    assert phi("mq", 1.0, 1.0) == math.sqrt(2.0)
    assert phi("imq", 1.0, 3.0) == 0.5
    assert phi("ga", 2.0, 0.25) == math.exp(-1.0)


# ------------------------------------------------------ polynomial border ----

def test_border_rank_by_surface():
    X, _ = fibonacci_sphere(2500)
    s = knn(X, 31, rows=[7])[0]
    assert poly_border(X[s], 2)[0].shape[1] == 9      # x^2+y^2+z^2 = 1 on the sphere
    assert poly_border(X[s], 1)[0].shape[1] == 4
    assert poly_border(X[s], 0)[0].shape[1] == 1
    P, _ = planar_patch(9, seed=1, jitter=0.3)
    sp = knn(P, 31, rows=[40])[0]
    assert poly_border(P[sp], 2)[0].shape[1] == 6     # z = 0: 4 monomials vanish
    T, _ = jittered_torus(40, 120)
    st = knn(T, 50, rows=[100])[0]
    assert poly_border(T[st], 2)[0].shape[1] == 10
    U = poly_border(X[s], 2)[0]
    assert np.allclose(U.T @ U, np.eye(9), atol=1e-12)


# --------------------------------------------------------------- weights ----

def _rows(step=97):
    return np.arange(0, 2500, step)


def test_row_sums_vanish(sphere2500):
    """Constants are reproduced and have zero surface gradient: L 1 = 0."""
    X, nrm, idx = sphere2500
    rows = _rows()
    W = build_weights(X, nrm, idx, 4.0, rows=rows)   # kappa ~ 5e6
    s = np.abs(W).sum(axis=1)
    assert np.max(np.abs(W.sum(axis=1)) / s) < 1e-11


def test_first_harmonics_exact_on_unit_sphere(sphere2500):
    """x, y, z are degree-1 harmonics (Delta_S x = -2x) and their projected
    gradients are quadratics reproduced by the degree-2 border, so the
    discrete operator is exact on them."""
    X, nrm, idx = sphere2500
    rows = _rows()
    W = build_weights(X, nrm, idx, 4.0, rows=rows)
    s = np.abs(W).sum(axis=1)
    for d in range(3):
        lx = np.sum(W * X[idx[rows]][:, :, d], axis=1)
        assert np.max(np.abs(lx + 2.0 * X[rows, d]) / s) < 1e-11


def test_planar_quadratic_exact():
    """On a plane the surface Laplacian is the 2-D Laplacian; degree-2 border
    reproduces quadratics and their (linear) gradients exactly."""
    P, nrm = planar_patch(11, spacing=0.1, seed=2, jitter=0.3)
    idx = knn(P, 31, rows=[60])
    s = idx[0]
    w = stencil_weights(P[s], nrm[s], 3.0)
    x, y = P[s, 0], P[s, 1]
    q = 1.5 * x * x - 0.7 * x * y + 2.5 * y * y + 0.3 * x - 1.1 * y + 4.0
    assert abs(w @ q - 2 * (1.5 + 2.5)) < 1e-6 * np.abs(w).sum() * 1e-2


def test_normal_orientation_irrelevant(sphere2500):
    X, nrm, idx = sphere2500
    s = idx[11]
    a = stencil_weights(X[s], nrm[s], 2.0)
    b = stencil_weights(X[s], -nrm[s], 2.0)
    assert np.array_equal(a, b)


def test_rotation_translation_scale_invariance(sphere2500):
    X, nrm, idx = sphere2500
    s = idx[123]
    eps = 4.0
    w0 = stencil_weights(X[s], nrm[s], eps)
    k = stencil_kappa(X[s], eps)
    tol = max(1e-9, 0.5 * k * U64) * 4
    Q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((3, 3)))
    w1 = stencil_weights(X[s] @ Q.T + np.array([0.3, -2.0, 1.0]), nrm[s] @ Q.T, eps)
    assert np.linalg.norm(w1 - w0) / np.linalg.norm(w0) < tol
    sc = 2.5
    w2 = stencil_weights(sc * X[s], nrm[s], eps / sc)
    assert np.linalg.norm(w2 * sc * sc - w0) / np.linalg.norm(w0) < tol


def test_two_routes_agree(sphere2500):
    X, nrm, idx = sphere2500
    for i in (0, 500, 1700):
        s = idx[i]
        for eps in (4.0, 2.0):
            a = stencil_weights(X[s], nrm[s], eps)
            b = stencil_weights_row1(X[s], nrm[s], eps)
            k = stencil_kappa(X[s], eps)
            assert np.linalg.norm(a - b) / np.linalg.norm(a) < max(1e-9, 0.5 * k * U64)


@pytest.mark.slow
def test_against_60_digit_truth(sphere2500):
    X, nrm, idx = sphere2500
    for i, eps in ((3, 4.0), (1201, 2.0)):
        s = idx[i]
        wt = stencil_weights_mp(X[s], nrm[s], eps)
        w = stencil_weights(X[s], nrm[s], eps)
        k = stencil_kappa(X[s], eps)
        assert np.linalg.norm(w - wt) / np.linalg.norm(wt) < max(1e-12, 0.25 * k * U64)
        assert abs(wt.sum()) < 1e-14 * np.abs(wt).sum()


def test_spherical_harmonic_eigenrelation_converges():
    """Delta_S Y_l^m = -l(l+1) Y_l^m; at a fixed eps (condition number growing
    with N, as in Sec. 6.1) the n = 31 error falls at high order in sqrt(N)
    (the paper reports order four to five for n = 17 and 31)."""
    errs = []
    for N in (1000, 4000):
        X, nrm = fibonacci_sphere(N)
        idx = knn(X, 31)
        W = build_weights(X, nrm, idx, 2.0)
        L = assemble(idx, W)
        Y = real_sph_harm(4, -2, X)
        errs.append(np.linalg.norm(L @ Y + 20.0 * Y) / np.linalg.norm(20.0 * Y))
    assert errs[0] < 1e-2
    assert errs[1] < errs[0] / 16.0  # order >= 4 in sqrt(N) (measured 26x)


def test_spectrum_left_half_plane():
    """Sec. 5: stability needs Re(lambda) <= 0 for all eigenvalues of L_X."""
    X, nrm = fibonacci_sphere(1000)
    idx = knn(X, 31)
    L = assemble(idx, build_weights(X, nrm, idx, 2.0 * math.sqrt(1000 / 2500.0))).toarray()
    lam = np.linalg.eigvals(L)
    rho = np.abs(lam).max()
    assert lam.real.max() < 1e-9 * rho


def test_sparsity_matches_paper_fraction():
    g = golden()
    assert abs(31 / 10000 - g["nnz_fraction_rbc_N10000_n31"]) < 1e-12
    # printed to two decimals of a percent (0.615% shows as 0.62%)
    assert abs(31 / 5041 - g["nnz_fraction_dtorus_N5041_n31"]) < 6e-5
    X, nrm = fibonacci_sphere(5041)
    idx = knn(X, 31, rows=np.arange(5041))
    L = assemble(idx, np.ones(idx.shape))
    assert L.nnz == 31 * 5041


# ------------------------------------------------------ condition number ----

def test_kappa_two_node_closed_form():
    """n = 2, IMQ, constant border: A~ = [[1, a, 1], [a, 1, 1], [1, 1, 0]] has
    eigenvalues 1 - a and ((1+a) +- sqrt((1+a)^2 + 8))/2."""
    Xs = np.array([[0.0, 0.0, 0.0], [0.6, 0.0, 0.8]])
    eps = 0.75
    a = 1.0 / math.sqrt(1.0 + eps * eps * 1.0)
    lam = [1 - a, ((1 + a) + math.sqrt((1 + a) ** 2 + 8)) / 2, ((1 + a) - math.sqrt((1 + a) ** 2 + 8)) / 2]
    lam = np.abs(lam)
    assert abs(stencil_kappa(Xs, eps, "imq", 0) - lam.max() / lam.min()) < 1e-12 * lam.max() / lam.min()


def test_kappa2_of_diagonal():
    assert kappa2(np.diag([3.0, -0.5, 2.0])) == 6.0


def test_kappa_decreases_with_eps(sphere2500):
    X, _, idx = sphere2500
    s = idx[42]
    ks = [stencil_kappa(X[s], e) for e in np.linspace(1.5, 8.0, 14)]
    assert all(a > b for a, b in zip(ks, ks[1:]))


def test_bisection_hits_target():
    X, _ = fibonacci_sphere(10000)
    s = knn(X, 50, rows=[17])[0]
    kT = 1e12
    eps, kap, ev, st = bisect_eps(X[s], kT)
    assert st == 0
    assert stencil_kappa(X[s], eps - 1e-4) > kT >= stencil_kappa(X[s], eps + 1e-4)
    rho = math.sqrt(np.max(np.sum((X[s] - X[s[0]]) ** 2, axis=1)))
    assert 0.4 < eps * rho < 0.8
    assert abs(math.log(kap / kT)) < 0.01
    assert 18 <= ev <= 30


# --------------------------------------------------------------- stepper ----

def test_rk4_one_step_is_taylor_quartic():
    lam = -3.0
    L = assemble(np.array([[0]]), np.array([[lam]]))
    dt = 0.1
    (y,) = rk4(L, [np.array([1.0])], [1.0], dt=dt, nsteps=1)
    z = lam * dt
    assert abs(y[0] - (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24)) < 1e-15


def test_heat_decay_on_sphere_against_exact(sphere2500):
    """The N = 2500 unit-sphere heat run: u0 = Y_6^3 + 0.1 Y_2^1 decays as exp(-l(l+1)t).
    The error is discretisation error (measured 1.98e-3 at t = 0.1)."""
    X, nrm, idx = sphere2500
    L = assemble(idx, build_weights(X, nrm, idx, 2.0))
    u0 = real_sph_harm(6, 3, X) + 0.1 * real_sph_harm(2, 1, X)
    (u,) = rk4(L, [u0], [1.0], dt=1e-4, nsteps=1000)
    ue = math.exp(-42 * 0.1) * real_sph_harm(6, 3, X) + 0.1 * math.exp(-6 * 0.1) * real_sph_harm(2, 1, X)
    err = np.linalg.norm(u - ue) / np.linalg.norm(ue)
    assert err < 3e-3


def test_schnakenberg_fixed_point_and_uniform_mode(sphere2500):
    X, nrm, idx = sphere2500
    prm = {"a": 0.1, "b": 0.9, "gamma": 50.0}
    Ru, Rv = reaction("schnakenberg", [np.array([1.0]), np.array([0.9])], prm)
    assert abs(Ru[0]) < 1e-14 and abs(Rv[0]) < 1e-14
    L = assemble(idx, build_weights(X, nrm, idx, 4.0))
    # a spatially uniform state stays uniform and follows the kinetics ODE
    u0 = np.full(2500, 1.003)
    v0 = np.full(2500, 0.897)
    U, V = rk4(L, [u0, v0], [1.0, 10.0], "schnakenberg", prm, dt=1e-4, nsteps=50)
    one = assemble(np.array([[0]]), np.array([[0.0]]))
    u1, v1 = rk4(one, [u0[:1], v0[:1]], [1.0, 10.0], "schnakenberg", prm, dt=1e-4, nsteps=50)
    assert np.max(np.abs(U - u1[0])) < 1e-9 and np.max(np.abs(V - v1[0])) < 1e-9


def test_turing_model_equilibrium_from_table1():
    """Sec. 7: with alpha = -gamma (Table 1), (0, 0) is an equilibrium; the
    reaction is also odd-symmetric in (u, v) up to the quadratic tau2 terms."""
    g = golden()
    prm = {"alpha": g["turing_alpha"], "beta": g["turing_beta"], "gamma": g["turing_gamma"],
           "tau1": g["turing_spots_tau1"], "tau2": g["turing_spots_tau2"]}
    assert prm["alpha"] == -prm["gamma"]
    Ru, Rv = reaction("turing", [np.zeros(1), np.zeros(1)], prm)
    assert Ru[0] == 0.0 and Rv[0] == 0.0
    # linearisation at 0 is [[alpha, 1], [gamma, beta]]: check by differences
    h = 1e-7
    Ru1, Rv1 = reaction("turing", [np.array([h]), np.zeros(1)], prm)
    Ru2, Rv2 = reaction("turing", [np.zeros(1), np.array([h])], prm)
    J = np.array([[Ru1[0], Ru2[0]], [Rv1[0], Rv2[0]]]) / h
    assert np.allclose(J, [[prm["alpha"], 1.0], [prm["gamma"], prm["beta"]]], atol=1e-6)


def _turing_params(row):
    g = golden()
    return {"alpha": g["turing_alpha"], "beta": g["turing_beta"], "gamma": g["turing_gamma"],
            "tau1": g[f"turing_{row}_tau1"], "tau2": g[f"turing_{row}_tau2"]}


@pytest.mark.parametrize("row", ["spots", "stripes"])
def test_turing_nonlinear_terms_cancel_in_the_sum(row):
    """Eqs. turing1, turing2: the tau1 (cubic) and tau2 (quadratic) terms enter
    the two equations with opposite signs, so R_u + R_v is the linear part
    (alpha + gamma) u + (1 + beta) v for every state.  A wrong sign, power or
    coefficient in any one nonlinear term breaks this identity."""
    prm = _turing_params(row)
    rng = np.random.default_rng(11)
    u = rng.uniform(-3, 3, 2000)
    v = rng.uniform(-3, 3, 2000)
    Ru, Rv = reaction("turing", [u, v], prm)
    lin = (prm["alpha"] + prm["gamma"]) * u + (1.0 + prm["beta"]) * v
    scale = np.abs(Ru) + np.abs(Rv) + np.abs(lin)
    assert np.max(np.abs((Ru + Rv) - lin) / scale) < 1e-14


def test_turing_stripes_row_is_odd():
    """With tau2 = 0 (Table 1, stripes rows) only linear and cubic terms
    remain, so R(-u, -v) = -R(u, v) exactly."""
    prm = _turing_params("stripes")
    assert prm["tau2"] == 0.0
    rng = np.random.default_rng(12)
    u = rng.uniform(-3, 3, 500)
    v = rng.uniform(-3, 3, 500)
    Ru, Rv = reaction("turing", [u, v], prm)
    Nu, Nv = reaction("turing", [-u, -v], prm)
    assert np.array_equal(Nu, -Ru) and np.array_equal(Nv, -Rv)


@pytest.mark.parametrize("which,degree", [("tau1", 3), ("tau2", 2)])
def test_turing_nonlinear_terms_have_their_degree(which, degree):
    """Eqs. turing1, turing2: the tau1 terms are cubic and the tau2 terms
    quadratic in (u, v), and both are present in both equations.  Switching one
    parameter on changes R by a homogeneous polynomial of that degree: scaling
    the state by s scales the change by s^degree.  (Together with the sum
    identity this catches a pair of terms dropped or mis-powered together.)"""
    base = _turing_params("spots")
    on = dict(base)
    off = dict(base)
    off[which] = 0.0
    other = "tau2" if which == "tau1" else "tau1"
    on[other] = off[other] = 0.0
    rng = np.random.default_rng(13)
    u = rng.uniform(0.2, 1.0, 100)
    v = rng.uniform(0.2, 1.0, 100)
    for s in (0.5, 2.0, 3.0):
        d1 = [a - b for a, b in zip(reaction("turing", [u, v], on), reaction("turing", [u, v], off))]
        ds = [a - b for a, b in zip(reaction("turing", [s * u, s * v], on), reaction("turing", [s * u, s * v], off))]
        for a, b in zip(d1, ds):
            assert np.min(np.abs(a)) > 0.0  # the term is present in this equation
            assert np.allclose(b, s ** degree * a, rtol=1e-12, atol=0.0)


def test_laplacian_apply_equals_sparse_matvec():
    """(L_X u)_i = sum_k w_ik u_(idx_ik) (Sec. 4: row i of L_X holds stencil i's
    weights at its node indices) against a dense matrix filled entry by entry
    and against SciPy's CSR product, on ragged random data: N not a multiple
    of any tile, odd n, repeated indices inside a row (which add)."""
    rng = np.random.default_rng(14)
    for N, n in ((1, 1), (7, 3), (203, 31), (1000, 50)):
        idx = rng.integers(0, N, size=(N, n))
        idx[:, 0] = np.arange(N)
        if n > 2:
            idx[::3, 2] = idx[::3, 1]  # duplicate column in some rows
        W = rng.standard_normal((N, n))
        u = rng.standard_normal(N)
        got = laplacian_apply(idx, W, u)
        dense = np.zeros((N, N))
        for i in range(N):
            for k in range(n):
                dense[i, idx[i, k]] += W[i, k]
        ref = dense @ u
        csr = assemble(idx, W) @ u
        tol = 1e-15 * (np.abs(W) @ np.ones(n)) * np.max(np.abs(u)) * n
        assert np.all(np.abs(got - ref) <= tol)
        assert np.all(np.abs(got - csr) <= tol)


def test_ic_generators_are_seeded():
    a = schnakenberg_ic(100)
    b = schnakenberg_ic(100)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_kappa_mp_matches_fp64_where_fp64_resolves_it():
    """The high-precision kappa_2 agrees with the FP64 eigvalsh one to about
    kappa u where FP64 resolves it, and one node with the ones border gives
    [[phi(0), 1], [1, 0]] = [[1, 1], [1, 0]] (IMQ), whose eigenvalues
    (1 +- sqrt 5) / 2 give kappa = (1 + sqrt 5) / (sqrt 5 - 1).  At a target
    FP64 cannot resolve (kappa ~ 1e18), 50 and 80 digits agree."""
    from oracle.truth import stencil_kappa_mp

    X, _ = fibonacci_sphere(400)
    idx = knn(X, 17)
    for i in (0, 123, 399):
        for eps in (3.0, 6.0):
            k64 = stencil_kappa(X[idx[i]], eps, kernel="imq", degree=0)
            kmp = stencil_kappa_mp(X[idx[i]], eps, kernel="imq", degree=0)
            assert abs(kmp / k64 - 1.0) < 50 * k64 * U64 + 1e-13, (i, eps, k64, kmp)
    # one node and the ones border: [[phi(0), 1], [1, 0]] = [[1, 1], [1, 0]]
    k1 = stencil_kappa_mp(np.zeros((1, 3)), 2.0, kernel="imq", degree=0)
    assert abs(k1 - (1 + math.sqrt(5)) / (math.sqrt(5) - 1)) < 1e-14
    s = idx[7]
    k50 = stencil_kappa_mp(X[s], 0.05, kernel="imq", degree=0, dps=50)
    k80 = stencil_kappa_mp(X[s], 0.05, kernel="imq", degree=0, dps=80)
    assert k50 > 1e15 and abs(k50 / k80 - 1.0) < 1e-12


def test_bisect_mp_against_two_node_closed_form():
    """The high-precision bisection (Sec. 5) on two nodes at distance r with
    the constant border (IMQ).  A~ = [[1, p, 1], [p, 1, 1], [1, 1, 0]] with
    p = 1 / sqrt(1 + eps^2 r^2): (1, -1, 0) is an eigenvector with eigenvalue
    1 - p, and on its complement A~ acts as [[1 + p, sqrt 2], [sqrt 2, 0]],
    eigenvalues ((1 + p) +- sqrt((1 + p)^2 + 8)) / 2.  kappa_2(eps) from these
    closed forms matches the oracle's eigenvalues, its root at kappa_T (found
    to 40 digits) lies within tol / 2 of the returned eps, and a target the
    bracket cannot reach gives status 2."""
    import mpmath as mp

    from oracle.truth import bisect_eps_mp, stencil_kappa_mp

    r = 0.01
    X = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])

    def kappa_closed(e):
        p = 1 / mp.sqrt(1 + (e * r) ** 2)
        s = mp.sqrt((1 + p) ** 2 + 8)
        lam = [abs(1 - p), abs(((1 + p) + s) / 2), abs(((1 + p) - s) / 2)]
        return max(lam) / min(lam)

    with mp.workdps(40):
        for e in (0.5, 3.0, 20.0, 400.0):
            k = stencil_kappa_mp(X, e, kernel="imq", degree=0)
            assert abs(k / float(kappa_closed(mp.mpf(e))) - 1.0) < 1e-13, (e, k)
        for kT in (1e3, 1e6, 1e8):
            guess = math.sqrt(2 * 2.7320508 / kT) / r  # kappa ~ (1 + sqrt 3) / (eps^2 r^2 / 2) for small eps r
            root = mp.findroot(lambda e: mp.log(kappa_closed(e)) - mp.log(kT), mp.mpf(guess))
            eps, st = bisect_eps_mp(X, kT, kernel="imq", degree=0)
            assert st == 0
            assert abs(eps - float(root)) <= 0.5e-4 + 1e-12, (kT, eps, float(root))
    # the bracket [0.05, 20] / rho halved at most 8 times cannot reach kappa_T = 1e12 here
    _, st = bisect_eps_mp(X, 1e12, kernel="imq", degree=0)
    assert st == 2
