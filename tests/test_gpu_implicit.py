"""Semi-implicit BDF stepping (SBDF-k; the paper's BDF4 of Sec. 6 and SBDF2
of Sec. 7) on the GPU against the oracle's, which solves each step with a
sparse direct factorisation.  The GPU solves with BiCGSTAB to a relative
residual of 1e-12 per step (the paper's tolerance), so the two trajectories
agree to about that times the number of steps; the bar is 1e-10 relative L2.
"""
import math

import numpy as np
import pytest
import torch

from oracle.knn import knn as oracle_knn
from oracle.shape import bisect_eps
from oracle.stepper import assemble, imex_bdf, rk4
from oracle.weights import build_weights as oracle_weights
from synth import blob, fibonacci_sphere, real_sph_harm, schnakenberg_ic

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def sphere(lib):
    X, nrm = fibonacci_sphere(2500)
    idx = oracle_knn(X, 31)
    W = oracle_weights(X, nrm, idx, 2.0)
    _, perm = lib.knn(dev(X), 31)
    op = lib.Operator(dev(idx, torch.int32), dev(W), perm=perm)
    return X, idx, W, op


@pytest.mark.parametrize("order,with_history", [(1, False), (2, False), (3, False), (3, True), (4, False), (4, True)])
def test_bdf_forced_heat_matches_oracle(lib, sphere, order, with_history):
    """u_t = L u + exp(-5 t) F on the unit sphere with u = exp(-5t) Y_4^2 as
    the manufactured solution (F = (20 - 5) Y_4^2), dt = 4e-3 (about 2.6
    times the RK4 stability limit of this operator, 2.785 / rho(L) ~ 1.5e-3),
    40 steps."""
    X, idx, W, op = sphere
    Y = real_sph_harm(4, 2, X)
    F = 15.0 * Y
    dt, steps, t0 = 4e-3, 40, 0.1
    u0 = math.exp(-5 * t0) * Y
    hist = [[math.exp(-5 * (t0 - j * dt)) * Y] for j in range(1, order)] if with_history else None
    (ref,) = imex_bdf(assemble(idx, W), [u0], [1.0], dt=dt, nsteps=steps, order=order, t0=t0,
                      forcing=(-5.0, [F]), history=hist)
    H = dev(np.stack([h[0] for h in hist])[:, None, :]) if with_history else None
    got, its, res = op.step_imex(dev(u0), dt, steps, order=order, history=H, forcing=dev(F[None, :]), t0=t0, lam=-5.0)
    got = host(got)[0]
    print(f"[imex] order {order} history {with_history}: {its} BiCGSTAB iterations over {steps} steps, "
          f"worst relative residual {res:.1e}, |gpu - oracle| / |oracle| = {rel(got, ref):.2e}", flush=True)
    assert res <= 1e-12
    assert rel(got, ref) <= 1e-10
    # the step is well beyond the explicit limit yet stays on the manufactured solution
    ex = math.exp(-5 * (t0 + steps * dt)) * Y
    assert rel(got, ex) < 2e-2


def test_sbdf2_schnakenberg_matches_oracle(lib, sphere):
    """The Schnakenberg kinetics with SBDF2 (Sec. 7's scheme) at dt = 2e-4,
    40 times the RK4 limit of D_v = 10, against the oracle's SBDF2."""
    X, idx, W, op = sphere
    u0, v0 = schnakenberg_ic(len(X))
    prm = {"a": 0.1, "b": 0.9, "gamma": 50.0}
    dt, steps = 2e-4, 50
    (ru, rv) = imex_bdf(assemble(idx, W), [u0, v0], [1.0, 10.0], "schnakenberg", prm, dt=dt, nsteps=steps, order=2)
    got, its, res = op.step_imex(dev(np.stack([u0, v0])), dt, steps, order=2, D=(1.0, 10.0), reaction="schnakenberg",
                                 params=(0.1, 0.9, 50.0))
    g = host(got)
    print(f"[imex] SBDF2 Schnakenberg: {its} iterations, |du| {rel(g[0], ru):.2e} |dv| {rel(g[1], rv):.2e}",
          flush=True)
    assert rel(g[0], ru) <= 1e-10 and rel(g[1], rv) <= 1e-10


def test_turing_sbdf2_matches_oracle(lib, sphere):
    """The Turing system of Sec. 7 (Table 1 spots row) with SBDF2 at dt = 0.05."""
    X, idx, W, op = sphere
    rng = np.random.default_rng(5)
    u0 = rng.uniform(-0.01, 0.01, len(X))
    v0 = rng.uniform(-0.01, 0.01, len(X))
    prm = {"alpha": 0.899, "beta": -0.91, "gamma": -0.899, "tau1": 0.02, "tau2": 0.2}
    D = [0.516 * 0.01, 0.01]
    dt, steps = 0.05, 40
    (ru, rv) = imex_bdf(assemble(idx, W), [u0, v0], D, "turing", prm, dt=dt, nsteps=steps, order=2)
    got, its, res = op.step_imex(dev(np.stack([u0, v0])), dt, steps, order=2, D=D, reaction="turing",
                                 params=(0.899, -0.91, -0.899, 0.02, 0.2))
    g = host(got)
    assert rel(g[0], ru) <= 1e-10 and rel(g[1], rv) <= 1e-10


@pytest.fixture(scope="module")
def irregular(lib):
    """The implicit blob surface with N = 2000 Poisson-disk nodes, n = 31 and
    the oracle's per-stencil bisection to kappa_T = 1e10: a few dozen of its
    stencils give L a positive diagonal entry (eigenvalues still in the left
    half plane), the case where a diagonal preconditioner breaks down."""
    X, nrm = blob(2000)
    idx = oracle_knn(X, 31)
    eps = np.array([bisect_eps(X[idx[i]], 1e10)[0] for i in range(len(X))])
    W = oracle_weights(X, nrm, idx, eps)
    _, perm = lib.knn(dev(X), 31)
    op = lib.Operator(dev(idx, torch.int32), dev(W), perm=perm)
    return X, idx, W, op


@pytest.mark.parametrize("dt", [5e-3, 1e-2])
def test_sbdf2_irregular_operator_matches_oracle(lib, irregular, dt):
    """SBDF2 Schnakenberg (D = 1, 10) at Sec. 7's dt = 0.01 and half of it,
    about 53 and 27 times the RK4 limit of this operator (rho(L) ~ 1.5e3),
    against the oracle's direct solves."""
    X, idx, W, op = irregular
    assert np.sum(W[:, 0] > 0) > 0
    u0, v0 = schnakenberg_ic(len(X))
    prm = {"a": 0.1, "b": 0.9, "gamma": 50.0}
    steps = 20
    (ru, rv) = imex_bdf(assemble(idx, W), [u0, v0], [1.0, 10.0], "schnakenberg", prm, dt=dt, nsteps=steps, order=2)
    got, its, res = op.step_imex(dev(np.stack([u0, v0])), dt, steps, order=2, D=(1.0, 10.0), reaction="schnakenberg",
                                 params=(0.1, 0.9, 50.0), maxit=500)
    g = host(got)
    print(f"[imex] irregular operator, SBDF2 dt={dt}: {its} iterations over {2 * steps} solves, worst relative "
          f"residual {res:.1e}, |du| {rel(g[0], ru):.2e} |dv| {rel(g[1], rv):.2e}", flush=True)
    assert res <= 1e-12
    assert rel(g[0], ru) <= 1e-10 and rel(g[1], rv) <= 1e-10


def test_imex_reports_a_missed_tolerance(lib, sphere):
    X, idx, W, op = sphere
    u0 = real_sph_harm(3, 1, X)
    with pytest.raises(lib.RbffdError, match="did not reach"):
        op.step_imex(dev(u0), 1e-2, 3, order=2, tol=1e-14, maxit=1)


def test_imex_second_order_in_time(lib, sphere):
    """SBDF2 (BDF1 first step) on the forced heat problem: the time error
    against a 16x finer run falls by about 4 when dt halves.  (Exact-solution
    history would be inconsistent with the discrete operator by its spatial
    error and would pollute a pure time-order measurement.)"""
    X, idx, W, op = sphere
    Y = real_sph_harm(4, 2, X)
    F = 15.0 * Y
    T, t0 = 0.05, 0.0

    def run(dt):
        n = int(round(T / dt))
        got, _, _ = op.step_imex(dev(Y * math.exp(-5 * t0)), dt, n, order=2, forcing=dev(F[None, :]),
                                 t0=t0, lam=-5.0)
        return host(got)[0]

    fine = run(T / 400)
    e1 = rel(run(T / 25), fine)
    e2 = rel(run(T / 50), fine)
    print(f"[imex] SBDF2 time errors {e1:.2e} {e2:.2e} ratio {e1 / e2:.2f}", flush=True)
    assert 3.3 < e1 / e2 < 4.8


def test_imex_is_reproducible(lib, irregular):
    """Two identical SBDF2 runs (graph-replayed iterations, fixed-order block
    reductions) give the same bits, and the iteration counts agree."""
    X, idx, W, op = irregular
    u0, v0 = schnakenberg_ic(len(X))
    kw = dict(order=2, D=(1.0, 10.0), reaction="schnakenberg", params=(0.1, 0.9, 50.0), maxit=500)
    a, ia, ra = op.step_imex(dev(np.stack([u0, v0])), 1e-2, 10, **kw)
    b, ib, rb_ = op.step_imex(dev(np.stack([u0, v0])), 1e-2, 10, **kw)
    ha, hb = host(a), host(b)
    assert ia == ib and ra == rb_
    assert np.array_equal(ha.view(np.uint64), hb.view(np.uint64))


def test_imex_zero_steps_and_zero_state(lib, sphere):
    """nsteps = 0 returns the state unchanged; a zero state stays exactly zero
    (the first residual is zero, so no iteration runs)."""
    X, idx, W, op = sphere
    u0 = real_sph_harm(3, 1, X)
    got, its, _ = op.step_imex(dev(u0), 1e-2, 0, order=2)
    assert its == 0 and np.array_equal(host(got)[0], u0)
    z, its, res = op.step_imex(dev(np.zeros(len(X))), 1e-2, 3, order=2)
    assert its == 0 and not np.any(host(z))
