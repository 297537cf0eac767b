"""Method of lines with the sparse RBF-FD Laplacian (Sec. 4.2, eq. kernel_mol).

L_X is the N x N matrix whose row k holds the weights of stencil k at the
stencil's node indices (Sec. 4, the paragraph after the first-row weights).
The semi-discrete system du_s/dt = D_s L_X u_s + R_s(u) is advanced with the
classical fourth-order Runge-Kutta method (the paper uses BDF4 and SBDF2; the
explicit RK4 is the reading for these workloads).

Reactions:
  none         R = 0 (heat equation)
  schnakenberg R_u = gamma (a - u + u^2 v),  R_v = gamma (b - u^2 v)
  turing       the activator-inhibitor system of Sec. 7 (eqs. turing1,
               turing2): R_u = alpha u (1 - tau1 v^2) + v (1 - tau2 u),
               R_v = beta v (1 + alpha tau1 u v / beta) + u (gamma + tau2 v)
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = ["assemble", "reaction", "rhs", "rk4", "laplacian_apply", "BDF_COEFFS", "imex_bdf"]


def assemble(idx: np.ndarray, w: np.ndarray, N: int | None = None) -> sp.csr_matrix:
    """Sparse L_X with row i = weights of stencil i at its node indices."""
    Nr, n = idx.shape
    N = Nr if N is None else N
    rows = np.repeat(np.arange(Nr), n)
    return sp.csr_matrix((w.ravel(), (rows, idx.ravel())), shape=(Nr, N))


def laplacian_apply(idx, w, u):
    """(L_X u)_i = sum_j w_ij u_{idx_ij}, summed in slot order."""
    acc = np.zeros(len(idx))
    for k in range(idx.shape[1]):
        acc = acc + w[:, k] * u[idx[:, k]]
    return acc


def reaction(kind: str, Y, params):
    if kind == "none":
        return [np.zeros_like(y) for y in Y]
    if kind == "schnakenberg":
        a, b, g = params["a"], params["b"], params["gamma"]
        u, v = Y
        u2v = u * u * v
        return [g * (a - u + u2v), g * (b - u2v)]
    if kind == "turing":
        al, be, ga = params["alpha"], params["beta"], params["gamma"]
        t1, t2 = params["tau1"], params["tau2"]
        u, v = Y
        return [al * u * (1.0 - t1 * v * v) + v * (1.0 - t2 * u),
                be * v * (1.0 + al * t1 / be * u * v) + u * (ga + t2 * v)]
    raise ValueError(kind)


def rhs(L, Y, D, kind, params, t=0.0, forcing=None):
    """du_s/dt = D_s L u_s + R_s(u) + f_s(t) (eq. diffusion_scalar with the
    forcing of Sec. 6).  forcing = (lam, F): f_s(t, x_i) = exp(lam t) F[s][i],
    the form of the manufactured solutions (eqs. sph_forced, torus_forced)."""
    R = reaction(kind, Y, params)
    out = [D[s] * (L @ Y[s]) + R[s] for s in range(len(Y))]
    if forcing is not None:
        lam, F = forcing
        out = [out[s] + np.exp(lam * t) * F[s] for s in range(len(Y))]
    return out


def rk4(L, Y0, D, kind="none", params=None, dt=1e-4, nsteps=1, t0=0.0, forcing=None):
    """Classical RK4 from time t0: k1 = f(t, y), k2 = f(t + dt/2, y + dt/2 k1),
    k3 = f(t + dt/2, y + dt/2 k2), k4 = f(t + dt, y + dt k3),
    y+ = y + dt/6 (k1 + 2 k2 + 2 k3 + k4)."""
    Y = [np.array(y, dtype=np.float64) for y in Y0]
    S = len(Y)
    for i in range(nsteps):
        t = t0 + i * dt
        k1 = rhs(L, Y, D, kind, params, t, forcing)
        k2 = rhs(L, [Y[s] + 0.5 * dt * k1[s] for s in range(S)], D, kind, params, t + 0.5 * dt, forcing)
        k3 = rhs(L, [Y[s] + 0.5 * dt * k2[s] for s in range(S)], D, kind, params, t + 0.5 * dt, forcing)
        k4 = rhs(L, [Y[s] + dt * k3[s] for s in range(S)], D, kind, params, t + dt, forcing)
        Y = [Y[s] + (dt / 6.0) * (k1[s] + 2.0 * k2[s] + 2.0 * k3[s] + k4[s]) for s in range(S)]
    return Y


# Coefficients of the k-step backward difference formulas and of the
# extrapolation of the explicit terms (semi-implicit BDF, SBDF-k):
#   sum_{j=0}^{k} a_j u^{n+1-j} = dt (D L u^{n+1} + f(t_{n+1}) + sum_{j=1}^{k} b_j R(u^{n+1-j})).
# The paper time-steps diffusion with BDF4 (Sec. 6) and the Turing system
# with SBDF2 (Sec. 7); a is the standard BDF row, b the extrapolation of
# order k (R at t_{n+1} from the k previous values).
BDF_COEFFS = {
    1: ([1.0, -1.0], [1.0]),
    2: ([1.5, -2.0, 0.5], [2.0, -1.0]),
    3: ([11.0 / 6.0, -3.0, 1.5, -1.0 / 3.0], [3.0, -3.0, 1.0]),
    4: ([25.0 / 12.0, -4.0, 3.0, -4.0 / 3.0, 0.25], [4.0, -6.0, 4.0, -1.0]),
}


def imex_bdf(L, Y0, D, kind="none", params=None, dt=1e-4, nsteps=1, order=2, t0=0.0, forcing=None,
             history=None):
    """SBDF-`order` from time t0: the diffusion term and the forcing are taken
    at the new time (implicit; the forcing is a known function of t), the
    reaction is extrapolated from the previous values.  history (optional):
    the states at t0 - dt, t0 - 2 dt, ... (the paper starts BDF4 from the
    exact solution); without it, the first steps use the lower orders 1, 2,
    ... until enough history exists.  Each step solves
    (a_0 I - dt D_s L) u_s^{n+1} = rhs_s with a sparse direct solver."""
    import scipy.sparse.linalg as spla

    S = len(Y0)
    N = L.shape[0]
    hist = [[np.array(y, dtype=np.float64) for y in Y0]]          # u^n, u^{n-1}, ...
    for h in (history or [])[:order - 1]:
        hist.append([np.array(y, dtype=np.float64) for y in h])
    rh = [reaction(kind, Yh, params) for Yh in hist]                # R(u^n), ...
    I = sp.identity(N, format="csc")
    Lc = sp.csc_matrix(L)
    lu_cache = {}
    have = len(hist)
    for i in range(nsteps):
        k = min(order, have + i)
        a, b = BDF_COEFFS[k]
        t1 = t0 + (i + 1) * dt
        new = []
        for s in range(S):
            r = np.zeros(N)
            for j in range(1, k + 1):
                r -= a[j] * hist[j - 1][s]
                r += dt * b[j - 1] * rh[j - 1][s]
            if forcing is not None:
                lam, F = forcing
                r += dt * np.exp(lam * t1) * F[s]
            key = (k, s)
            if key not in lu_cache:
                lu_cache[key] = spla.splu((a[0] * I - (dt * D[s]) * Lc).tocsc())
            new.append(lu_cache[key].solve(r))
        hist.insert(0, new)
        rh.insert(0, reaction(kind, new, params))
        del hist[order:]
        del rh[order:]
    return hist[0]
