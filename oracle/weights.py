"""RBF-FD weights for the projected surface Laplacian, following the paper's route.

For a stencil P_1 = {x_1, ..., x_n} (centre first, Sec. 4):

1. Local interpolant with a polynomial border (eq. f_interp; the bordered
   system of eq. rbf_linsys with X replaced by P_1):  A~ = [[A, U], [U^T, 0]],
   A_ij = phi(||x_i - x_j||).
2. Projected gradient matrices (eqs. proj_mat, grad and grad_x_f_interp):
   (B^d)_ij = [Pi_i grad phi(||x - x_j||)]_d at x = x_i, with
   Pi_i = I - nu_i nu_i^T; the polynomial columns carry the projected
   gradients of the border basis.
3. G^d = B^d A~^{-1} restricted to the data columns, L_P = sum_d G^d G^d
   (eq. surface_lap_P1), and the weights are the first row of L_P.

Radial kernels (Sec. 2): Gaussian exp(-(eps r)^2), multiquadric
sqrt(1+(eps r)^2), inverse multiquadric 1/sqrt(1+(eps r)^2).  psi(r) =
phi'(r)/r is used for gradients (grad_x phi(||x - x_j||) = psi (x - x_j)).

Polynomial border.  Degree 0 is the paper's literal constant term with a
border of ones.  For degree 1 or 2 (not in the paper) the monomials are taken
in xi = (x - x_1)/rho, rho = max_j ||x_j - x_1||, and replaced by an
orthonormal basis of their numerical range: P = U S V^T, keep s_j >
rank_tol * s_1, U_r = P V_r S_r^{-1}.  On the sphere and ellipsoid a
quadratic combination vanishes identically on the surface, so P is exactly
rank-deficient there; the dropped combination has zero projected gradient,
so the weights are unchanged in exact arithmetic.

Everything is FP64 NumPy/LAPACK; nothing here is blocked, fused or reordered
beyond the definitions above.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import lu_factor, lu_solve, solve

__all__ = [
    "KERNELS",
    "phi",
    "psi",
    "monomials",
    "poly_border",
    "local_matrix",
    "projected_gradients",
    "stencil_weights",
    "stencil_weights_row1",
    "build_weights",
]

KERNELS = ("mq", "imq", "ga")


def phi(kernel: str, eps: float, r2):
    """phi(r) from the squared distance r2 (Sec. 2)."""
    e = (eps * eps) * r2
    if kernel == "mq":
        return np.sqrt(1.0 + e)
    if kernel == "imq":
        return 1.0 / np.sqrt(1.0 + e)
    if kernel == "ga":
        return np.exp(-e)
    raise ValueError(kernel)


def psi(kernel: str, eps: float, r2):
    """phi'(r)/r from the squared distance r2 (no 1/r singularity)."""
    e2 = eps * eps
    e = e2 * r2
    if kernel == "mq":
        return e2 / np.sqrt(1.0 + e)
    if kernel == "imq":
        return -e2 / (np.sqrt(1.0 + e) * (1.0 + e))
    if kernel == "ga":
        return -2.0 * e2 * np.exp(-e)
    raise ValueError(kernel)


def monomials(xi: np.ndarray, degree: int):
    """Monomials of total degree <= degree in xi (n x 3) and their xi-gradients.

    Order: 1, xi_x, xi_y, xi_z, xi_x^2, xi_y^2, xi_z^2, xi_x xi_y, xi_x xi_z, xi_y xi_z.
    Returns P (n x M) and dP (n x M x 3).
    """
    n = len(xi)
    x, y, z = xi[:, 0], xi[:, 1], xi[:, 2]
    one = np.ones(n)
    zero = np.zeros(n)
    cols = [one]
    grads = [(zero, zero, zero)]
    if degree >= 1:
        cols += [x, y, z]
        grads += [(one, zero, zero), (zero, one, zero), (zero, zero, one)]
    if degree >= 2:
        cols += [x * x, y * y, z * z, x * y, x * z, y * z]
        grads += [(2 * x, zero, zero), (zero, 2 * y, zero), (zero, zero, 2 * z),
                  (y, x, zero), (z, zero, x), (zero, z, y)]
    if degree > 2:
        raise ValueError("degree must be 0, 1 or 2")
    P = np.stack(cols, axis=1)
    dP = np.stack([np.stack(g, axis=1) for g in grads], axis=1)
    return P, dP


def poly_border(Xs: np.ndarray, degree: int, rank_tol: float = 1e-10):
    """Border basis U (n x r) and its x-gradients gU (n x r x 3) at the stencil nodes.

    Degree 0: the paper's column of ones (gradient zero).  Degree 1/2: the
    orthonormal range basis of the monomials in xi (module docstring).
    Also returns rho and the singular values of the monomial matrix.
    """
    n = len(Xs)
    d = Xs - Xs[0]
    rho = float(np.sqrt(np.max(np.sum(d * d, axis=1))))
    if degree == 0:
        return np.ones((n, 1)), np.zeros((n, 1, 3)), rho, np.array([np.sqrt(n)])
    xi = d / rho
    P, dP = monomials(xi, degree)
    _, s, Vt = np.linalg.svd(P, full_matrices=False)
    r = int(np.sum(s > rank_tol * s[0]))
    T = Vt[:r].T / s[:r]
    U = P @ T
    gU = np.einsum("nmd,mr->nrd", dP, T) / rho
    return U, gU, rho, s


def local_matrix(Xs: np.ndarray, eps: float, kernel: str, U: np.ndarray):
    """A~ = [[A, U], [U^T, 0]] with A_ij = phi(||x_i - x_j||)."""
    n = len(Xs)
    r = U.shape[1]
    D = Xs[:, None, :] - Xs[None, :, :]
    r2 = (D[..., 0] * D[..., 0] + D[..., 1] * D[..., 1]) + D[..., 2] * D[..., 2]
    At = np.zeros((n + r, n + r))
    At[:n, :n] = phi(kernel, eps, r2)
    At[:n, n:] = U
    At[n:, :n] = U.T
    return At, D, r2


def projected_gradients(Xs, Ns, eps, kernel, U, gU, D=None, r2=None):
    """B^d (3 x n x m): [Pi_i grad phi(||x - x_j||)]_d at x_i, and Pi_i grad q_k(x_i)."""
    n = len(Xs)
    r = U.shape[1]
    if D is None:
        D = Xs[:, None, :] - Xs[None, :, :]
        r2 = (D[..., 0] * D[..., 0] + D[..., 1] * D[..., 1]) + D[..., 2] * D[..., 2]
    nu = Ns / np.linalg.norm(Ns, axis=1, keepdims=True)
    Pi = np.eye(3)[None, :, :] - nu[:, :, None] * nu[:, None, :]  # n x 3 x 3
    ps = psi(kernel, eps, r2)  # n x n
    # grad phi(||x - x_j||) at x_i = psi(r_ij) (x_i - x_j)
    gphi = ps[..., None] * D  # n x n x 3
    B = np.zeros((3, n, n + r))
    B[:, :, :n] = np.einsum("iab,ijb->aij", Pi, gphi)
    B[:, :, n:] = np.einsum("iab,ikb->aik", Pi, gU)
    return B


def stencil_weights(Xs, Ns, eps, kernel="mq", degree=2, rank_tol=1e-10, return_parts=False):
    """First row of L_P = sum_d G^d G^d, G^d = B^d A~^{-1}[:, :n] (eq. surface_lap_P1)."""
    n = len(Xs)
    U, gU, rho, _ = poly_border(Xs, degree, rank_tol)
    At, D, r2 = local_matrix(Xs, eps, kernel, U)
    B = projected_gradients(Xs, Ns, eps, kernel, U, gU, D, r2)
    m = At.shape[0]
    E = np.zeros((m, n))
    E[:n, :n] = np.eye(n)
    AinvE = solve(At, E, assume_a="sym")
    G = [B[k] @ AinvE for k in range(3)]
    LP = G[0] @ G[0] + G[1] @ G[1] + G[2] @ G[2]
    if return_parts:
        return LP[0].copy(), {"At": At, "B": B, "G": G, "LP": LP, "U": U, "rho": rho}
    return LP[0].copy()


def stencil_weights_row1(Xs, Ns, eps, kernel="mq", degree=2, rank_tol=1e-10):
    """The same first row, formed without G^d: a cross-check of the route above.

    g_d = (A~^{-1} b_d)[:n] with b_d = (row 1 of B^d)^T is the first row of G^d;
    r = sum_d (B^d)^T g_d; w = (A~^{-1} r)[:n]  (A~ is symmetric).
    """
    n = len(Xs)
    U, gU, _, _ = poly_border(Xs, degree, rank_tol)
    At, D, r2 = local_matrix(Xs, eps, kernel, U)
    B = projected_gradients(Xs, Ns, eps, kernel, U, gU, D, r2)
    lu = lu_factor(At)
    rv = np.zeros(At.shape[0])
    for k in range(3):
        g = lu_solve(lu, B[k][0])[:n]
        rv += B[k].T @ g
    return lu_solve(lu, rv)[:n]


def build_weights(X, nrm, idx, eps, kernel="mq", degree=2, rank_tol=1e-10, rows=None,
                  route="full"):
    """Weights for every stencil (rows of idx, centre first) at a scalar or per-row eps."""
    idx = np.asarray(idx)
    rows = np.arange(len(idx)) if rows is None else np.asarray(rows)
    eps_arr = np.broadcast_to(np.asarray(eps, dtype=np.float64), (len(idx),))
    fn = stencil_weights if route == "full" else stencil_weights_row1
    W = np.empty((len(rows), idx.shape[1]))
    for t, i in enumerate(rows):
        s = idx[i]
        W[t] = fn(X[s], nrm[s], float(eps_arr[i]), kernel, degree, rank_tol)
    return W
