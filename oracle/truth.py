"""60-digit reference weights for small stencils (mpmath).

Every entry of the bordered system, the border basis (monomials in xi, their
SVD and the orthonormal range basis), the projected gradients and L_P is
formed in mpmath at `dps` digits from the FP64 node coordinates, following
the same definitions as ``oracle.weights`` (first row of sum_d G^d G^d).
Used to measure how far an FP64 computation of the weights sits from the
exact weights of the same stencil.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np

__all__ = ["stencil_weights_mp", "stencil_kappa_mp", "bisect_eps_mp"]


def _phi_psi(kernel, e2, r2):
    t = 1 + e2 * r2
    if kernel == "mq":
        s = mp.sqrt(t)
        return s, e2 / s
    if kernel == "imq":
        s = mp.sqrt(t)
        return 1 / s, -e2 / (s * t)
    if kernel == "ga":
        g = mp.exp(-e2 * r2)
        return g, -2 * e2 * g
    raise ValueError(kernel)


def _border_mp(X, degree, rank_tol):
    """Border basis and its x-gradients (3 matrices n x r) in mpmath."""
    n = len(X)
    if degree == 0:
        U = mp.ones(n, 1)
        return U, [mp.zeros(n, 1) for _ in range(3)]
    rho = mp.sqrt(max((X[j][0] - X[0][0]) ** 2 + (X[j][1] - X[0][1]) ** 2
                      + (X[j][2] - X[0][2]) ** 2 for j in range(n)))
    rows, grows = [], []
    for j in range(n):
        x, y, z = [(X[j][c] - X[0][c]) / rho for c in range(3)]
        row = [mp.mpf(1), x, y, z]
        g = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
        if degree >= 2:
            row += [x * x, y * y, z * z, x * y, x * z, y * z]
            g += [(2 * x, 0, 0), (0, 2 * y, 0), (0, 0, 2 * z), (y, x, 0), (z, 0, x), (0, z, y)]
        rows.append(row)
        grows.append(g)
    M = len(rows[0])
    P = mp.matrix(rows)
    _, S, V = mp.svd_r(P, full_matrices=False, compute_uv=True)
    s = [S[k] for k in range(M)]
    order = sorted(range(M), key=lambda k: -s[k])
    keep = [k for k in order if s[k] > rank_tol * s[order[0]]]
    r = len(keep)
    T = mp.zeros(M, r)
    for c, k in enumerate(keep):
        for l in range(M):
            T[l, c] = V[k, l] / s[k]
    U = P * T
    gU = []
    for a in range(3):
        dP = mp.matrix([[mp.mpf(grows[j][l][a]) / rho for l in range(M)] for j in range(n)])
        gU.append(dP * T)
    return U, gU


def stencil_weights_mp(Xs, Ns, eps, kernel="mq", degree=2, rank_tol=1e-10, dps=60):
    """First row of L_P in `dps`-digit arithmetic; returns float64 weights."""
    with mp.workdps(dps):
        n = len(Xs)
        X = [[mp.mpf(float(v)) for v in row] for row in Xs]
        U, gU = _border_mp(X, degree, rank_tol)
        r = U.cols
        m = n + r
        nu = []
        for row in Ns:
            v = [mp.mpf(float(c)) for c in row]
            s = mp.sqrt(v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
            nu.append([c / s for c in v])
        e2 = mp.mpf(float(eps)) ** 2
        A = mp.zeros(m, m)
        Bd = [mp.zeros(n, m) for _ in range(3)]
        for i in range(n):
            Pi = [[(1 if a == b else 0) - nu[i][a] * nu[i][b] for b in range(3)] for a in range(3)]
            for j in range(n):
                d = [X[i][c] - X[j][c] for c in range(3)]
                r2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
                ph, ps = _phi_psi(kernel, e2, r2)
                A[i, j] = ph
                for a in range(3):
                    Bd[a][i, j] = ps * sum(Pi[a][b] * d[b] for b in range(3))
            for k in range(r):
                A[i, n + k] = U[i, k]
                A[n + k, i] = U[i, k]
                g = [gU[c][i, k] for c in range(3)]
                for a in range(3):
                    Bd[a][i, n + k] = sum(Pi[a][b] * g[b] for b in range(3))
        Ainv = mp.inverse(A)
        AinvE = mp.zeros(m, n)
        for i in range(m):
            for j in range(n):
                AinvE[i, j] = Ainv[i, j]
        LP = mp.zeros(n, n)
        for a in range(3):
            G = Bd[a] * AinvE
            LP += G * G
        return np.array([float(LP[0, j]) for j in range(n)])


def _local_matrix_mp(X, e2, kernel, U):
    n = len(X)
    r = U.cols
    A = mp.zeros(n + r, n + r)
    for i in range(n):
        for j in range(n):
            d = [X[i][c] - X[j][c] for c in range(3)]
            A[i, j] = _phi_psi(kernel, e2, d[0] ** 2 + d[1] ** 2 + d[2] ** 2)[0]
        for k in range(r):
            A[i, n + k] = U[i, k]
            A[n + k, i] = U[i, k]
    return A


def stencil_kappa_mp(Xs, eps, kernel="mq", degree=0, rank_tol=1e-10, dps=50):
    """kappa_2 of the bordered local matrix (Sec. 5, eq. target_cond:
    max|lambda| / min|lambda|, A~ symmetric) from its eigenvalues in
    `dps`-digit arithmetic, for targets beyond what FP64 resolves."""
    with mp.workdps(dps):
        X = [[mp.mpf(float(v)) for v in row] for row in Xs]
        U, _ = _border_mp(X, degree, rank_tol)
        A = _local_matrix_mp(X, mp.mpf(float(eps)) ** 2, kernel, U)
        ev = mp.eigsy(A, eigvals_only=True)
        lam = [abs(ev[i]) for i in range(len(ev))]
        return float(max(lam) / min(lam))


def bisect_eps_mp(Xs, kappa_T, kernel="mq", degree=0, tol=1e-4, lo_mult=0.05, hi_mult=20.0, max_expand=8, dps=50):
    """The bisection of Sec. 5 (as oracle.shape.bisect_eps: bracket
    [lo_mult, hi_mult] / rho expanded by halving / doubling, then halving the
    bracket until it is tol wide; kappa > kappa_T moves lo) with every kappa_2
    from stencil_kappa_mp.  Returns (eps, status): 0 ok, 2 no bracket."""
    d = np.asarray(Xs) - np.asarray(Xs)[0]
    rho = float(np.sqrt(np.max(np.sum(d * d, axis=1))))

    def above(e):
        return stencil_kappa_mp(Xs, e, kernel, degree, dps=dps) > kappa_T

    lo, hi = lo_mult / rho, hi_mult / rho
    ok = True
    t = 0
    while not above(lo) and t < max_expand:
        lo *= 0.5
        t += 1
    ok = ok and above(lo)
    t = 0
    while above(hi) and t < max_expand:
        hi *= 2.0
        t += 1
    ok = ok and not above(hi)
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if above(mid):
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi), (0 if ok else 2)
