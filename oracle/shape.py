"""Per-stencil shape parameter for a target condition number (Sec. 5).

kappa(A~(eps)) is the 2-norm condition number of the bordered interpolation
matrix; A~ is symmetric, so it is max|lambda| / min|lambda| (eq. target_cond
and the sentence after it).  The paper seeks the zero of
F(eps) = log(kappa(A~(eps)) / kappa_T), unique because kappa grows
monotonically as eps decreases, and solves it to an absolute tolerance of
1e-4 without naming the root finder.

Reading used here: bisection on eps.  The bracket is [lo_mult, hi_mult]/rho
(rho = stencil radius); while kappa(lo) <= kappa_T, lo is halved, and while
kappa(hi) > kappa_T, hi is doubled, at most max_expand times each (else the
stencil's status is "no bracket").  Then, while hi - lo > tol:
mid = (lo + hi)/2; kappa(mid) > kappa_T sends lo to mid, otherwise hi to mid.
The result is the final midpoint and kappa there.  A non-finite kappa counts
as "above target".
"""
from __future__ import annotations

import numpy as np

from .weights import local_matrix, poly_border

__all__ = ["kappa2", "stencil_kappa", "bisect_eps", "select_eps_all",
           "STATUS_OK", "STATUS_FALLBACK", "STATUS_NO_BRACKET"]

STATUS_OK = 0
STATUS_FALLBACK = 1
STATUS_NO_BRACKET = 2


def kappa2(At: np.ndarray) -> float:
    """max|lambda| / min|lambda| of a symmetric matrix (eigvalsh)."""
    lam = np.abs(np.linalg.eigvalsh(At))
    lo = lam.min()
    return float(lam.max() / lo) if lo > 0 else float("inf")


def stencil_kappa(Xs, eps, kernel="mq", degree=2, rank_tol=1e-10, border=None):
    U = border if border is not None else poly_border(Xs, degree, rank_tol)[0]
    At, _, _ = local_matrix(Xs, eps, kernel, U)
    return kappa2(At)


def _above(k, kT):
    return (not np.isfinite(k)) or k > kT


def bisect_eps(Xs, kappa_T, kernel="mq", degree=2, rank_tol=1e-10, tol=1e-4,
               lo_mult=0.05, hi_mult=20.0, max_expand=8):
    """Bisection of the module docstring.  Returns (eps, kappa, evaluations, status)."""
    U, _, rho, _ = poly_border(Xs, degree, rank_tol)

    def K(e):
        return stencil_kappa(Xs, e, kernel, degree, rank_tol, border=U)

    lo = lo_mult / rho
    hi = hi_mult / rho
    evals = 0
    status = STATUS_OK
    k_lo = K(lo)
    evals += 1
    t = 0
    while not _above(k_lo, kappa_T) and t < max_expand:
        lo *= 0.5
        k_lo = K(lo)
        evals += 1
        t += 1
    if not _above(k_lo, kappa_T):
        status = STATUS_NO_BRACKET
    k_hi = K(hi)
    evals += 1
    t = 0
    while _above(k_hi, kappa_T) and t < max_expand:
        hi *= 2.0
        k_hi = K(hi)
        evals += 1
        t += 1
    if _above(k_hi, kappa_T):
        status = STATUS_NO_BRACKET
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if _above(K(mid), kappa_T):
            lo = mid
        else:
            hi = mid
        evals += 1
    eps = 0.5 * (lo + hi)
    return eps, K(eps), evals + 1, status


def select_eps_all(X, idx, kappa_T, rows=None, **kw):
    """bisect_eps for every stencil row (or the given rows)."""
    rows = np.arange(len(idx)) if rows is None else np.asarray(rows)
    eps = np.empty(len(rows))
    kap = np.empty(len(rows))
    st = np.empty(len(rows), dtype=np.int32)
    for t, i in enumerate(rows):
        eps[t], kap[t], _, st[t] = bisect_eps(X[idx[i]], kappa_T, **kw)
    return eps, kap, st
