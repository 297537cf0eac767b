"""Seeded initial conditions: real spherical harmonics and noisy steady states."""
from __future__ import annotations

import math

import numpy as np
from scipy.special import sph_harm_y

__all__ = ["real_sph_harm", "random_sph_harm_ic", "schnakenberg_ic", "sphere_heat_series",
           "sphere_forced", "torus_forced", "bump_centres"]


def real_sph_harm(l: int, m: int, X: np.ndarray) -> np.ndarray:
    """Orthonormal real spherical harmonic Y_l^m at the directions of X (N x 3).

    theta is the colatitude and phi the longitude.  m > 0 takes sqrt(2) times
    the real part of the complex harmonic, m < 0 sqrt(2) times the imaginary
    part of the order-|m| harmonic, and m = 0 the complex harmonic itself.
    """
    r = np.linalg.norm(X, axis=1)
    theta = np.arccos(np.clip(X[:, 2] / r, -1.0, 1.0))
    phi = np.arctan2(X[:, 1], X[:, 0])
    Y = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return math.sqrt(2.0) * Y.real
    if m < 0:
        return math.sqrt(2.0) * Y.imag
    return Y.real.copy()


def random_sph_harm_ic(X: np.ndarray, terms: int = 8, lmax: int = 10, seed: int = 1):
    """Sum of `terms` real harmonics, l ~ U{1..lmax}, m ~ U{-l..l}, coefficients N(0,1).

    Returns (u0, [(l, m, coef), ...]).  l = 0 is excluded so that every term decays.
    """
    rng = np.random.default_rng(seed)
    spec = []
    u = np.zeros(len(X))
    for _ in range(terms):
        l = int(rng.integers(1, lmax + 1))
        m = int(rng.integers(-l, l + 1))
        c = float(rng.standard_normal())
        spec.append((l, m, c))
        u += c * real_sph_harm(l, m, X)
    return u, spec


def schnakenberg_ic(N: int, a: float = 0.1, b: float = 0.9, amp: float = 0.01, seed: int = 2):
    """Steady state (a+b, b/(a+b)^2) plus U(-amp, amp) noise on both species."""
    rng = np.random.default_rng(seed)
    us = a + b
    vs = b / (a + b) ** 2
    u = us + rng.uniform(-amp, amp, size=N)
    v = vs + rng.uniform(-amp, amp, size=N)
    return u, v


def sphere_heat_series(X: np.ndarray, t: float, terms: int = 30) -> np.ndarray:
    """Exact heat-equation solution on the unit sphere used in Sec. 6.1:
    u(t) = 20/(3 pi) sum_{l=1}^{terms} exp(-l^2/9) exp(-l(l+1) t) Y_l^l,
    with the real harmonic of degree l and order l (the series is truncated
    after 30 terms, as in the paper)."""
    u = np.zeros(len(X))
    for l in range(1, terms + 1):
        u += math.exp(-l * l / 9.0) * math.exp(-l * (l + 1) * t) * real_sph_harm(l, l, X)
    return 20.0 / (3.0 * math.pi) * u


def bump_centres(kind: str, count: int = 23, seed: int = 9) -> np.ndarray:
    """Seeded centres of the manufactured solutions of Sec. 6: `count` points
    uniform on the unit sphere (kind "sphere", count x 3) or angle pairs
    (phi_k, lam_k) uniform in [-pi, pi]^2 (kind "torus", count x 2)."""
    rng = np.random.default_rng(seed)
    if kind == "sphere":
        v = rng.standard_normal((count, 3))
        return v / np.linalg.norm(v, axis=1, keepdims=True)
    return rng.uniform(-math.pi, math.pi, size=(count, 2))


def sphere_forced(X: np.ndarray, centres: np.ndarray):
    """Manufactured solution of the forced diffusion problem on the unit
    sphere (Sec. 6.1, eq. sph_forced): u(t, x) = exp(-5t) g(x) with g a sum
    of bumps exp(-10 (1 - xi_k . x)) about the centres xi_k.

    Returns (g, F): the forcing is f(t, x) = exp(-5t) F(x) with
    F = -5 g - Lap_S g, so that u_t = Lap_S u + f.  For a bump
    h = exp(-10 (1 - cos theta)), theta the angle to its centre,
    Lap_S h = h'' + cot(theta) h' = (100 sin^2 theta - 20 cos theta) h."""
    c = X @ centres.T                      # cos theta_k, N x count
    h = np.exp(-10.0 * (1.0 - c))
    g = h.sum(axis=1)
    lap = ((100.0 * (1.0 - c * c) - 20.0 * c) * h).sum(axis=1)
    return g, -5.0 * g - lap


def torus_forced(phi: np.ndarray, lam: np.ndarray, centres: np.ndarray, a: float = 9.0, b: float = 3.0):
    """Manufactured solution of the forced diffusion problem on the torus of
    eq. torus (Sec. 6.1, eq. torus_forced): u(t) = exp(-5t) g with
    g = sum_k exp(-a^2 (1 - cos(lam - lam_k)) - b^2 (1 - cos(phi - phi_k))),
    a = 9, b = 3.

    Returns (g, F), F = -5 g - Lap g, with the intrinsic Laplacian of the
    torus given in Sec. 6.1: Lap g = g_ll / rho^2 + (9 / rho) d/dphi (rho g_p),
    rho = 1 + cos(phi) / 3."""
    P = phi[:, None] - centres[None, :, 0]
    L = lam[:, None] - centres[None, :, 1]
    h = np.exp(-a * a * (1.0 - np.cos(L)) - b * b * (1.0 - np.cos(P)))
    h_ll = (-a * a * np.cos(L) + a ** 4 * np.sin(L) ** 2) * h
    h_p = -b * b * np.sin(P) * h
    h_pp = (-b * b * np.cos(P) + b ** 4 * np.sin(P) ** 2) * h
    rho = 1.0 + np.cos(phi) / 3.0
    rho_p = -np.sin(phi) / 3.0
    g = h.sum(axis=1)
    lap = (h_ll.sum(axis=1) / rho ** 2 + 9.0 * (h_pp.sum(axis=1) + (rho_p / rho) * h_p.sum(axis=1)))
    return g, -5.0 * g - lap
