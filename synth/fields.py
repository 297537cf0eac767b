"""Seeded initial conditions: real spherical harmonics and noisy steady states."""
from __future__ import annotations

import math

import numpy as np
from scipy.special import sph_harm_y

__all__ = ["real_sph_harm", "random_sph_harm_ic", "schnakenberg_ic"]


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
