"""Seeded node sets with unit normals on closed surfaces.

The paper's own node sets (maximal-determinant nodes, the red blood cell,
the double torus, the bumpy sphere, Frog and Bunny point clouds) are not
available, so these generators stand in for them with the same kinds of
structure: quasi-uniform nodes on the sphere (Fibonacci spiral), a jittered
parametric grid on the torus of Sec. 6 (eq. torus), ellipsoids, and a
Poisson-disk-thinned point cloud on an implicit surface (standing in for the
reconstructed point clouds of Sec. 7.2).

Every function returns ``(X, nrm)`` as float64 arrays of shape ``(N, 3)``.
"""
from __future__ import annotations

import math

import numpy as np

GENERATOR_VERSION = 2  # part of the cache key; bump when a generator changes

__all__ = [
    "fibonacci_sphere",
    "jittered_torus",
    "torus_grid_for_count",
    "ellipsoid",
    "blob",
    "planar_patch",
    "surface_batch",
    "icosahedral_sphere",
    "staggered_torus",
    "torus_angles",
    "cached",
]


def fibonacci_sphere(N: int, radius: float = 1.0):
    """Fibonacci-spiral nodes on a sphere: z_i = 1-(2i+1)/N, lon_i = i*pi*(3-sqrt 5).

    Normals are the exact outward unit normals (the node direction).
    """
    i = np.arange(N, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / N
    lon = i * (math.pi * (3.0 - math.sqrt(5.0)))
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    U = np.stack([s * np.cos(lon), s * np.sin(lon), z], axis=1)
    return radius * U, U.copy()


def jittered_torus(n_phi: int, n_lam: int, R: float = 1.0, r: float = 1.0 / 3.0,
                   jitter: float = 0.25, seed: int = 3):
    """Parametric torus (R + r cos phi) cos lam, (R + r cos phi) sin lam, r sin phi.

    A tensor grid of n_phi x n_lam cells over [-pi, pi)^2 in (phi, lam), each
    node moved by U(-jitter, jitter) cells in both directions (seeded).
    Normals are analytic: (cos phi cos lam, cos phi sin lam, sin phi).
    """
    rng = np.random.default_rng(seed)
    dphi = 2.0 * math.pi / n_phi
    dlam = 2.0 * math.pi / n_lam
    P, L = np.meshgrid(np.arange(n_phi, dtype=np.float64), np.arange(n_lam, dtype=np.float64),
                       indexing="ij")
    P = P.ravel()
    L = L.ravel()
    jp = rng.uniform(-jitter, jitter, size=P.shape)
    jl = rng.uniform(-jitter, jitter, size=L.shape)
    phi = -math.pi + (P + 0.5 + jp) * dphi
    lam = -math.pi + (L + 0.5 + jl) * dlam
    c = R + r * np.cos(phi)
    X = np.stack([c * np.cos(lam), c * np.sin(lam), r * np.sin(phi)], axis=1)
    nrm = np.stack([np.cos(phi) * np.cos(lam), np.cos(phi) * np.sin(lam), np.sin(phi)], axis=1)
    return X, nrm


def torus_grid_for_count(N: int, R: float, r: float):
    """(n_phi, n_lam) with n_phi * n_lam close to N and cells roughly square."""
    aspect = R / r  # mean toroidal / poloidal circumference
    n_phi = max(3, int(round(math.sqrt(N / aspect))))
    n_lam = max(3, int(round(N / n_phi)))
    return n_phi, n_lam


def ellipsoid(N: int, a: float, b: float, c: float):
    """Fibonacci nodes mapped to the ellipsoid x^2/a^2 + y^2/b^2 + z^2/c^2 = 1.

    Normals are the normalised gradient (x/a^2, y/b^2, z/c^2).
    """
    U, _ = fibonacci_sphere(N)
    X = U * np.array([a, b, c])
    g = X / np.array([a * a, b * b, c * c])
    return X, g / np.linalg.norm(g, axis=1, keepdims=True)


def _blob_f_grad(P, C, s2):
    d = P[:, None, :] - C[None, :, :]
    e = np.exp(-np.sum(d * d, axis=2) / s2)
    f = e.sum(axis=1)
    g = -2.0 / s2 * np.einsum("ij,ijk->ik", e, d)
    return f, g


def blob(N: int, seed: int = 4, ncentres: int = 8, s2: float = 0.3, level: float = 0.5,
         oversample: float = 3.0):
    """Point cloud on the implicit surface sum_i exp(-|x-c_i|^2/s2) = level.

    Centres are U([-1,1]^3) (seeded).  Candidates drawn uniformly in a box
    around the centres are kept near the level set, Newton-projected onto it
    until |f - level| < 1e-13, and thinned to a Poisson-disk set (no two nodes
    closer than half the grid spacing, see _poisson_disk) of exactly N nodes.
    Normals are -grad f / |grad f| (outward, since f decreases outwards).
    """
    rng = np.random.default_rng(seed)
    C = rng.uniform(-1.0, 1.0, size=(ncentres, 3))
    lo = C.min(axis=0) - 1.2
    hi = C.max(axis=0) + 1.2
    pts = []
    have = 0
    need = int(oversample * N) + 1000
    chunk = 1 << 20
    while have < need:
        P = rng.uniform(lo, hi, size=(chunk, 3))
        f, _ = _blob_f_grad(P, C, s2)
        P = P[np.abs(f - level) < 0.25]
        done = np.zeros(len(P), dtype=bool)
        for _ in range(60):
            act = np.flatnonzero(~done)
            if len(act) == 0:
                break
            Q = P[act]
            f, g = _blob_f_grad(Q, C, s2)
            gg = np.sum(g * g, axis=1)
            gg = np.where(gg > 1e-8, gg, np.inf)  # flat spots: leave in place, rejected below
            step = ((f - level) / gg)[:, None] * g
            step_n = np.linalg.norm(step, axis=1)
            # damp long steps so that candidates do not jump between sheets
            scale = np.minimum(1.0, 0.1 / np.maximum(step_n, 1e-300))[:, None]
            P[act] = Q - scale * step
            done[act] = (np.abs(f - level) < 1e-14) | (step_n < 1e-15) | ~np.isfinite(gg)
        f, _ = _blob_f_grad(P, C, s2)
        P = P[np.abs(f - level) < 1e-13]
        pts.append(P)
        have += len(P)
    P = np.concatenate(pts)[:need]
    P = P[rng.permutation(len(P))]
    X = _poisson_disk(P, N, lo, hi, rng)
    _, g = _blob_f_grad(X, C, s2)
    nrm = -g / np.linalg.norm(g, axis=1, keepdims=True)
    return np.ascontiguousarray(X), np.ascontiguousarray(nrm)


def _grid_first(P, lo, ext, h):
    key = np.floor((P - lo) / h).astype(np.int64)
    dims = np.floor(ext / h).astype(np.int64) + 2
    lin = (key[:, 0] * dims[1] + key[:, 1]) * dims[2] + key[:, 2]
    _, first = np.unique(lin, return_index=True)
    return np.sort(first)


def _mis(Q, r, prio):
    """Maximal independent set of the graph 'closer than r' (parallel rounds:
    a node joins when its priority beats every undecided neighbour's)."""
    from scipy.spatial import cKDTree

    pairs = cKDTree(Q).query_pairs(r, output_type="ndarray")
    keep = np.zeros(len(Q), dtype=bool)
    und = np.ones(len(Q), dtype=bool)
    i, j = pairs[:, 0], pairs[:, 1]
    while und.any():
        act = und[i] & und[j]
        mx = np.full(len(Q), -1.0)
        np.maximum.at(mx, i[act], prio[j[act]])
        np.maximum.at(mx, j[act], prio[i[act]])
        win = und & (prio > mx)
        keep |= win
        und &= ~win
        lose = np.zeros(len(Q), dtype=bool)
        lose[j[win[i] & und[j]]] = True
        lose[i[win[j] & und[i]]] = True
        und &= ~lose
    return np.flatnonzero(keep)


def _poisson_disk(P, N, lo, hi, rng):
    """Exactly N of the candidates P with no two closer than h/2, where h is a
    grid spacing: keep the first candidate of each grid cell, drop close pairs
    by a maximal independent set, shrink h until at least N remain, then keep
    a seeded random N of them."""
    ext = hi - lo
    h_lo, h_hi = 1e-6, float(ext.max())
    for _ in range(60):  # largest h whose grid holds ~1.4 N candidates
        h = math.sqrt(h_lo * h_hi)
        if len(_grid_first(P, lo, ext, h)) >= 1.4 * N:
            h_lo = h
        else:
            h_hi = h
        if h_hi / h_lo < 1.0 + 1e-3:
            break
    h = h_lo
    for _ in range(20):
        k = _grid_first(P, lo, ext, h)
        Q = P[k]
        keep = _mis(Q, 0.5 * h, rng.random(len(Q)))
        if len(keep) >= N:
            sel = np.sort(rng.permutation(len(keep))[:N])
            return Q[keep[sel]]
        h *= 0.95
    raise RuntimeError("blob: not enough candidates for the Poisson-disk set")


def planar_patch(n_side: int, spacing: float = 0.125, seed: int | None = None, jitter: float = 0.0):
    """A planar patch in z = 0 (normals +z): a lattice, optionally jittered."""
    g = (np.arange(n_side, dtype=np.float64) - (n_side - 1) / 2.0) * spacing
    Xg, Yg = np.meshgrid(g, g, indexing="ij")
    X = np.stack([Xg.ravel(), Yg.ravel(), np.zeros(n_side * n_side)], axis=1)
    if seed is not None and jitter > 0:
        rng = np.random.default_rng(seed)
        X[:, :2] += rng.uniform(-jitter, jitter, size=(len(X), 2)) * spacing
    nrm = np.zeros_like(X)
    nrm[:, 2] = 1.0
    return X, nrm


def surface_batch(count: int = 64, seed: int = 5, n_min: int = 2000, n_max: int = 60000,
                  stencil_sizes=(31, 50, 70, 101)):
    """A seeded batch of spheres, tori and ellipsoids of uneven size.

    Sphere radius, ellipsoid semi-axes and torus major radius are U[0.5, 2];
    the torus minor radius is R*U[0.2, 0.45].  N is floor(exp(U[ln n_min,
    ln n_max])) and the stencil size is drawn uniformly from stencil_sizes.
    Returns a list of dicts with keys kind, X, nrm, n, params.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind = ("sphere", "torus", "ellipsoid")[int(rng.integers(0, 3))]
        N = int(math.floor(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        n = int(stencil_sizes[int(rng.integers(0, len(stencil_sizes)))])
        if kind == "sphere":
            rad = float(rng.uniform(0.5, 2.0))
            X, nrm = fibonacci_sphere(N, rad)
            params = {"radius": rad}
        elif kind == "torus":
            R = float(rng.uniform(0.5, 2.0))
            r = R * float(rng.uniform(0.2, 0.45))
            n_phi, n_lam = torus_grid_for_count(N, R, r)
            X, nrm = jittered_torus(n_phi, n_lam, R, r, seed=int(rng.integers(0, 2**31)))
            params = {"R": R, "r": r}
        else:
            ax = rng.uniform(0.5, 2.0, size=3)
            X, nrm = ellipsoid(N, *ax)
            params = {"axes": ax.tolist()}
        out.append({"kind": kind, "X": X, "nrm": nrm, "n": n, "params": params})
    return out


def icosahedral_sphere(level: int):
    """Icosahedral nodes on the unit sphere (the node sets of Sec. 6.1).

    The 12 vertices of an icosahedron; every triangle is split into four by
    its edge midpoints, pushed out to the sphere, `level` times.  N = 10 4^level
    + 2 (642, 2562, 10242, 40962 for levels 3..6).  Normals are the exact unit
    normals (the node directions).
    """
    g = (1.0 + math.sqrt(5.0)) / 2.0
    V = [(-1, g, 0), (1, g, 0), (-1, -g, 0), (1, -g, 0), (0, -1, g), (0, 1, g), (0, -1, -g), (0, 1, -g),
         (g, 0, -1), (g, 0, 1), (-g, 0, -1), (-g, 0, 1)]
    V = [np.array(v, dtype=np.float64) / math.sqrt(1.0 + g * g) for v in V]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        mid = {}

        def midpoint(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in mid:
                v = V[a] + V[b]
                V.append(v / np.linalg.norm(v))
                mid[key] = len(V) - 1
            return mid[key]

        F2 = []
        for a, b, c in F:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            F2 += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = F2
    X = np.array(V)
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    return X, X.copy()


def staggered_torus(m: int, R: float = 1.0, r: float = 1.0 / 3.0):
    """The staggered grid on the torus of Sec. 6.1 (eq. torus): m angles in
    phi and 3m in lam, equally spaced on [-pi, pi) (the endpoint pi dropped),
    their direct product, and the same grid shifted by half a cell in both
    angles (pi/m in phi, pi/(3m) in lam).  N = 6 m^2 (600, 2400, 5400,
    21600, 38400 for m = 10, 20, 30, 60, 80).  Normals are analytic."""
    phi0 = -math.pi + 2.0 * math.pi * np.arange(m) / m
    lam0 = -math.pi + 2.0 * math.pi * np.arange(3 * m) / (3 * m)
    out_p, out_l = [], []
    for dp, dl in ((0.0, 0.0), (math.pi / m, math.pi / (3 * m))):
        P, L = np.meshgrid(phi0 + dp, lam0 + dl, indexing="ij")
        out_p.append(P.ravel())
        out_l.append(L.ravel())
    phi = np.concatenate(out_p)
    lam = np.concatenate(out_l)
    c = R + r * np.cos(phi)
    X = np.stack([c * np.cos(lam), c * np.sin(lam), r * np.sin(phi)], axis=1)
    nrm = np.stack([np.cos(phi) * np.cos(lam), np.cos(phi) * np.sin(lam), np.sin(phi)], axis=1)
    return X, nrm


def torus_angles(X: np.ndarray, R: float = 1.0):
    """Intrinsic angles (phi, lam) of points on the torus of eq. torus."""
    lam = np.arctan2(X[:, 1], X[:, 0])
    phi = np.arctan2(X[:, 2], np.hypot(X[:, 0], X[:, 1]) - R)
    return phi, lam


def cached(fn, *args, **kw):
    """Call a generator, keeping its arrays in a .npz under $TMPDIR for reuse
    by later processes on the same machine (plain arrays, no pickles)."""
    import hashlib
    import os
    import tempfile

    key = hashlib.sha1(repr((GENERATOR_VERSION, fn.__name__, args, sorted(kw.items()))).encode()).hexdigest()[:16]
    d = os.path.join(os.environ.get("TMPDIR", tempfile.gettempdir()), "rbffd_synth_cache")
    path = os.path.join(d, f"{fn.__name__}_{key}.npz")
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            return z["X"], z["nrm"]
    X, nrm = fn(*args, **kw)
    os.makedirs(d, exist_ok=True)
    tmp = path + f".{os.getpid()}.tmp.npz"
    np.savez(tmp, X=X, nrm=nrm)
    os.replace(tmp, path)
    return X, nrm
