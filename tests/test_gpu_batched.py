"""Batched weights over many surfaces (persistent launches, autotuned
schedule) and the block-diagonal operator of many surfaces.

The batched build runs the same per-stencil routine as the plain build, so
its outputs are compared bit for bit with per-surface rbffd_build_weights;
the plain build is itself held to the oracle in test_gpu_parity.py, and a
sample of the batch is checked against the oracle here too.  The batched
operator is compared with the per-surface operators (bit for bit: the same
sums in the same order) and, for one surface, with the oracle.
"""
import json
import os

import numpy as np
import pytest
import torch

from oracle.shape import bisect_eps
from oracle.stepper import laplacian_apply
from oracle.weights import build_weights as oracle_weights
from synth import surface_batch

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def batch():
    """Nine surfaces: spheres, tori, ellipsoids; n in {31, 50, 70, 101}; N ragged."""
    surfs = surface_batch(count=9, seed=17, n_min=400, n_max=2500)
    return [(dev(s["X"]), dev(s["nrm"]), s["n"]) for s in surfs], surfs


def _same(a, b):
    return torch.equal(a, b) or (torch.isnan(a).equal(torch.isnan(b)) and
                                 torch.equal(torch.nan_to_num(a, nan=0.0), torch.nan_to_num(b, nan=0.0)))


@pytest.mark.parametrize("tuning", [None, "odd"])
def test_batched_matches_plain_bitwise(lib, batch, tuning):
    surfs, meta = batch
    print(f"[batched] {len(surfs)} surfaces n={[s[2] for s in surfs]} N={[s[0].shape[0] for s in surfs]} "
          f"tuning={tuning}", flush=True)
    tun = None
    if tuning == "odd":  # item sizes that leave ragged tails, one group per CU, given order
        tun = [dict(stencils_per_item=7, groups_per_cu=1, order=1), dict(stencils_per_item=3, groups_per_cu=1, order=1)]
    got = lib.build_weights_batched(surfs, tuning=tun, eps_mode="bisect", kappa_target=1e12)
    for (X, nrm, n), g in zip(surfs, got):
        ref = lib.build_weights(X, nrm, n, eps_mode="bisect", kappa_target=1e12)
        torch.cuda.synchronize()
        assert torch.equal(g.idx, ref.idx)
        assert _same(g.w, ref.w)
        assert torch.equal(g.eps, ref.eps)
        assert _same(g.kappa, ref.kappa)
        assert torch.equal(g.status, ref.status)
        assert torch.equal(g.nevals, ref.nevals)


def test_batched_sample_against_oracle(lib, batch):
    surfs, meta = batch
    got = lib.build_weights_batched(surfs, eps_mode="bisect", kappa_target=1e12)
    rng = np.random.default_rng(5)
    for s in (0, 4, 8):
        X, nrm, n = meta[s]["X"], meta[s]["nrm"], meta[s]["n"]
        idx = host(got[s].idx)
        eg = host(got[s].eps)
        for i in rng.choice(len(X), 4, replace=False):
            eo, _, _, sto = bisect_eps(X[idx[i]], 1e12)
            assert sto == 0 and abs(eg[i] - eo) <= 2e-4, (s, i, eg[i], eo)
        rows = rng.choice(len(X), 4, replace=False)
        wo = oracle_weights(X, nrm, idx, eg, rows=rows)
        wg = host(got[s].w)[rows]
        k = host(got[s].kappa)[rows]
        err = np.linalg.norm(wg - wo, axis=1) / np.linalg.norm(wo, axis=1)
        assert np.all(err <= np.maximum(1e-9, 0.5 * k * 2.0 ** -53)), err


def test_autotune_and_cache(lib, batch, tmp_path):
    surfs, _ = batch
    path = str(tmp_path / "tune.json")
    t1 = lib.autotune_batched(surfs, cache_path=path, retune=True, eps_mode="bisect", kappa_target=1e12)
    assert len(t1) == 2
    for t in t1:
        assert t["stencils_per_item"] >= 1 and t["groups_per_cu"] in (1, 2) and t["order"] in (0, 1)
        assert t["us_per_stencil"] > 0
    data = json.load(open(path))
    assert len(data) == 2 and all("bucket" in k for k in data)
    # cached: same schedule without timing again
    t2 = lib.autotune_batched(surfs, cache_path=path, eps_mode="bisect", kappa_target=1e12)
    assert [(t["stencils_per_item"], t["groups_per_cu"], t["order"]) for t in t1] == \
           [(t["stencils_per_item"], t["groups_per_cu"], t["order"]) for t in t2]
    got = lib.build_weights_batched(surfs, tuning=t2, eps_mode="bisect", kappa_target=1e12)
    ref = lib.build_weights_batched(surfs, eps_mode="bisect", kappa_target=1e12)
    for g, r in zip(got, ref):
        assert _same(g.w, r.w)


def test_batched_errors(lib, batch):
    surfs, _ = batch
    X, nrm, _ = surfs[0]
    with pytest.raises(lib.RbffdError, match="surface 1"):
        lib.build_weights_batched([surfs[0], (X, nrm, 125)], eps_mode="fixed", eps=2.0)
    with pytest.raises(lib.RbffdError):
        lib.build_weights_batched(surfs[:2], tuning=[dict(stencils_per_item=0, groups_per_cu=1, order=0)] * 2)
    assert lib.build_weights_batched([], eps_mode="fixed") == []


@pytest.fixture(scope="module")
def batch_ops(lib, batch):
    surfs, meta = batch
    res = lib.build_weights_batched(surfs[:4], eps_mode="bisect", kappa_target=1e10)
    parts = []
    for (X, nrm, n), r in zip(surfs[:4], res):
        _, perm = lib.knn(X, n)
        parts.append((r.idx, r.w, perm))
    return parts, meta[:4]


def test_batched_operator_apply_matches_per_surface(lib, batch_ops):
    parts, meta = batch_ops
    bop = lib.Operator.batched(parts)
    Ns = [p[0].shape[0] for p in parts]
    rng = np.random.default_rng(2)
    u = [rng.standard_normal(N) for N in Ns]
    ucat = dev(np.concatenate(u))
    for prec in ("f64", "f32"):
        got = host(bop.apply(ucat, prec=prec))
        off = 0
        for (idx, w, perm), us, N in zip(parts, u, Ns):
            ref = host(lib.Operator(idx, w, perm).apply(dev(us), prec=prec))
            assert np.array_equal(got[off:off + N], ref), prec
            off += N
    # one surface against the oracle's CSR operator (FP64)
    idx, w, _ = parts[1]
    ref = laplacian_apply(host(idx), host(w), u[1])
    g = host(bop.apply(ucat, prec="f64"))[Ns[0]:Ns[0] + Ns[1]]
    assert np.max(np.abs(g - ref)) <= 1e-13 * np.max(np.abs(host(w)).sum(axis=1) * np.max(np.abs(u[1])))


def test_batched_operator_step_matches_per_surface(lib, batch_ops):
    parts, _ = batch_ops
    bop = lib.Operator.batched(parts)
    Ns = [p[0].shape[0] for p in parts]
    rng = np.random.default_rng(3)
    u0 = [rng.standard_normal((2, N)) for N in Ns]
    state = dev(np.concatenate(u0, axis=1))
    params = (0.1, 0.9, 50.0)
    for prec in ("f64", "f32"):
        got = host(bop.step(state, 1e-6, 23, prec=prec, D=(1.0, 10.0), reaction="schnakenberg", params=params,
                            graph_steps=5))
        assert np.all(np.isfinite(got))
        off = 0
        for (idx, w, perm), us, N in zip(parts, u0, Ns):
            ref = host(lib.Operator(idx, w, perm).step(dev(us), 1e-6, 23, prec=prec, D=(1.0, 10.0),
                                                       reaction="schnakenberg", params=params, graph_steps=5))
            assert np.array_equal(got[:, off:off + N], ref), prec
            off += N


def test_batched_given_and_learned_modes_bitwise(lib, batch):
    """Per-surface eps arrays (given) and proposals with the kappa-band check
    (learned) go through the batched launch exactly as through the plain one."""
    surfs, _ = batch
    rng = np.random.default_rng(21)
    eps_in = []
    for X, nrm, n in surfs:
        idx, _ = lib.knn(X, n)
        rho = torch.sqrt(((X[idx.long()] - X[idx[:, :1].long()]) ** 2).sum(-1).max(1).values)
        eps_in.append(torch.as_tensor(rng.uniform(0.4, 0.9, X.shape[0])).cuda() / rho)
    for mode, kw in (("given", {}), ("learned", {"kappa_target": 1e12, "band": (1e11, 1e13)})):
        got = lib.build_weights_batched(surfs, eps_in=eps_in, eps_mode=mode, **kw)
        for (X, nrm, n), e, g in zip(surfs, eps_in, got):
            ref = lib.build_weights(X, nrm, n, eps_in=e, eps_mode=mode, **kw)
            torch.cuda.synchronize()
            assert _same(g.w, ref.w) and torch.equal(g.eps, ref.eps) and torch.equal(g.status, ref.status), mode


def test_batched_edge_surfaces(lib):
    """An empty surface, a tiny ragged one (N = 130), and the largest system
    (n = 118 with the degree-2 border, m = 128) in one batch."""
    from synth import ellipsoid, fibonacci_sphere

    X0 = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    Xa, na = fibonacci_sphere(130)
    Xb, nb = ellipsoid(1500, 1.0, 0.7, 0.5)
    surfs = [(X0, X0, 31), (dev(Xa), dev(na), 20), (dev(Xb), dev(nb), 118)]
    got = lib.build_weights_batched(surfs, eps_mode="bisect", kappa_target=1e10)
    assert got[0].w.shape == (0, 31)
    for (X, nrm, n), g in zip(surfs[1:], got[1:]):
        ref = lib.build_weights(X, nrm, n, eps_mode="bisect", kappa_target=1e10)
        torch.cuda.synchronize()
        assert _same(g.w, ref.w) and torch.equal(g.eps, ref.eps)
        assert torch.all(g.status == 0)
    # the largest system against the oracle on a few rows
    idx = host(got[2].idx)
    eg = host(got[2].eps)
    rows = np.array([0, 700, 1499])
    wo = oracle_weights(Xb, nb, idx, eg, rows=rows)
    wg = host(got[2].w)[rows]
    k = host(got[2].kappa)[rows]
    err = np.linalg.norm(wg - wo, axis=1) / np.linalg.norm(wo, axis=1)
    assert np.all(err <= np.maximum(1e-9, 0.5 * k * 2.0 ** -53)), err


def test_autotune_cache_file_read_by_a_new_process(lib, batch, tmp_path):
    """A second process reads the schedule from the JSON file written by the
    first (no timing: the cached per-stencil time comes back unchanged)."""
    import subprocess
    import sys

    surfs, meta = batch
    path = str(tmp_path / "tune2.json")
    t1 = lib.autotune_batched(surfs[:3], cache_path=path, retune=True, eps_mode="bisect", kappa_target=1e12)
    np.savez(str(tmp_path / "surf.npz"), **{f"X{i}": m["X"] for i, m in enumerate(meta[:3])},
             **{f"N{i}": m["nrm"] for i, m in enumerate(meta[:3])}, n=np.array([m["n"] for m in meta[:3]]))
    code = f"""
import json, sys, numpy as np, torch
sys.path.insert(0, {repr(str(__import__('pathlib').Path(__file__).resolve().parents[1]))})
import paper_1404_0812_amd as rb
z = np.load({repr(str(tmp_path / 'surf.npz'))})
surfs = [(torch.as_tensor(z[f'X{{i}}']).cuda(), torch.as_tensor(z[f'N{{i}}']).cuda(), int(z['n'][i])) for i in range(3)]
t = rb.autotune_batched(surfs, cache_path={repr(path)}, eps_mode='bisect', kappa_target=1e12)
print(json.dumps(t))
"""
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    t2 = json.loads(out.stdout.strip().splitlines()[-1])
    for a, b in zip(t1, t2):
        assert (a["stencils_per_item"], a["groups_per_cu"], a["order"]) == (b["stencils_per_item"], b["groups_per_cu"], b["order"])
        assert abs(a["us_per_stencil"] - b["us_per_stencil"]) <= 1e-5 * max(1.0, a["us_per_stencil"])


def test_batch64_sample_against_oracle(lib):
    """The 64-surface batch at its full size (N log-uniform in [2000, 60000],
    n in {31, 50, 70, 101}, bisection to kappa_T = 1e12): two seeded rows of
    every surface against the oracle's bisection and weights."""
    import math

    from oracle.shape import stencil_kappa

    meta = surface_batch()
    surfs = [(dev(s["X"]), dev(s["nrm"]), s["n"]) for s in meta]
    print(f"[batch64] {sum(len(s['X']) for s in meta)} stencils", flush=True)
    got = lib.build_weights_batched(surfs, eps_mode="bisect", kappa_target=1e12)
    rng = np.random.default_rng(64)
    worst = 0.0
    for s, m in enumerate(meta):
        X, nrm, n = m["X"], m["nrm"], m["n"]
        idx = host(got[s].idx)
        eg, st = host(got[s].eps), host(got[s].status)
        assert np.all(st == 0), (s, np.unique(st))
        rows = rng.choice(len(X), 2, replace=False)
        for i in rows:
            eo, _, _, sto = bisect_eps(X[idx[i]], 1e12)
            assert sto == 0
            if abs(eg[i] - eo) > 2e-4:  # a decision at kappa(mid) ~ kappa_T within FP64's evaluation error
                k = stencil_kappa(X[idx[i]], eg[i])
                print(f"[batch64] surface {s} ({m['kind']}, n={n}) row {i}: eps {eg[i]:.6f} vs {eo:.6f}, "
                      f"oracle kappa at gpu eps {k:.6e}", flush=True)
                assert abs(math.log(k / 1e12)) < 1e-3
        wo = oracle_weights(X, nrm, idx, eg, rows=rows)
        k = np.array([stencil_kappa(X[idx[i]], eg[i]) for i in rows])
        wg = host(got[s].w)[rows]
        err = np.linalg.norm(wg - wo, axis=1) / np.linalg.norm(wo, axis=1)
        worst = max(worst, float(np.max(err / (k * 2.0 ** -53))))
        assert np.all(err <= np.maximum(1e-9, 0.5 * k * 2.0 ** -53)), (s, err, k)
    print(f"[batch64] weights: max err/(kappa u) {worst:.4f}", flush=True)
