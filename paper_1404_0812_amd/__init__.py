"""RBF-FD surface diffusion on MI355X: Python binding of librbffd.so.

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Arrays are torch CUDA tensors (device memory);
results come back as new tensors.  Each Context owns a HIP stream at the
default priority; calls order themselves after the caller's current stream
and make it wait for their results.
"""
from __future__ import annotations

import atexit
import ctypes
import weakref
from dataclasses import dataclass

import torch

from . import _lib

KERNELS = {"mq": 0, "imq": 1, "ga": 2}
EPS_MODES = {"fixed": 0, "given": 1, "bisect": 2, "learned": 3}
REACTIONS = {"none": 0, "schnakenberg": 1, "turing": 2}
PRECS = {"f64": 0, "f32": 1}

RBFFD_E_ARG, RBFFD_E_HIP, RBFFD_E_NOMEM, RBFFD_E_UNSUPPORTED, RBFFD_E_NONFINITE, RBFFD_E_NOCONV = -1, -2, -3, -4, -5, -6
ST_OK, ST_FALLBACK, ST_NO_BRACKET, ST_NONFINITE, ST_SINGULAR, ST_DUPLICATE, ST_BAD_INDEX, ST_BAD_NORMAL = range(8)


class RbffdError(RuntimeError):
    pass


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    return t.to(dtype).contiguous()


class Context:
    """A library context bound to its own HIP stream on the current device."""

    def __init__(self, device=None):
        self.lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.Stream(device=self.device)
        h = ctypes.c_void_p()
        rc = self.lib.rbffd_create(ctypes.byref(h), ctypes.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise RbffdError(f"rbffd_create failed ({rc})")
        self.h = h
        _LIVE_CTX.add(self)

    def close(self):
        if getattr(self, "h", None):
            self.lib.rbffd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc):
        if rc != 0:
            msg = self.lib.rbffd_last_error(self.h)
            raise RbffdError(f"rbffd error {rc}: {msg.decode() if msg else ''}")

    def enter(self, *tensors):
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        for t in tensors:
            if t is not None:
                t.record_stream(self.stream)

    def leave(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)


_DEFAULT = {}
_LIVE_OPS = weakref.WeakSet()
_LIVE_CTX = weakref.WeakSet()


@atexit.register
def _release_all():
    """Free operators, then contexts, while the HIP runtime is still up (the
    order in which the interpreter would otherwise collect them is arbitrary)."""
    for op in list(_LIVE_OPS):
        try:
            op.close()
        except Exception:
            pass
    for c in list(_LIVE_CTX):
        try:
            c.close()
        except Exception:
            pass


def default_context():
    dev = torch.cuda.current_device()
    if dev not in _DEFAULT:
        _DEFAULT[dev] = Context(dev)
    return _DEFAULT[dev]


def default_opts():
    o = _lib.WeightOpts()
    _lib.load().rbffd_default_opts(ctypes.byref(o))
    return o


def make_opts(n, kernel="mq", degree=2, eps_mode="fixed", eps=2.0, kappa_target=1e12, eps_tol=1e-4,
              bracket=(0.05, 20.0), band=(1e11, 1e13), rank_tol=1e-10, band_stop=False, max_expand=8):
    o = default_opts()
    o.n = int(n)
    o.kernel = KERNELS[kernel]
    o.poly_degree = int(degree)
    o.eps_mode = EPS_MODES[eps_mode]
    o.eps_fixed = float(eps)
    o.kappa_target = float(kappa_target)
    o.eps_tol = float(eps_tol)
    o.bracket_lo, o.bracket_hi = float(bracket[0]), float(bracket[1])
    o.band_lo, o.band_hi = float(band[0]), float(band[1])
    o.rank_tol = float(rank_tol)
    o.band_stop = 1 if band_stop else 0
    o.max_expand = int(max_expand)
    return o


def knn(xyz, n, ctx=None, with_perm=True):
    """Stencils (N x n int32, centre first) and the spatial order perm (N int32)."""
    ctx = ctx or default_context()
    xyz = _dev(xyz, torch.float64, "xyz")
    N = xyz.shape[0]
    idx = torch.empty((N, n), dtype=torch.int32, device=xyz.device)
    perm = torch.empty(N, dtype=torch.int32, device=xyz.device) if with_perm else None
    ctx.enter(xyz, idx, perm)
    ctx.check(ctx.lib.rbffd_knn(ctx.h, N, _ptr(xyz), int(n), _ptr(idx), _ptr(perm)))
    ctx.leave()
    return idx, perm


@dataclass
class Weights:
    idx: torch.Tensor
    w: torch.Tensor
    eps: torch.Tensor
    kappa: torch.Tensor
    status: torch.Tensor
    nevals: torch.Tensor


def build_weights_dd(xyz, nrm, n, idx=None, eps_in=None, ctx=None, **kw):
    """build_weights in double-double arithmetic (constant border, MQ/IMQ, n + 1 <= 48)."""
    return build_weights(xyz, nrm, n, idx=idx, eps_in=eps_in, ctx=ctx, _entry="rbffd_build_weights_dd", **kw)


def build_weights(xyz, nrm, n, idx=None, eps_in=None, ctx=None, _entry="rbffd_build_weights", **kw):
    """RBF-FD weights of the projected surface Laplacian (see make_opts for keywords)."""
    ctx = ctx or default_context()
    o = make_opts(n, **kw)
    xyz = _dev(xyz, torch.float64, "xyz")
    nrm = _dev(nrm, torch.float64, "nrm")
    N = xyz.shape[0]
    dev = xyz.device
    idx_in = _dev(idx, torch.int32, "idx") if idx is not None else None
    eps_t = _dev(eps_in, torch.float64, "eps_in") if eps_in is not None else None
    idx_out = idx_in if idx_in is not None else torch.empty((N, n), dtype=torch.int32, device=dev)
    w = torch.empty((N, n), dtype=torch.float64, device=dev)
    eps = torch.empty(N, dtype=torch.float64, device=dev)
    kap = torch.empty(N, dtype=torch.float64, device=dev)
    st = torch.empty(N, dtype=torch.int32, device=dev)
    ne = torch.empty(N, dtype=torch.int32, device=dev)
    ctx.enter(xyz, nrm, idx_in, eps_t, idx_out, w, eps, kap, st, ne)
    ctx.check(getattr(ctx.lib, _entry)(ctx.h, N, _ptr(xyz), _ptr(nrm), ctypes.byref(o), _ptr(idx_in),
                                       _ptr(eps_t), _ptr(idx_out) if idx_in is None else ctypes.c_void_p(0),
                                       _ptr(w), _ptr(eps), _ptr(kap), _ptr(st), _ptr(ne)))
    ctx.leave()
    return Weights(idx_out, w, eps, kap, st, ne)


def kappa(xyz, idx, eps_in, n=None, ctx=None, **kw):
    """kappa_2 of each stencil's bordered local matrix at eps_in."""
    ctx = ctx or default_context()
    idx = _dev(idx, torch.int32, "idx")
    n = idx.shape[1] if n is None else n
    o = make_opts(n, **kw)
    xyz = _dev(xyz, torch.float64, "xyz")
    eps_t = _dev(eps_in, torch.float64, "eps_in")
    N = xyz.shape[0]
    out = torch.empty(N, dtype=torch.float64, device=xyz.device)
    ctx.enter(xyz, idx, eps_t, out)
    ctx.check(ctx.lib.rbffd_kappa(ctx.h, N, _ptr(xyz), ctypes.byref(o), _ptr(idx), _ptr(eps_t), _ptr(out)))
    ctx.leave()
    return out


# ---------------------------------------------------------------- batched ----

def _tuning_array(tuning):
    arr = (_lib.BatchTuning * _lib.BUCKETS)()
    for b, t in enumerate(tuning):
        arr[b].stencils_per_item = int(t["stencils_per_item"])
        arr[b].groups_per_cu = int(t["groups_per_cu"])
        arr[b].order = int(t["order"])
        arr[b].us_per_stencil = float(t.get("us_per_stencil", 0.0))
    return arr


def _batch_surfaces(surfaces, eps_in, dev):
    """Descriptors and output tensors of a batched build (surfaces: list of (xyz, nrm, n[, idx]))."""
    descs = (_lib.Surface * len(surfaces))()
    keep, outs = [], []
    for s, surf in enumerate(surfaces):
        xyz, nrm, n = surf[0], surf[1], int(surf[2])
        idx = surf[3] if len(surf) > 3 else None
        xyz = _dev(xyz, torch.float64, "xyz")
        nrm = _dev(nrm, torch.float64, "nrm")
        N = xyz.shape[0]
        idx_in = _dev(idx, torch.int32, "idx") if idx is not None else None
        e_in = _dev(eps_in[s], torch.float64, "eps_in") if eps_in is not None else None
        idx_out = idx_in if idx_in is not None else torch.empty((N, n), dtype=torch.int32, device=dev)
        r = Weights(idx_out, torch.empty((N, n), dtype=torch.float64, device=dev),
                    torch.empty(N, dtype=torch.float64, device=dev), torch.empty(N, dtype=torch.float64, device=dev),
                    torch.empty(N, dtype=torch.int32, device=dev), torch.empty(N, dtype=torch.int32, device=dev))
        d = descs[s]
        d.N, d.n = N, n
        d.xyz, d.nrm = xyz.data_ptr(), nrm.data_ptr()
        d.idx = idx_in.data_ptr() if idx_in is not None else None
        d.eps_in = e_in.data_ptr() if e_in is not None else None
        d.idx_out = idx_out.data_ptr() if idx_in is None else None
        d.w, d.eps, d.kappa = r.w.data_ptr(), r.eps.data_ptr(), r.kappa.data_ptr()
        d.status, d.nevals = r.status.data_ptr(), r.nevals.data_ptr()
        keep += [xyz, nrm, idx_in, e_in, idx_out, r.w, r.eps, r.kappa, r.status, r.nevals]
        outs.append(r)
    return descs, keep, outs


def autotune_batched(surfaces, eps_in=None, cache_path=None, retune=False, ctx=None, **kw):
    """Schedules (one dict per bucket) chosen by the library's autotuner; see build_weights_batched."""
    ctx = ctx or default_context()
    o = make_opts(int(surfaces[0][2]) if surfaces else 31, **kw)
    descs, keep, _ = _batch_surfaces(surfaces, eps_in, ctx.device)
    out = (_lib.BatchTuning * _lib.BUCKETS)()
    ctx.enter(*keep)
    path = cache_path.encode() if cache_path else None
    ctx.check(ctx.lib.rbffd_autotune_batched(ctx.h, len(surfaces), descs, ctypes.byref(o), path, int(bool(retune)),
                                             out))
    ctx.leave()
    return [dict(stencils_per_item=t.stencils_per_item, groups_per_cu=t.groups_per_cu, order=t.order,
                 us_per_stencil=t.us_per_stencil) for t in out]


def build_weights_batched(surfaces, eps_in=None, tuning=None, ctx=None, **kw):
    """Weights of many surfaces in persistent launches.

    surfaces: list of (xyz, nrm, n) or (xyz, nrm, n, idx) with each surface's
    own stencil size n; eps_in: per-surface eps tensors for given/learned
    modes; tuning: per-bucket schedules from autotune_batched (None: the
    library default).  Other keywords as make_opts (n is per surface).
    Returns one Weights per surface."""
    ctx = ctx or default_context()
    o = make_opts(int(surfaces[0][2]) if surfaces else 31, **kw)
    descs, keep, outs = _batch_surfaces(surfaces, eps_in, ctx.device)
    tun = _tuning_array(tuning) if tuning is not None else None
    ctx.enter(*keep)
    ctx.check(ctx.lib.rbffd_build_weights_batched(ctx.h, len(surfaces), descs, ctypes.byref(o), tun))
    ctx.leave()
    return outs


class Operator:
    """Sparse L_X built from caller-order stencils and weights.

    Operator(idx, w, perm) holds one surface; Operator.batched([(idx, w,
    perm), ...]) holds many (block-diagonal, state arrays concatenated by
    surface)."""

    def __init__(self, idx, w, perm=None, ctx=None):
        self.ctx = ctx or default_context()
        idx = _dev(idx, torch.int32, "idx")
        w = _dev(w, torch.float64, "w")
        perm = _dev(perm, torch.int32, "perm") if perm is not None else None
        self.N, self.n = idx.shape
        h = ctypes.c_void_p()
        self.ctx.enter(idx, w, perm)
        self.ctx.check(self.ctx.lib.rbffd_op_create(self.ctx.h, self.N, self.n, _ptr(idx), _ptr(w), _ptr(perm),
                                                    ctypes.byref(h)))
        self.ctx.leave()
        self.h = h
        _LIVE_OPS.add(self)

    @classmethod
    def batched(cls, parts, ctx=None):
        self = cls.__new__(cls)
        self.ctx = ctx or default_context()
        descs = (_lib.OpSurface * len(parts))()
        keep = []
        for s, part in enumerate(parts):
            idx = _dev(part[0], torch.int32, "idx")
            w = _dev(part[1], torch.float64, "w")
            perm = _dev(part[2], torch.int32, "perm") if len(part) > 2 and part[2] is not None else None
            descs[s].N, descs[s].n = idx.shape
            descs[s].idx, descs[s].w = idx.data_ptr(), w.data_ptr()
            descs[s].perm = perm.data_ptr() if perm is not None else None
            keep += [idx, w, perm]
        self.N = sum(int(d.N) for d in descs)
        self.n = max(int(d.n) for d in descs)
        h = ctypes.c_void_p()
        self.ctx.enter(*keep)
        self.ctx.check(self.ctx.lib.rbffd_op_create_batched(self.ctx.h, len(parts), descs, ctypes.byref(h)))
        self.ctx.leave()
        self.h = h
        _LIVE_OPS.add(self)
        return self

    def close(self):
        if getattr(self, "h", None):
            if getattr(self.ctx, "h", None):  # the context must still exist
                self.ctx.lib.rbffd_op_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self):
        """(slices, slices with an LDS-staged halo, rows in them, halo entries)."""
        v = [ctypes.c_int64() for _ in range(4)]
        self.ctx.check(self.ctx.lib.rbffd_op_stats(self.h, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def apply(self, u, prec="f64"):
        u = _dev(u, torch.float64, "u")
        out = torch.empty_like(u)
        self.ctx.enter(u, out)
        self.ctx.check(self.ctx.lib.rbffd_apply(self.ctx.h, self.h, PRECS[prec], _ptr(u), _ptr(out)))
        self.ctx.leave()
        return out

    def step(self, state, dt, nsteps, prec="f64", D=(1.0,), reaction="none", params=(), graph_steps=0,
             forcing=None, t0=0.0, lam=0.0):
        """Advance state (S x N float64, S = 1 or 2) by nsteps RK4 steps; returns the new state.

        forcing (S x N float64, optional): f_s(t, x_i) = exp(lam t) forcing[s, i],
        the state being at time t0 on entry.  Raises RbffdError if the state
        becomes non-finite."""
        st = _dev(state, torch.float64, "state").clone()
        if st.dim() == 1:
            st = st.unsqueeze(0)
        S = st.shape[0]
        Darr = (ctypes.c_double * max(2, len(D)))(*[float(x) for x in D])
        prm = (ctypes.c_double * 5)(*([float(x) for x in params] + [0.0] * (5 - len(params))))
        if forcing is None:
            self.ctx.enter(st)
            rc = self.ctx.lib.rbffd_step(self.ctx.h, self.h, S, _ptr(st), PRECS[prec], Darr,
                                         REACTIONS[reaction], prm, float(dt), int(nsteps), int(graph_steps))
        else:
            F = _dev(forcing, torch.float64, "forcing").reshape(st.shape)
            self.ctx.enter(st, F)
            rc = self.ctx.lib.rbffd_step_forced(self.ctx.h, self.h, S, _ptr(st), PRECS[prec], Darr,
                                                REACTIONS[reaction], prm, float(dt), int(nsteps), int(graph_steps),
                                                float(t0), _ptr(F), float(lam))
        self.ctx.leave()
        self.ctx.check(rc)
        return st

    def step_imex(self, state, dt, nsteps, order=2, D=(1.0,), reaction="none", params=(), history=None,
                  forcing=None, t0=0.0, lam=0.0, tol=1e-12, maxit=200):
        """Semi-implicit BDF steps (FP64).  history: (order-1) x S x N states at
        t0 - dt, t0 - 2 dt, ... or None.  Returns (state, iterations, worst
        relative residual)."""
        st = _dev(state, torch.float64, "state").clone()
        if st.dim() == 1:
            st = st.unsqueeze(0)
        S = st.shape[0]
        Darr = (ctypes.c_double * max(2, len(D)))(*[float(x) for x in D])
        prm = (ctypes.c_double * 5)(*([float(x) for x in params] + [0.0] * (5 - len(params))))
        H = _dev(history, torch.float64, "history").contiguous() if history is not None else None
        F = _dev(forcing, torch.float64, "forcing").reshape(st.shape) if forcing is not None else None
        its = ctypes.c_int64()
        res = ctypes.c_double()
        self.ctx.enter(st, H, F)
        rc = self.ctx.lib.rbffd_step_imex(self.ctx.h, self.h, S, _ptr(st), Darr, REACTIONS[reaction], prm, float(dt),
                                          int(nsteps), int(order), _ptr(H), float(t0), _ptr(F), float(lam),
                                          float(tol), int(maxit), ctypes.byref(its), ctypes.byref(res))
        self.ctx.leave()
        self.ctx.check(rc)
        return st, its.value, res.value


# ------------------------------------------------------------ learned eps ----

MLP_IN = 128
MLP_HIDDEN = 128
MLP_PARAMS = _lib.MLP_PARAMS


def mlp_init(seed=0, n_in=98, bias_out=0.0):
    """He-uniform initial parameters (FP32 numpy); padded input columns are zero."""
    import numpy as np

    rng = np.random.default_rng(seed)
    H, F = MLP_HIDDEN, MLP_IN
    W1 = np.zeros((H, F))
    W1[:, :n_in] = rng.uniform(-1, 1, size=(H, n_in)) * np.sqrt(6.0 / n_in)
    W2 = rng.uniform(-1, 1, size=(H, H)) * np.sqrt(6.0 / H)
    w3 = rng.uniform(-1, 1, size=H) * np.sqrt(6.0 / H) * 0.1
    p = np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), w3, [bias_out]])
    assert p.size == MLP_PARAMS
    return p.astype(np.float32)


def mlp_features(xyz, nrm, idx, ctx=None):
    """BF16 features (N x 128, stored as int16) and stencil radii (N, FP64)."""
    ctx = ctx or default_context()
    xyz = _dev(xyz, torch.float64, "xyz")
    nrm = _dev(nrm, torch.float64, "nrm")
    idx = _dev(idx, torch.int32, "idx")
    N, n = idx.shape
    feats = torch.empty((N, MLP_IN), dtype=torch.int16, device=xyz.device)
    rho = torch.empty(N, dtype=torch.float64, device=xyz.device)
    ctx.enter(xyz, nrm, idx, feats, rho)
    ctx.check(ctx.lib.rbffd_mlp_features(ctx.h, N, _ptr(xyz), _ptr(nrm), _ptr(idx), n, _ptr(feats), _ptr(rho)))
    ctx.leave()
    return feats, rho


def mlp_forward(params, feats, ctx=None):
    ctx = ctx or default_context()
    params = _dev(params, torch.float32, "params")
    feats = _dev(feats, torch.int16, "feats")
    y = torch.empty(feats.shape[0], dtype=torch.float32, device=feats.device)
    ctx.enter(params, feats, y)
    ctx.check(ctx.lib.rbffd_mlp_forward(ctx.h, _ptr(params), feats.shape[0], _ptr(feats), _ptr(y)))
    ctx.leave()
    return y


def mlp_grad(params, feats, target, ctx=None):
    ctx = ctx or default_context()
    params = _dev(params, torch.float32, "params")
    feats = _dev(feats, torch.int16, "feats")
    target = _dev(target, torch.float32, "target")
    g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=feats.device)
    loss = torch.empty(1, dtype=torch.float32, device=feats.device)
    ctx.enter(params, feats, target, g, loss)
    ctx.check(ctx.lib.rbffd_mlp_grad(ctx.h, _ptr(params), feats.shape[0], _ptr(feats), _ptr(target), _ptr(g),
                                     _ptr(loss)))
    ctx.leave()
    return g, loss


class MLP:
    """The shape-parameter regressor with its Adam state, on the device."""

    def __init__(self, params, ctx=None):
        self.ctx = ctx or default_context()
        dev = torch.device("cuda", self.ctx.device.index)
        self.params = torch.as_tensor(params, dtype=torch.float32).to(dev).contiguous().clone()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0

    def train(self, feats, target, steps, batch=4096, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, seed=1):
        feats = _dev(feats, torch.int16, "feats")
        target = _dev(target, torch.float32, "target")
        o = _lib.TrainOpts(lr, betas[0], betas[1], eps, int(batch), int(steps), int(seed), int(self.step))
        losses = torch.empty(max(1, steps), dtype=torch.float32, device=feats.device)
        self.ctx.enter(self.params, self.m, self.v, feats, target, losses)
        self.ctx.check(self.ctx.lib.rbffd_mlp_train(self.ctx.h, _ptr(self.params), _ptr(self.m), _ptr(self.v),
                                                    feats.shape[0], _ptr(feats), _ptr(target), ctypes.byref(o),
                                                    _ptr(losses)))
        self.ctx.leave()
        self.step += steps
        return losses[:steps]

    def forward(self, feats):
        return mlp_forward(self.params, feats, ctx=self.ctx)

    def predict_eps(self, xyz, nrm, idx):
        xyz = _dev(xyz, torch.float64, "xyz")
        nrm = _dev(nrm, torch.float64, "nrm")
        idx = _dev(idx, torch.int32, "idx")
        N, n = idx.shape
        eps = torch.empty(N, dtype=torch.float64, device=xyz.device)
        self.ctx.enter(self.params, xyz, nrm, idx, eps)
        self.ctx.check(self.ctx.lib.rbffd_predict_eps(self.ctx.h, _ptr(self.params), N, _ptr(xyz), _ptr(nrm),
                                                      _ptr(idx), n, _ptr(eps)))
        self.ctx.leave()
        return eps
