"""ctypes declarations of librbffd.so (the C ABI in include/rbffd.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbffd.so")

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p


class WeightOpts(ctypes.Structure):
    _fields_ = [
        ("n", c_int32),
        ("kernel", c_int32),
        ("poly_degree", c_int32),
        ("eps_mode", c_int32),
        ("eps_fixed", c_double),
        ("kappa_target", c_double),
        ("eps_tol", c_double),
        ("bracket_lo", c_double),
        ("bracket_hi", c_double),
        ("band_lo", c_double),
        ("band_hi", c_double),
        ("rank_tol", c_double),
        ("band_stop", c_int32),
        ("max_expand", c_int32),
    ]


class TrainOpts(ctypes.Structure):
    _fields_ = [
        ("lr", c_double),
        ("beta1", c_double),
        ("beta2", c_double),
        ("adam_eps", c_double),
        ("batch", c_int32),
        ("steps", c_int32),
        ("seed", ctypes.c_uint64),
        ("step0", c_int64),
    ]


class Surface(ctypes.Structure):
    _fields_ = [
        ("N", c_int64),
        ("n", c_int32),
        ("reserved", c_int32),
        ("xyz", c_void_p),
        ("nrm", c_void_p),
        ("idx", c_void_p),
        ("eps_in", c_void_p),
        ("idx_out", c_void_p),
        ("w", c_void_p),
        ("eps", c_void_p),
        ("kappa", c_void_p),
        ("status", c_void_p),
        ("nevals", c_void_p),
    ]


class BatchTuning(ctypes.Structure):
    _fields_ = [
        ("stencils_per_item", c_int32),
        ("groups_per_cu", c_int32),
        ("order", c_int32),
        ("reserved", c_int32),
        ("us_per_stencil", c_double),
    ]


class OpSurface(ctypes.Structure):
    _fields_ = [
        ("N", c_int64),
        ("n", c_int32),
        ("reserved", c_int32),
        ("idx", c_void_p),
        ("w", c_void_p),
        ("perm", c_void_p),
    ]


BUCKETS = 2
MLP_PARAMS = 33153

# name -> (restype, argtypes)
SIGNATURES = {
    "rbffd_default_opts": (None, [ctypes.POINTER(WeightOpts)]),
    "rbffd_create": (c_int32, [ctypes.POINTER(c_void_p), c_void_p]),
    "rbffd_destroy": (c_int32, [c_void_p]),
    "rbffd_last_error": (ctypes.c_char_p, [c_void_p]),
    "rbffd_knn": (c_int32, [c_void_p, c_int64, c_void_p, c_int32, c_void_p, c_void_p]),
    "rbffd_build_weights": (c_int32, [c_void_p, c_int64, c_void_p, c_void_p, ctypes.POINTER(WeightOpts),
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p]),
    "rbffd_build_weights_dd": (c_int32, [c_void_p, c_int64, c_void_p, c_void_p, ctypes.POINTER(WeightOpts),
                                         c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                         c_void_p]),
    "rbffd_kappa": (c_int32, [c_void_p, c_int64, c_void_p, ctypes.POINTER(WeightOpts), c_void_p, c_void_p,
                              c_void_p]),
    "rbffd_op_create": (c_int32, [c_void_p, c_int64, c_int32, c_void_p, c_void_p, c_void_p,
                                  ctypes.POINTER(c_void_p)]),
    "rbffd_op_destroy": (c_int32, [c_void_p]),
    "rbffd_op_stats": (c_int32, [c_void_p, ctypes.POINTER(c_int64), ctypes.POINTER(c_int64), ctypes.POINTER(c_int64),
                                 ctypes.POINTER(c_int64)]),
    "rbffd_op_create_batched": (c_int32, [c_void_p, c_int32, ctypes.POINTER(OpSurface), ctypes.POINTER(c_void_p)]),
    "rbffd_build_weights_batched": (c_int32, [c_void_p, c_int32, ctypes.POINTER(Surface), ctypes.POINTER(WeightOpts),
                                              ctypes.POINTER(BatchTuning)]),
    "rbffd_autotune_batched": (c_int32, [c_void_p, c_int32, ctypes.POINTER(Surface), ctypes.POINTER(WeightOpts),
                                         ctypes.c_char_p, c_int32, ctypes.POINTER(BatchTuning)]),
    "rbffd_apply": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "rbffd_apply_noalloc": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "rbffd_step": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_int32, ctypes.POINTER(c_double), c_int32,
                             ctypes.POINTER(c_double), c_double, c_int64, c_int32]),
    "rbffd_step_imex": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, ctypes.POINTER(c_double), c_int32,
                                  ctypes.POINTER(c_double), c_double, c_int64, c_int32, c_void_p, c_double, c_void_p,
                                  c_double, c_double, c_int32, ctypes.POINTER(c_int64), ctypes.POINTER(c_double)]),
    "rbffd_step_forced": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_int32, ctypes.POINTER(c_double),
                                    c_int32, ctypes.POINTER(c_double), c_double, c_int64, c_int32, c_double,
                                    c_void_p, c_double]),
    "rbffd_mlp_features": (c_int32, [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_int32, c_void_p,
                                     c_void_p]),
    "rbffd_mlp_forward": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
    "rbffd_mlp_grad": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]),
    "rbffd_mlp_train": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p,
                                  ctypes.POINTER(TrainOpts), c_void_p]),
    "rbffd_predict_eps": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_int32,
                                    c_void_p]),
}

_LIB = None


def load():
    """Load librbffd.so; raises if it has not been built (no fallback exists)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1404_0812_amd.build` "
                "(there is no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB
