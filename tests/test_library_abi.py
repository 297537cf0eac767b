"""CPU-side checks of the C ABI: the library loads and exports every declared symbol.

No compute call is made (there is no GPU here).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbffd.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rbffd_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("rbffd_create", "rbffd_destroy", "rbffd_build_weights", "rbffd_step", "rbffd_knn",
                 "rbffd_kappa", "rbffd_op_create", "rbffd_apply"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1404_0812_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("librbffd.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    # every declared symbol has a ctypes signature in the binding
    assert set(declared()) <= set(_lib.SIGNATURES)


def test_opts_struct_layout_matches_defaults():
    from paper_1404_0812_amd import _lib

    lib = _lib.load()
    o = _lib.WeightOpts()
    lib.rbffd_default_opts(ctypes.byref(o))   # host-only function
    assert (o.n, o.kernel, o.poly_degree, o.eps_mode) == (31, 0, 2, 0)
    assert o.eps_fixed == 2.0 and o.kappa_target == 1e12 and o.eps_tol == 1e-4
    assert (o.bracket_lo, o.bracket_hi, o.band_lo, o.band_hi) == (0.05, 20.0, 1e11, 1e13)
    assert o.rank_tol == 1e-10 and o.band_stop == 0 and o.max_expand == 8


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1404_0812_amd import _lib

    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_LIB", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib.load()
