"""The C-ABI library loads and exports every symbol include/rt.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2309_11257_amd", "librt.so")


def declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b((?:rt|sg)_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = declared("rt.h")
    for n in ("rt_init_background", "rt_step", "rt_deposit_flux", "rt_split_merge"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="librt.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        for name in declared(h):
            assert hasattr(lib, name), f"{name} declared in {h} is not exported"


@pytest.mark.skipif(not os.path.exists(LIB), reason="librt.so not built")
def test_create_rejects_bad_config_without_touching_the_gpu():
    from paper_2309_11257_amd import _rt
    L = _rt.lib()
    h = ctypes.c_void_p()
    cfg = _rt.Config(0, 0, 0, 4, 4, 0, 1.0, 1.0, 1.0, 1.0, 10, _rt.ALLOC_FN(), _rt.FREE_FN(), None, None)
    assert L.rt_create(ctypes.byref(cfg), ctypes.byref(h)) == _rt.RT_E_ARG  # nx = 0
    cfg = _rt.Config(7, 0, 4, 4, 4, 0, 1.0, 1.0, 1.0, 1.0, 10, _rt.ALLOC_FN(), _rt.FREE_FN(), None, None)
    assert L.rt_create(ctypes.byref(cfg), ctypes.byref(h)) == _rt.RT_E_ARG  # geometry
    cfg = _rt.Config(0, 0, 4, 4, 4, 0, -1.0, 1.0, 1.0, 1.0, 10, _rt.ALLOC_FN(), _rt.FREE_FN(), None, None)
    assert L.rt_create(ctypes.byref(cfg), ctypes.byref(h)) == _rt.RT_E_ARG  # dx
    # single precision addresses ray fields with 32-bit byte offsets
    cfg = _rt.Config(0, _rt.RT_FP32, 4, 4, 4, 0, 1.0, 1.0, 1.0, 1.0, 1 << 30, _rt.ALLOC_FN(), _rt.FREE_FN(), None,
                     None)
    assert L.rt_create(ctypes.byref(cfg), ctypes.byref(h)) == _rt.RT_E_UNSUPPORTED
    assert L.rt_step(None, 1.0, 0) == _rt.RT_E_ARG
    assert L.rt_deposit_flux(None, None, None, 0) == _rt.RT_E_ARG
