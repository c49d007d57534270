"""CPU checks of the C ABI boundary: the library loads, exports every entry
point include/ctm.h declares, and the binding refuses to run without it."""
import ctypes
import os
import re

import pytest

from paper_1906_02220_amd import ctm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ctm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("ctm_context_create", "ctm_env_init_tensor", "ctm_env_init_purification",
                     "ctm_sweep", "ctm_norm", "ctm_bond_metric", "ctm_expect"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(ctm.LIB_PATH), "build the library first (python -m paper_1906_02220_amd.build)"
    lib = ctypes.CDLL(ctm.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) == set(ctm.SIGNATURES)


def test_binding_fails_loudly_without_library(tmp_path):
    saved = ctm._lib
    try:
        ctm._lib = None
        with pytest.raises(ImportError):
            ctm.load_library(str(tmp_path / "missing.so"))
    finally:
        ctm._lib = saved


def test_opts_struct_matches_header_defaults():
    o = ctm.default_opts()
    assert o.precision == ctm.CTM_PREC_F64
    assert o.eps_cut == 1e-12
    assert o.seed == 0x5eed


def test_context_without_gpu_reports_device_error():
    """On a machine without a gfx950 device, context creation must fail with
    CTM_EDEVICE rather than fall back to anything."""
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        pytest.skip("a GPU is present")
    lib = ctm.load_library()
    h = ctypes.c_void_p()
    rc = lib.ctm_context_create(0, ctypes.byref(h))
    assert rc == ctm.CTM_EDEVICE
