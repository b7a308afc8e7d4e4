"""The C ABI: every function include/eag.h declares is exported by the
built library and bound by the Python layer; host-side validation and
workspace queries need no GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eag.h")
LIB = os.path.join(ROOT, "paper_2601_23065_amd", "libeag.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eag_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_2601_23065_amd import _lib
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header(lib):
    from paper_2601_23065_amd import _lib
    assert set(declared_functions()) <= set(_lib.SIGNATURES)
    assert lib.missing_symbols == []


def test_struct_sizes_match_the_header(lib):
    from paper_2601_23065_amd import _lib
    # sizes the C compiler gives the structs (x86-64 SysV)
    assert ctypes.sizeof(_lib.TraceParams) == 56
    assert ctypes.sizeof(_lib.Camera) == 48
    assert ctypes.sizeof(_lib.Surfels) == 64


def test_defaults_and_queries(lib):
    from paper_2601_23065_amd import _lib
    p = _lib.TraceParams()
    lib.eag_default_params(ctypes.byref(p))
    assert (p.spp, p.max_depth, p.rr_start, p.kbuf) == (4, 5, 3, 16)
    assert abs(p.tau_E - 0.1) < 1e-7 and abs(p.T_min - 1e-4) < 1e-10
    assert p.depth_quantum == 2.0 ** -13
    assert lib.eag_abi_version() == 1
    assert lib.eag_bvh_bytes(0) == 0 and lib.eag_bvh_bytes(1000) > 1000 * 48
    assert lib.eag_build_workspace_bytes(1000) > 0
    assert lib.eag_trace_workspace_bytes(1000) >= 1000 * 32


def test_host_validation_without_gpu(lib):
    from paper_2601_23065_amd import _lib
    s = _lib.Surfels()
    s.n = 0
    out = ctypes.c_void_p()
    st = lib.eag_build_bvh(ctypes.byref(s), None, 0, None, 0, None, ctypes.byref(out))
    assert st == -1 and b"surfel count" in lib.eag_last_error()
    # a resolve with bad sizes is rejected before any launch
    assert lib.eag_accum_resolve(None, 10, 1, None, None) == -1
    e = _lib.Edit()
    e.kind = 99
    a = _lib.SurfelAttrs()
    a.n = 10
    assert lib.eag_apply_edit(ctypes.byref(e), ctypes.byref(a), None) == -1
