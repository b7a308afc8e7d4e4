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
    assert lib.eag_abi_version() == 2
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


def test_host_validation_of_the_baking_stage0_and_edit_calls(lib):
    from paper_2601_23065_amd import _lib
    C = ctypes
    fake = C.c_void_p(0x1000)      # never dereferenced: every call below fails validation first
    # Adam: the step counts from 1, the rates lie in [0, 1)
    a = _lib.Adam(0.01, 0.9, 0.999, 1e-15)
    assert lib.eag_adam_step(fake, fake, fake, fake, 10, C.byref(a), 0, None) == -1
    assert b"step" in lib.eag_last_error()
    bad = _lib.Adam(0.01, 1.0, 0.999, 1e-15)
    assert lib.eag_adam_step(fake, fake, fake, fake, 10, C.byref(bad), 1, None) == -1
    assert lib.eag_adam_step(None, fake, fake, fake, 10, C.byref(a), 1, None) == -1
    # loss: null buffers, negative counts
    assert lib.eag_bake_loss(None, fake, 10, fake, fake, None) == -1
    assert lib.eag_bake_loss(fake, fake, -1, fake, fake, None) == -1
    # motions: a zero quaternion, a non-finite pivot
    g = _lib.SurfelsOut()
    g.n = 10
    g.pos = g.rot = fake
    zero = (C.c_float * 4)(0, 0, 0, 0)
    one = (C.c_float * 4)(1, 0, 0, 0)
    z3 = (C.c_float * 3)(0, 0, 0)
    nan3 = (C.c_float * 3)(float("nan"), 0, 0)
    assert lib.eag_move_surfels(C.byref(g), fake, 1, zero, z3, z3, None) == -1
    assert b"quaternion" in lib.eag_last_error()
    assert lib.eag_move_surfels(C.byref(g), fake, 1, one, nan3, z3, None) == -1
    assert lib.eag_move_surfels(C.byref(g), None, 3, one, z3, z3, None) == -1
    assert lib.eag_delete_surfels(C.byref(g), fake, -2, None) == -1
    # duplication: the destination must hold n + count surfels
    s = _lib.Surfels()
    s.n = 10
    for k in ("pos", "rot", "scale", "opacity", "albedo", "radiance", "emissive"):
        setattr(s, k, fake)
    d = _lib.SurfelsOut()
    d.n = 12
    for k in ("pos", "rot", "scale", "opacity", "albedo", "radiance", "emissive"):
        setattr(d, k, fake)
    assert lib.eag_duplicate_surfels(C.byref(s), fake, 3, C.byref(d), one, z3, z3, None) == -1
    assert b"n + count" in lib.eag_last_error()
    # stage-0 loss workspace is a pure size query
    cam = _lib.Camera()
    cam.width, cam.height = 16, 8
    assert lib.eag_stage0_loss_workspace_bytes(C.byref(cam), 2) >= 16 * 8 * 2 * 16
    assert lib.eag_stage0_loss_workspace_bytes(None, 1) == 0
    assert lib.eag_bake_workspace_bytes(0, C.byref(cam), 1) == 0


def test_host_validation_of_the_emitter_sampling_calls(lib):
    from paper_2601_23065_amd import _lib
    C = ctypes
    fake = C.c_void_p(0x1000)      # never dereferenced: every call below fails validation first
    s = _lib.Surfels()
    s.n = 10
    for k in ("pos", "rot", "scale", "opacity", "albedo", "radiance", "emissive"):
        setattr(s, k, fake)
    p = _lib.TraceParams()
    lib.eag_default_params(C.byref(p))
    out = C.c_void_p()
    assert lib.eag_emitters_bytes(0) == 0 and lib.eag_emitters_bytes(1000) > 1000 * 17 * 4
    p.tau_E = -0.5
    assert lib.eag_build_emitters(C.byref(s), C.byref(p), 0.0, fake, 1 << 20, fake, 1 << 20, None, C.byref(out)) == -1
    assert b"tau_E" in lib.eag_last_error()
    lib.eag_default_params(C.byref(p))
    p.k_sigma = 4.0
    assert lib.eag_build_emitters(C.byref(s), C.byref(p), 0.0, fake, 1 << 20, fake, 1 << 20, None, C.byref(out)) == -1
    assert b"k_sigma" in lib.eag_last_error()
    lib.eag_default_params(C.byref(p))
    for bad in (0.3, -1.0, 4096.0):
        assert lib.eag_build_emitters(C.byref(s), C.byref(p), bad, fake, 1 << 20, fake, 1 << 20, None,
                                      C.byref(out)) == -1
        assert b"power of two" in lib.eag_last_error()
    odd = C.c_void_p(0x1010)
    assert lib.eag_build_emitters(C.byref(s), C.byref(p), 0.5, odd, 1 << 20, fake, 1 << 20, None, C.byref(out)) == -1
    assert b"aligned" in lib.eag_last_error()
    assert lib.eag_emitters_get_info(None, None, None, None) == -1
    assert lib.eag_path_trace_mis(None, C.byref(s), None, None, C.byref(p), 0, 1, None, None, None, 0, None) == -1
    lib.eag_emitters_destroy(None)
