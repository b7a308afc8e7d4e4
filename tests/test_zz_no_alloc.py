"""The entry point that allocates nothing, eag_trace_rays_noalloc, against
eag_trace_rays (its allocating counterpart, same kernels): outputs, blended
hit lists, hit counts and traversal statistics equal bit for bit, on two
calls in a row, the second with a smaller scene and fewer rays; a scene
past the static scratch's size is rejected."""
import ctypes as C

import numpy as np
import pytest
import torch

import scenegen as sg
from tests._util import gpu_scene

pytestmark = pytest.mark.gpu
MAX_HITS = 96


def _buffers(m):
    # filled with values neither call writes, so that a missed write shows
    return (torch.full((12, m), -123.0, device="cuda"), torch.full((m, MAX_HITS), -7, dtype=torch.int32, device="cuda"),
            torch.full((m,), -7, dtype=torch.int32, device="cuda"), torch.full((m, 3), -7, dtype=torch.int32, device="cuda"))


def _both(scene, n_rays, seed, p):
    from paper_2601_23065_amd import _lib as L
    from paper_2601_23065_amd.api import BVH, _aligned, _bytes, _ptr
    lib = L.load()
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    O, D = sg.random_rays(scene, n_rays, seed=seed)
    o = torch.from_numpy(O.astype(np.float64)).cuda().contiguous()
    d = torch.from_numpy(D.astype(np.float64)).cuda().contiguous()
    sc, pc = gs.c(), p.c()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ref = _buffers(n_rays)
    ws = _bytes(lib.eag_trace_workspace_bytes(scene.n), gs.device)
    wp, wb = _aligned(ws)
    L.check(lib.eag_trace_rays(bvh.h, C.byref(sc), C.byref(pc), n_rays, _ptr(o), _ptr(d), _ptr(ref[0]), _ptr(ref[1]),
                               _ptr(ref[2]), MAX_HITS, _ptr(ref[3]), wp, wb, stream))
    got = _buffers(n_rays)
    L.check(lib.eag_trace_rays_noalloc(bvh.h, C.byref(sc), C.byref(pc), n_rays, _ptr(o), _ptr(d), _ptr(got[0]),
                                       _ptr(got[1]), _ptr(got[2]), MAX_HITS, _ptr(got[3]), stream))
    torch.cuda.synchronize()
    return ref, got


def test_noalloc_equals_trace_rays_on_two_calls():
    from paper_2601_23065_amd import _lib as L
    from paper_2601_23065_amd.api import Params
    L.check(L.load().eag_init())
    p = Params()
    for scene, n_rays, seed in ((sg.room_scene(60000, (4.0, 3.0, 2.5), 5, seed=9), 3000, 13),
                                (sg.cloud_scene(1500, seed=3), 700, 14)):
        ref, got = _both(scene, n_rays, seed, p)
        print(f"{scene.n} surfels, {n_rays} rays: mean hits {float(ref[2].float().mean()):.1f}")
        assert int(ref[2].sum()) > 0
        for a, b in zip(ref, got):
            assert torch.equal(a, b)


def test_noalloc_rejects_a_scene_past_its_scratch():
    import ctypes
    from paper_2601_23065_amd import EagError
    from paper_2601_23065_amd import _lib as L
    from paper_2601_23065_amd.api import BVH, Params, _ptr
    lib = L.load()
    L.check(lib.eag_init())
    scene = sg.cloud_scene((1 << 18) + 1, seed=2)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    o = torch.zeros((3, 4), dtype=torch.float64, device="cuda")
    d = torch.zeros((3, 4), dtype=torch.float64, device="cuda")
    d[2] = 1.0
    out = torch.zeros((12, 4), device="cuda")
    sc, pc = gs.c(), Params().c()
    with pytest.raises(EagError, match="2\\^18"):
        L.check(lib.eag_trace_rays_noalloc(bvh.h, ctypes.byref(sc), ctypes.byref(pc), 4, _ptr(o), _ptr(d), _ptr(out),
                                           None, None, 0, None, ctypes.c_void_p(0)))
