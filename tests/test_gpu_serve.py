"""The render server: results of requests served together equal the same
requests rendered alone (bit for bit), edits apply to requests submitted
after them only, cancellation, and admission when the arena is small."""
import numpy as np
import pytest
import torch

import scenegen as sg
from tests._util import gpu_scene

pytestmark = pytest.mark.gpu


def _scene():
    return sg.room_scene(30000, (4.0, 3.0, 2.5), 4, seed=51, emissive_frac=0.01)


def _alone(gs, bvh, cam, p):
    from paper_2601_23065_amd.api import path_trace, resolve
    return resolve(path_trace(bvh, gs, cam, p), p.spp)


def _requests(scene):
    from paper_2601_23065_amd.api import Params
    cams = sg.interior_cameras(scene, 4, 16, 16, seed=9)
    sizes = [(40, 30), (64, 48), (17, 9), (33, 33)]
    out = []
    for i, (c, (w, h)) in enumerate(zip(cams, sizes)):
        cam = sg.Camera(c.eye, c.look_at, c.up, 70.0, w, h)
        out.append((cam, Params(spp=4 + 2 * i, max_depth=4, rr_start=2, camera_id=10 + i, seed=5)))
    return out


def test_mixed_equals_alone():
    from paper_2601_23065_amd.api import BVH, Server
    scene = _scene()
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    reqs = _requests(scene)
    srv = Server(gs, arena_bytes=64 << 20, max_live_requests=4, paths_per_launch=20000)
    tickets = [srv.submit(cam, p) for cam, p in reqs]
    res = [srv.wait(t) for t, _ in tickets]
    srv.close()
    for (cam, p), (t, out), r in zip(reqs, tickets, res):
        assert r["status"] == 0
        assert r["t_done"] >= r["t_admit"] >= r["t_submit"]
        ref = _alone(gs, bvh, cam, p)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (cam.width, cam.height)


def test_requests_with_different_segment_parameters():
    """Requests whose T_min, t_min or k_sigma differ are never traced in one
    launch with another request's values: each equals its render alone."""
    import dataclasses
    from paper_2601_23065_amd.api import BVH, Server
    scene = _scene()
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    reqs = _requests(scene)
    reqs = [(cam, dataclasses.replace(p, **kw)) for (cam, p), kw in
            zip(reqs, ({}, {"T_min": 1e-2}, {"t_min": 1e-2}, {"k_sigma": 2.0}))]
    srv = Server(gs, arena_bytes=64 << 20, max_live_requests=4, paths_per_launch=20000)
    tickets = [srv.submit(cam, p) for cam, p in reqs]
    res = [srv.wait(t) for t, _ in tickets]
    srv.close()
    for (cam, p), (t, out), r in zip(reqs, tickets, res):
        assert r["status"] == 0
        ref = _alone(gs, bvh, cam, p)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), p


def test_edits_are_ordered_with_submits():
    from paper_2601_23065_amd import EDIT_SCALE_RADIANCE
    from paper_2601_23065_amd.api import BVH, Server, apply_edit
    scene = _scene()
    gs = gpu_scene(scene)
    reqs = _requests(scene)
    cam, p = reqs[1]
    em = np.nonzero(scene.emissive > 0)[0]
    off = em[: em.size // 2].astype(np.int32)
    srv = Server(gs, arena_bytes=64 << 20, max_live_requests=4, paths_per_launch=20000)
    t_before, out_before = srv.submit(cam, p)
    t_edit = srv.edit(EDIT_SCALE_RADIANCE, off, (0.0, 0.0, 0.0))
    t_after, out_after = srv.submit(cam, p)
    rb, re, ra = srv.wait(t_before), srv.wait(t_edit), srv.wait(t_after)
    srv.close()
    assert rb["status"] == 0 and re["status"] == 0 and ra["status"] == 0
    assert ra["version"] == re["version"] != rb["version"]
    bvh = BVH(gs)
    ref_before = _alone(gs, bvh, cam, p)
    edited = gpu_scene(scene)
    apply_edit(edited, EDIT_SCALE_RADIANCE, torch.from_numpy(off).cuda(), (0.0, 0.0, 0.0))
    ref_after = _alone(edited, BVH(edited), cam, p)
    torch.cuda.synchronize()
    assert torch.equal(out_before, ref_before)
    assert torch.equal(out_after, ref_after)
    assert float(ref_after.sum()) < float(ref_before.sum())


def test_cancel_and_small_arena_admission():
    from paper_2601_23065_amd.api import Params, Server
    scene = _scene()
    gs = gpu_scene(scene)
    reqs = _requests(scene)
    from paper_2601_23065_amd import load
    lib = load()
    # room for the scene and about one 64x48 accumulator at a time
    need = lib.eag_serve_arena_bytes(scene.n, 3, 64 * 48 * 24 + 4096)
    srv = Server(gs, arena_bytes=need, max_live_requests=4, paths_per_launch=8192)
    big = sg.Camera(reqs[0][0].eye, reqs[0][0].look_at, (0.0, 0.0, 1.0), 70.0, 64, 48)
    t_big, _ = srv.submit(big, Params(spp=512, max_depth=4))
    srv.cancel(t_big)
    done = [srv.submit(cam, p) for cam, p in reqs]
    res = [srv.wait(t) for t, _ in done]
    r_big = srv.wait(t_big)
    srv.close()
    assert r_big["status"] == -5          # EAG_ERR_CANCELLED
    assert all(r["status"] == 0 for r in res)
