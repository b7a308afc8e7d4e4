"""Parity at the benchmark's full size: the 1M-surfel 8x6x3 m room with 40
boxes, one 1024x768 camera, 64 spp, max depth 5, Russian roulette from depth
3, traced in one launch over all samples (the configuration the benchmark
times). Sampled pixels are compared with the oracle's sum over their 64
paths, computed one path at a time; a pixel is compared only when none of
its paths carries a decision-margin flag."""
import multiprocessing as mp
import os

import numpy as np
import pytest

import scenegen as sg
from tests._util import gpu_scene, rel_err

pytestmark = pytest.mark.gpu

_ORACLE = {}


def _oracle_job(args):
    import oracle.render as R
    pixel, samples = args
    out = R.path_trace(_ORACLE["sc"], _ORACLE["cam"], _ORACLE["prm"], pixels=np.array([pixel]), samples=samples)
    return pixel, out["value"][0].sum(axis=0), int(out["flags"][0].astype(bool).any())


def test_path_trace_full_size_sampled_pixels():
    from oracle import Params as OParams
    from oracle.tracer import Scene64
    from paper_2601_23065_amd.api import BVH, Params, path_trace

    scene, cams, cfg = sg.config(3)
    cam = cams[0]
    p = Params(spp=cfg["spp"], max_depth=cfg["max_depth"], rr_start=cfg["rr_start"], seed=0, camera_id=0)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    acc = path_trace(bvh, gs, cam, p, 0, p.spp)
    got = acc.cpu().numpy().reshape(-1, 3).astype(np.float64) / 2.0 ** 32

    rng = np.random.default_rng(11)
    pixels = rng.choice(cam.width * cam.height, 3, replace=False)
    _ORACLE.update(sc=Scene64(scene), cam=cam,
                   prm=OParams(spp=p.spp, max_depth=p.max_depth, rr_start=p.rr_start, seed=0, camera_id=0))
    jobs = [(int(px), list(range(s0, s0 + 8))) for px in pixels for s0 in range(0, p.spp, 8)]
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        res = pool.map(_oracle_job, jobs, chunksize=1)
    ref = {int(px): np.zeros(3) for px in pixels}
    flagged = {int(px): 0 for px in pixels}
    for px, v, f in res:
        ref[px] += v
        flagged[px] |= f
    ok = [px for px in ref if not flagged[px]]
    print(f"pixels {list(ref)} flagged {flagged} gpu {[got[px] for px in ok]} oracle {[ref[px] for px in ok]}")
    assert len(ok) >= 2
    err = rel_err(np.stack([got[px] for px in ok]), np.stack([ref[px] for px in ok]))
    assert err.max() <= 1e-4


def _oracle_pixels(scene, cam, prm, pixels, samples, chunk):
    from oracle.tracer import Scene64
    _ORACLE.update(sc=Scene64(scene), cam=cam, prm=prm)
    jobs = [(int(px), list(range(s0, min(s0 + chunk, samples)))) for px in pixels for s0 in range(0, samples, chunk)]
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        res = pool.map(_oracle_job, jobs, chunksize=1)
    ref = {int(px): np.zeros(3) for px in pixels}
    flagged = {int(px): 0 for px in pixels}
    for px, v, f in res:
        ref[px] += v
        flagged[px] |= f
    return ref, flagged


def test_rooms5m_after_edit_and_refit_sampled_pixels():
    """The 5M-surfel three-room scene at 1920x1080, depth 8, RR from 3:
    radiance zeroed on half the emitters and albedo changed on 10% of the
    surfels on the device, the BVH refitted, then 8 samples traced in one
    launch; sampled pixels against the oracle on the same edited scene."""
    from oracle import Params as OParams
    from paper_2601_23065_amd import EDIT_SET_ALBEDO, EDIT_SET_RADIANCE
    from paper_2601_23065_amd.api import BVH, Params, apply_edit, path_trace
    import torch

    scene, cams, cfg = sg.config(4)
    cam = cams[0]
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    rng = np.random.default_rng(4)
    emit = np.nonzero(scene.emissive > 0)[0]
    off = np.sort(rng.choice(emit, emit.size // 2, replace=False)).astype(np.int32)
    grp = np.sort(rng.choice(scene.n, scene.n // 10, replace=False)).astype(np.int32)
    color = (0.7, 0.2, 0.4)
    apply_edit(gs, EDIT_SET_RADIANCE, torch.from_numpy(off).cuda(), (0.0, 0.0, 0.0))
    apply_edit(gs, EDIT_SET_ALBEDO, torch.from_numpy(grp).cuda(), color)
    bvh.refit(gs)
    spp = 8
    p = Params(spp=spp, max_depth=cfg["max_depth"], rr_start=cfg["rr_start"], seed=0, camera_id=0)
    got = path_trace(bvh, gs, cam, p, 0, spp).cpu().numpy().reshape(-1, 3).astype(np.float64) / 2.0 ** 32

    edited = scene.copy()
    edited.radiance[:, off] = 0.0
    edited.albedo[:, grp] = np.asarray(color, dtype=np.float32)[:, None]
    pixels = np.random.default_rng(12).choice(cam.width * cam.height, 3, replace=False)
    prm = OParams(spp=spp, max_depth=p.max_depth, rr_start=p.rr_start, seed=0, camera_id=0)
    ref, flagged = _oracle_pixels(edited, cam, prm, pixels, spp, 2)
    ok = [px for px in ref if not flagged[px]]
    print(f"pixels {list(ref)} flagged {flagged} gpu {[got[px] for px in ok]} oracle {[ref[px] for px in ok]}")
    assert len(ok) >= 2
    err = rel_err(np.stack([got[px] for px in ok]), np.stack([ref[px] for px in ok]))
    assert err.max() <= 1e-4


def _sb_oracle_job(args):
    from oracle.render import single_bounce
    ci, pixels = args
    prm = _ORACLE["prm"][ci]
    out = single_bounce(_ORACLE["sc"], _ORACLE["cams"][ci], prm, pixels=pixels)
    # camera segment: Nt, Dt, A, P as the forward state stores them
    seg = np.array([np.concatenate([c.Nt, [c.Dt, c.A], c.P]) for c in out["cam"]])
    return ci, out["L"], out["R1"], out["branch"], out["flags"], seg


def test_single_bounce_config2_sampled_pixels():
    """The single-bounce forward at the reconstruction step's full size: the
    100k-surfel room, 8 cameras at 256x256, 8 spp, all cameras in one call
    (the launch the benchmark times). On 32 sampled pixels per camera, the
    branch taken, every secondary sample's R1 and the pixel value match the
    oracle wherever it flags no decision."""
    import torch
    from oracle import Params as OParams
    from oracle.tracer import Scene64
    from paper_2601_23065_amd.api import BVH, Params, render_single_bounce

    scene, cams, cfg = sg.config(2)
    p = Params(spp=cfg["spp"], seed=0, camera_id=0)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    rgb, state = render_single_bounce(bvh, gs, cams, p, keep_state=True)
    torch.cuda.synchronize()
    nc, hw, S = len(cams), cams[0].width * cams[0].height, p.spp
    rgb = rgb.cpu().numpy().reshape(nc, hw, 3).astype(np.float64)
    st = state[:nc * hw * 28].view(nc, hw, 28).cpu().numpy()
    cs = state[:nc * hw * 28].view(nc * hw, 28)[:, :24].contiguous().view(torch.float64).view(nc, hw, 12)
    cs = cs[..., [0, 1, 2, 3, 5, 9, 10, 11]].cpu().numpy()        # Nt(3), Dt, A, P(3)
    r1 = state[nc * hw * 28:].view(torch.float64).view(nc, hw, S, 3).cpu().numpy()

    rng = np.random.default_rng(21)
    picks = [np.sort(rng.choice(hw, 32, replace=False)) for _ in range(nc)]
    _ORACLE.update(sc=Scene64(scene), cams=cams,
                   prm=[OParams(spp=S, seed=0, camera_id=ci) for ci in range(nc)])
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        res = pool.map(_sb_oracle_job, list(enumerate(picks)), chunksize=1)
    n_ok = n_reflect = 0
    for ci, L, R1, branch, flags, seg in res:
        pix = picks[ci]
        ok = flags == 0
        n_ok += int(ok.sum())
        refl = ok & (branch == 2)
        n_reflect += int(refl.sum())
        np.testing.assert_array_equal(st[ci, pix, 25].astype(int)[ok], branch[ok])
        e1 = rel_err(r1[ci, pix][ok], R1[ok])
        eL = rel_err(rgb[ci, pix][ok], L[ok])
        es = rel_err(cs[ci, pix][refl], seg[refl])
        e1, eL, es = (float(e.max()) if e.size else 0.0 for e in (e1, eL, es))
        print(f"camera {ci}: unflagged {ok.sum()}/{pix.size} reflect {refl.sum()} R1 err {e1:.2e} "
              f"L err {eL:.2e} Nt/Dt/A/P err {es:.2e} nonzero L {np.count_nonzero(L[ok].sum(-1))}")
        assert e1 <= 1e-4 and eL <= 1e-4 and es <= 1e-4
    assert n_ok >= 0.5 * nc * 32 and n_reflect > 0
