"""Parity of the Stage-0 path (Sec. 3.2, Eq. 4) with the FP64 oracle: the
Nt, Dt, R, E images per pixel, the objective and its image gradient
(including the distance-normal term), the adjoint of a linear function of
the images for every parameter, and the whole render-loss-adjoint chain."""
import numpy as np
import pytest
import torch

import scenegen as sg
from oracle.stage0 import image_objective, images_vjp, stage0_images, stage0_objective
from oracle.tracer import Scene64
from tests._util import gpu_scene, oracle_params, rel_err

pytestmark = pytest.mark.gpu

KEYS = ("Nt", "Dt", "R", "E")
SLICES = {"Nt": slice(0, 3), "Dt": slice(3, 4), "R": slice(4, 7), "E": slice(7, 8)}


def _room():
    scene = sg.room_scene(16000, (3.0, 2.5, 2.5), 3, seed=31, emissive_frac=0.02)
    rng = np.random.default_rng(4)
    scene.radiance[:] = rng.uniform(0.0, 2.0, scene.radiance.shape).astype(np.float32)
    cams = [sg.Camera((0.4, 0.4, 1.0), (1.6, 1.3, 2.4), (0.0, 0.0, 1.0), 80.0, 20, 14),
            sg.Camera((2.6, 2.0, 1.2), (0.5, 0.6, 0.8), (0.0, 0.0, 1.0), 70.0, 20, 14)]
    return scene, cams


def _split(img):
    """[M, 8] -> dict of the four images (Dt and E as [M])."""
    return {k: (img[:, SLICES[k]] if k in ("Nt", "R") else img[:, SLICES[k]][:, 0]) for k in KEYS}


def _targets(M, seed):
    rng = np.random.default_rng(seed)
    n = rng.normal(size=(M, 3))
    return {"rgb": rng.uniform(0.0, 2.0, (M, 3)), "normal": n / np.linalg.norm(n, axis=1, keepdims=True),
            "mask": (rng.uniform(size=M) < 0.3).astype(np.float64)}


def _gpu_targets(tg, cams):
    H, W = cams[0].height, cams[0].width
    c = len(cams)
    f = lambda a, k: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32).reshape(c, H, W, k)).cuda()  # noqa: E731
    return f(tg["rgb"], 3), f(tg["normal"], 3), f(tg["mask"], 1)


def test_stage0_images():
    from paper_2601_23065_amd.api import BVH, Params, render_stage0
    scene, cams = _room()
    p = Params(spp=1)
    gs = gpu_scene(scene)
    images, _ = render_stage0(BVH(gs), gs, cams, p)
    images = images.cpu().numpy().reshape(len(cams), -1, 8).astype(np.float64)
    for ci, cam in enumerate(cams):
        prm = oracle_params(p)
        prm.camera_id = ci
        ref, segs = stage0_images(Scene64(scene), cam, prm)
        ok = np.array([s.flags == 0 for s in segs])
        got = _split(images[ci])
        for k in KEYS:
            m = ok if ref[k].ndim == 1 else np.broadcast_to(ok[:, None], ref[k].shape)
            err = rel_err(got[k], ref[k], m)
            print(f"camera {ci} {k}: err {err.max():.2e}")
            assert err.max() <= 1e-4
        assert np.array_equal(np.abs(got["Nt"]).sum(1) > 0, ref["hit"])


def test_stage0_loss_and_image_gradient():
    from paper_2601_23065_amd.api import Params, stage0_loss
    scene, cams = _room()
    cam = cams[0]
    p = Params(spp=1)
    ref_img, _ = stage0_images(Scene64(scene), cam, oracle_params(p))
    # the same (float32) images on both sides
    img8 = np.zeros((cam.width * cam.height, 8), dtype=np.float32)
    for k in KEYS:
        img8[:, SLICES[k]] = np.asarray(ref_img[k], dtype=np.float32).reshape(img8.shape[0], -1)
    img = _split(img8.astype(np.float64))
    img["hit"] = np.abs(img["Nt"]).sum(1) > 0
    tg = _targets(img8.shape[0], 5)
    weights = (1.0, 0.5, 0.7, 0.3)
    ref_loss, ref_g = image_objective(img, tg, weights, cam, oracle_params(p))
    loss, d = stage0_loss(torch.from_numpy(img8).cuda().view(1, cam.height, cam.width, 8), *_gpu_targets(tg, [cam]),
                          [cam], p, weights)
    d = _split(d.cpu().numpy().reshape(-1, 8).astype(np.float64))
    print(f"loss {float(loss):.10e} oracle {ref_loss:.10e}")
    assert abs(float(loss) - ref_loss) <= 1e-6 * ref_loss
    for k in KEYS:
        err = rel_err(d[k], ref_g[k])
        print(f"d{k}: err {err.max():.2e}")
        assert err.max() <= 1e-5


def test_stage0_adjoint_of_a_linear_function():
    from paper_2601_23065_amd.api import BVH, Params, render_stage0, stage0_backward
    scene, cams = _room()
    p = Params(spp=1)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    _, state = render_stage0(bvh, gs, cams, p)
    rng = np.random.default_rng(7)
    M = cams[0].width * cams[0].height
    d8 = np.zeros((len(cams), M, 8), dtype=np.float32)
    ref = None
    for ci, cam in enumerate(cams):
        prm = oracle_params(p)
        prm.camera_id = ci
        fwd = stage0_images(Scene64(scene), cam, prm)
        ok = np.array([s.flags == 0 for s in fwd[1]]) & fwd[0]["hit"]
        d8[ci][ok] = rng.uniform(-1.0, 1.0, (int(ok.sum()), 8))
        g = images_vjp(scene, cam, prm, _split(d8[ci].astype(np.float64)), fwd=fwd)
        ref = g if ref is None else {k: ref[k] + g[k] for k in ref}
    got = stage0_backward(bvh, gs, cams, p, torch.from_numpy(d8).cuda(), state)
    for k in ref:
        err = rel_err(got[k].cpu().numpy().astype(np.float64), ref[k])
        print(f"{k}: err {err.max():.2e}")
        assert err.max() <= 1e-3


def test_stage0_render_loss_adjoint_chain():
    from paper_2601_23065_amd.api import BVH, Params, render_stage0, stage0_backward, stage0_loss
    scene, cams = _room()
    cam = cams[1]
    p = Params(spp=1)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    tg = _targets(cam.width * cam.height, 9)
    weights = (1.0, 0.5, 0.7, 0.3)
    images, state = render_stage0(bvh, gs, [cam], p)
    loss, d = stage0_loss(images, *_gpu_targets(tg, [cam]), [cam], p, weights)
    got = stage0_backward(bvh, gs, [cam], p, d, state)
    ref_loss, ref, _, fwd = stage0_objective(scene, cam, oracle_params(p), tg, weights)
    assert all(s.flags == 0 for s in fwd[1])
    print(f"loss {float(loss):.8e} oracle {ref_loss:.8e}")
    assert abs(float(loss) - ref_loss) <= 1e-5 * ref_loss
    for k in ref:
        err = rel_err(got[k].cpu().numpy().astype(np.float64), ref[k])
        print(f"{k}: err {err.max():.2e}")
        assert err.max() <= 1e-3


def test_stage0_on_an_empty_view():
    """A camera looking out of the room's bounds from outside: every pixel
    misses, the images are zero, only the colour and emission terms remain
    (against constant targets, in closed form), and the adjoint is zero."""
    from oracle.bake import pq
    from paper_2601_23065_amd.api import BVH, Params, render_stage0, stage0_backward, stage0_loss
    scene, _ = _room()
    cam = sg.Camera((10.0, 10.0, 10.0), (20.0, 20.0, 20.0), (0.0, 0.0, 1.0), 30.0, 12, 9)
    p = Params(spp=1)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    images, state = render_stage0(bvh, gs, [cam], p)
    assert float(images.abs().max()) == 0.0
    M = cam.width * cam.height
    tg = {"rgb": np.full((M, 3), 0.5), "normal": np.tile([0.0, 0.0, 1.0], (M, 1)), "mask": np.full(M, 1.0)}
    loss, d = stage0_loss(images, *_gpu_targets(tg, [cam]), [cam], p, (1.0, 1.0, 1.0, 0.5))
    ref = abs(float(pq(0.0) - pq(0.5))) + 0.5 * 1.0
    assert abs(float(loss) - ref) <= 1e-12 * ref
    g = stage0_backward(bvh, gs, [cam], p, d, state)
    assert all(float(v.abs().max()) == 0.0 for v in g.values())
