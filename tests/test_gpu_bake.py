"""Parity of the light-baking path (Sec. 3.4, Eq. 10) with the FP64 oracle:
the 0-bounce image per pixel, its radiance gradient, the PQ-L1 loss and its
gradient, the projected Adam step, one fused bake iteration against the
separate calls, and a bake that fits path-traced targets of an edited room."""
import numpy as np
import pytest
import torch

import scenegen as sg
from oracle.bake import adam_step as o_adam, bake_loss as o_loss, zero_bounce_radiance_grad
from oracle.render import zero_bounce
from oracle.tracer import Scene64
from tests._util import gpu_scene, oracle_params, rel_err

pytestmark = pytest.mark.gpu


def _room():
    scene = sg.room_scene(16000, (3.0, 2.5, 2.5), 3, seed=31, emissive_frac=0.02)
    cams = [sg.Camera((0.4, 0.4, 1.0), (1.6, 1.3, 2.4), (0.0, 0.0, 1.0), 80.0, 20, 14),
            sg.Camera((2.6, 2.0, 1.2), (0.5, 0.6, 0.8), (0.0, 0.0, 1.0), 70.0, 20, 14)]
    rng = np.random.default_rng(4)
    scene.radiance[:] = rng.uniform(0.0, 2.0, scene.radiance.shape).astype(np.float32)
    return scene, cams


def test_zero_bounce_and_radiance_gradient():
    from paper_2601_23065_amd.api import BVH, Params, render_zero_bounce, zero_bounce_backward
    scene, cams = _room()
    p = Params(spp=1)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    rgb = render_zero_bounce(bvh, gs, cams, p).cpu().numpy().reshape(len(cams), -1, 3)
    rng = np.random.default_rng(6)
    sc = Scene64(scene)
    dL = np.zeros(rgb.shape, dtype=np.float32)
    ref_g = np.zeros((scene.n, 3))
    n_ok = 0
    for ci, cam in enumerate(cams):
        prm = oracle_params(p)
        prm.camera_id = ci
        L0, segs = zero_bounce(sc, cam, prm)
        ok = np.array([s.flags == 0 for s in segs])
        n_ok += int(ok.sum())
        err = rel_err(rgb[ci], L0, np.broadcast_to(ok[:, None], L0.shape))
        print(f"camera {ci}: unflagged {ok.mean():.3f} L0 err {err.max():.2e}")
        assert ok.mean() >= 0.98 and err.max() <= 1e-4
        # the loss gradient of unflagged pixels only: flagged ones may blend other hits
        dL[ci][ok] = rng.uniform(-1.0, 1.0, (int(ok.sum()), 3))
        ref_g += zero_bounce_radiance_grad(sc, cam, prm, dL[ci].astype(np.float64))
    g = zero_bounce_backward(bvh, gs, cams, p, torch.from_numpy(dL).cuda().view(len(cams), cams[0].height,
                                                                              cams[0].width, 3))
    g = g.cpu().numpy().T
    err = rel_err(g, ref_g)
    print(f"radiance grad err {err.max():.2e}, surfels touched {np.count_nonzero(ref_g.any(axis=1))}")
    assert np.count_nonzero(ref_g.any(axis=1)) > 100
    assert err.max() <= 1e-4


def test_bake_loss_and_adam():
    from paper_2601_23065_amd.api import Adam, adam_step, bake_loss
    rng = np.random.default_rng(8)
    rgb = rng.uniform(0.0, 4.0, (3, 17, 23, 3)).astype(np.float32)
    tgt = rng.uniform(0.0, 4.0, rgb.shape).astype(np.float32)
    rgb[0, 0, 0] = -0.5          # a negative value: PQ reads it as 0, slope 0
    tgt[1, 2, 3] = rgb[1, 2, 3]  # equal values: zero gradient
    loss, dL = bake_loss(torch.from_numpy(rgb).cuda(), torch.from_numpy(tgt).cuda())
    ref_loss, ref_dL = o_loss(rgb.astype(np.float64), tgt.astype(np.float64))
    assert abs(float(loss) - ref_loss) <= 1e-12 * ref_loss
    np.testing.assert_allclose(dL.cpu().numpy(), ref_dL, rtol=2e-6, atol=1e-30)
    # three projected Adam steps
    a = Adam(lr=0.05)
    r = rng.uniform(0.0, 1.0, 4000)
    r[:50] = 0.01                # driven below zero, then clamped
    m = np.zeros_like(r)
    v = np.zeros_like(r)
    rt, mt, vt = (torch.from_numpy(x.astype(np.float32)).cuda() for x in (r, m, v))
    for step in (1, 2, 3):
        gr = rng.uniform(-1.0, 1.0, r.size)
        gr[:50] = 1.0
        adam_step(rt, torch.from_numpy(gr.astype(np.float32)).cuda(), mt, vt, a, step)
        r, m, v = o_adam(r.astype(np.float32).astype(np.float64), gr.astype(np.float32).astype(np.float64), m, v,
                         step, a.lr, a.beta1, a.beta2, a.eps)
        np.testing.assert_allclose(rt.cpu().numpy(), r, rtol=1e-5, atol=1e-6)
    assert np.all(rt.cpu().numpy()[:50] == 0.0)


def test_bake_step_equals_the_separate_calls():
    from paper_2601_23065_amd.api import (Adam, Baker, BVH, Params, adam_step, bake_loss, render_zero_bounce,
                                          zero_bounce_backward)
    scene, cams = _room()
    p = Params(spp=1)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    rng = np.random.default_rng(12)
    tgt = torch.from_numpy(rng.uniform(0.0, 2.0, (len(cams), 14, 20, 3)).astype(np.float32)).cuda()
    adam = Adam(lr=0.02)
    # separate calls on a copy of the radiance
    r0 = gs.t["radiance"].clone()
    rgb = render_zero_bounce(bvh, gs, cams, p)
    loss_sep, dL = bake_loss(rgb, tgt)
    g = zero_bounce_backward(bvh, gs, cams, p, dL)
    m, v = torch.zeros_like(r0), torch.zeros_like(r0)
    r_sep = r0.clone()
    adam_step(r_sep, g, m, v, adam, 1)
    # the fused step
    baker = Baker(bvh, gs, cams, p, tgt, adam)
    loss = float(baker.step())
    assert abs(loss - float(loss_sep)) <= 1e-12 * float(loss_sep)
    # gradients summed in a different order can round differently; where
    # |g| is far from 0 the first step is exactly -lr sign(g)
    big = (g.abs() > 1e-6).cpu().numpy()
    np.testing.assert_allclose(gs.t["radiance"].cpu().numpy()[big], r_sep.cpu().numpy()[big], rtol=1e-6, atol=1e-7)


def test_bake_fits_path_traced_targets_of_an_edited_room():
    """Targets: path-traced images (depth 3, 64 spp) of the room with half
    its emitters switched off. Baking starts from the unedited radiance and
    must lower the PQ-L1 loss to well under half its first value."""
    from paper_2601_23065_amd import EDIT_SET_RADIANCE
    from paper_2601_23065_amd.api import Adam, Baker, BVH, Params, apply_edit, path_trace, resolve
    scene, cams = _room()
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    emit = np.nonzero(scene.emissive > 0)[0]
    off = np.sort(np.random.default_rng(2).choice(emit, emit.size // 2, replace=False)).astype(np.int32)
    r_before = gs.t["radiance"].clone()
    apply_edit(gs, EDIT_SET_RADIANCE, torch.from_numpy(off).cuda(), (0.0, 0.0, 0.0))
    pt = Params(spp=64, max_depth=3, rr_start=0)
    tg = []
    for ci, cam in enumerate(cams):
        pt.camera_id = ci
        tg.append(resolve(path_trace(bvh, gs, cam, pt), pt.spp))
    targets = torch.stack(tg)
    gs.t["radiance"].copy_(r_before)
    baker = Baker(bvh, gs, cams, Params(spp=1), targets, Adam(lr=0.05))
    losses = [float(baker.step()) for _ in range(60)]
    print(f"loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0]
    assert float(gs.t["radiance"].min()) >= 0.0
