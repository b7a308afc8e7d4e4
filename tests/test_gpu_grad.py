"""Parity of the hand-written single-bounce adjoint with the oracle's
gradient (1e-3) and with float64 central finite differences of the oracle's
forward pass (1e-2), on pixels the oracle does not flag."""
import numpy as np
import pytest
import torch

import scenegen as sg
from oracle.grad import PARAMS, signature, single_bounce_grad
from oracle.render import single_bounce
from oracle.tracer import Scene64
from tests._util import coplanar_stack, gpu_scene, oracle_params, rel_err

pytestmark = pytest.mark.gpu


def _gpu_grads(scene, cams, p, dL):
    from paper_2601_23065_amd.api import BVH, render_single_bounce, single_bounce_backward
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    rgb, state = render_single_bounce(bvh, gs, cams, p, keep_state=True)
    g = single_bounce_backward(bvh, gs, cams, p, torch.from_numpy(dL).cuda(), state)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}, rgb.cpu().numpy()


def _unflagged_pixels(sc, cam, prm, count, seed):
    rng = np.random.default_rng(seed)
    cand = rng.choice(cam.width * cam.height, count * 3, replace=False)
    fwd = single_bounce(sc, cam, prm, pixels=cand)
    ok = cand[(fwd["flags"] == 0) & (fwd["branch"] > 0)]
    return np.sort(ok[:count])


def _compare(scene, cams, p, n_pix, seed, tol=1e-3):
    prm = oracle_params(p)
    sc = Scene64(scene)
    H, W = cams[0].height, cams[0].width
    rng = np.random.default_rng(seed)
    dL = np.zeros((len(cams), H * W, 3), dtype=np.float32)
    ref = {k: 0.0 for k in PARAMS}
    for ci, cam in enumerate(cams):
        prm_c = oracle_params(p)
        prm_c.camera_id = p.camera_id + ci
        pix = _unflagged_pixels(sc, cam, prm_c, n_pix, seed + ci)
        c = rng.uniform(-1, 1, (pix.size, 3)).astype(np.float32)
        dL[ci, pix] = c
        g, _, _ = single_bounce_grad(scene, cam, prm_c, pix, dL_dI=c.astype(np.float64))
        for k in PARAMS:
            ref[k] = ref[k] + g[k]
    got, _ = _gpu_grads(scene, cams, p, dL.reshape(len(cams), H, W, 3))
    worst = {}
    for k in PARAMS:
        e = rel_err(got[k], ref[k])
        worst[k] = float(e.max())
    print("max rel err", {k: f"{v:.2e}" for k, v in worst.items()})
    for k, v in worst.items():
        assert v <= tol, (k, v)
    return ref, got


def test_adjoint_config1_cloud():
    from paper_2601_23065_amd.api import Params
    scene, cams, cfg = sg.config(1)
    _compare(scene, cams, Params(spp=cfg["spp"]), 300, seed=1)


def test_adjoint_room_bounce_chain():
    from paper_2601_23065_amd.api import Params
    scene = sg.room_scene(20000, (3.0, 2.5, 2.5), 3, seed=41, emissive_frac=0.02)
    cams = sg.interior_cameras(scene, 2, 48, 40, seed=5)
    _compare(scene, cams, Params(spp=4, seed=9), 120, seed=3)


def test_adjoint_detached_bounce():
    from paper_2601_23065_amd import DETACH_BOUNCE
    from paper_2601_23065_amd.api import Params
    scene = sg.room_scene(20000, (3.0, 2.5, 2.5), 3, seed=41, emissive_frac=0.02)
    cams = sg.interior_cameras(scene, 1, 48, 40, seed=6)
    _compare(scene, cams, Params(spp=4, flags=DETACH_BOUNCE), 120, seed=4)


@pytest.mark.slow
def test_adjoint_config2_masked():
    """100k-surfel room, 8 cameras at 256x256, 8 spp; 48 unflagged pixels
    per camera carry the loss."""
    from paper_2601_23065_amd.api import Params
    scene, cams, cfg = sg.config(2)
    _compare(scene, cams, Params(spp=cfg["spp"]), 48, seed=7)


def test_adjoint_deep_stack_beyond_the_record_slots():
    """A 300-layer coplanar stack filling a 90x90 image: the camera pass
    blends 300 hits per pixel, 2.43 M in all, more than the 2^21 record slots
    its workspace holds on a 256-CU device (one 1024-slot chunk per wave of
    the persistent grid), so the last hits take the atomic path; every pixel
    is an emitter pixel (E > tau_E), whose gradient flows through the camera
    segment alone."""
    from paper_2601_23065_amd.api import Params
    scene = coplanar_stack(300, 5)
    cam = sg.Camera((0.0, 0.0, -2.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 5.0, 90, 90)
    _compare(scene, [cam], Params(spp=2, seed=5), 40, seed=8)


def test_adjoint_against_finite_differences():
    from paper_2601_23065_amd.api import Params
    scene = sg.room_scene(8000, (3.0, 2.5, 2.5), 2, seed=43, emissive_frac=0.03)
    cam = sg.Camera((0.5, 0.6, 1.2), (2.5, 1.9, 1.9), (0.0, 0.0, 1.0), 75.0, 32, 24)
    p = Params(spp=3, seed=4)
    prm = oracle_params(p)
    sc = Scene64(scene)
    pix = _unflagged_pixels(sc, cam, prm, 40, 11)
    rng = np.random.default_rng(12)
    c = rng.uniform(-1, 1, (pix.size, 3))
    dL = np.zeros((1, cam.height * cam.width, 3), dtype=np.float32)
    dL[0, pix] = c
    got, _ = _gpu_grads(scene, [cam], p, dL.reshape(1, cam.height, cam.width, 3))
    base = {k: np.asarray(v, dtype=np.float64).copy() for k, v in scene.arrays().items()}
    fwd0 = single_bounce(Scene64(base), cam, prm, pixels=pix, keep_segments=True)
    sig0 = signature(fwd0)
    hit = sorted({int(h) for s in fwd0["cam"] for h in s.hits})
    scale = max(np.abs(v).max() for v in got.values())
    checked = tries = 0
    while checked < 50 and tries < 400:
        tries += 1
        k = PARAMS[rng.integers(len(PARAMS))]
        i = int(rng.choice(hit))
        comp = int(rng.integers(base[k].shape[0])) if base[k].ndim == 2 else None
        val = base[k][comp, i] if comp is not None else base[k][i]
        h = 1e-6 * max(1.0, abs(val))
        f = []
        same = True
        for sgn in (1, -1):
            pert = {kk: vv.copy() for kk, vv in base.items()}
            if comp is not None:
                pert[k][comp, i] += sgn * h
            else:
                pert[k][i] += sgn * h
            out = single_bounce(Scene64(pert), cam, prm, pixels=pix, keep_segments=True)
            same &= signature(out) == sig0
            f.append(float((out["L"] * c).sum()))
        if not same:
            continue
        fd = (f[0] - f[1]) / (2 * h)
        ad = got[k][comp, i] if comp is not None else got[k][i]
        assert abs(ad - fd) <= 1e-2 * max(abs(fd), 1e-2 * scale), (k, comp, i, ad, fd)
        checked += 1
    assert checked == 50


def test_autograd_function_matches_oracle_gradient():
    """SingleBounceRender.apply on leaf tensors, a masked linear loss, and
    loss.backward(): every leaf's .grad against the oracle's gradient of the
    same loss (1e-3); the emissive input gets no gradient."""
    from paper_2601_23065_amd.api import BVH, Params, SingleBounceRender
    scene = sg.room_scene(20000, (3.0, 2.5, 2.5), 3, seed=41, emissive_frac=0.02)
    cams = sg.interior_cameras(scene, 2, 48, 40, seed=5)
    p = Params(spp=4, seed=9)
    sc = Scene64(scene)
    H, W = cams[0].height, cams[0].width
    rng = np.random.default_rng(13)
    c = np.zeros((len(cams), H * W, 3))
    ref = {k: 0.0 for k in PARAMS}
    for ci, cam in enumerate(cams):
        prm = oracle_params(p)
        prm.camera_id = p.camera_id + ci
        pix = _unflagged_pixels(sc, cam, prm, 100, 30 + ci)
        c[ci, pix] = rng.uniform(-1, 1, (pix.size, 3))
        g, _, _ = single_bounce_grad(scene, cam, prm, pix, dL_dI=c[ci, pix])
        for k in PARAMS:
            ref[k] = ref[k] + g[k]
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    leaves = {k: gs.t[k].clone().requires_grad_(True) for k in PARAMS}
    emissive = gs.t["emissive"].clone()
    rgb = SingleBounceRender.apply(leaves["pos"], leaves["rot"], leaves["scale"], leaves["opacity"],
                                   leaves["albedo"], leaves["radiance"], emissive, bvh, gs, cams, p)
    assert rgb.requires_grad and rgb.shape == (len(cams), H, W, 3)
    loss = (rgb * torch.from_numpy(c.reshape(len(cams), H, W, 3)).float().cuda()).sum()
    loss.backward()
    assert emissive.grad is None
    for k in PARAMS:
        got = leaves[k].grad.cpu().numpy().astype(np.float64)
        e = rel_err(got, ref[k])
        print(f"{k}: max rel err {e.max():.2e}")
        assert e.max() <= 1e-3, k


_FD = {}


def _near(O, W, p, n, tu, tv, su, sv, k2):
    """Rays (O, W [R, 3]) that come within 1.1 k_sigma of one surfel's
    tangent-plane ellipse at t > 0: the only rays a small change of that
    surfel can affect."""
    den = W @ n
    with np.errstate(divide="ignore", invalid="ignore"):
        t = ((p - O) @ n) / den
        y = O + t[:, None] * W - p
        q2 = (y @ tu / su) ** 2 + (y @ tv / sv) ** 2
    return (np.abs(den) > 1e-12) & (t > 0) & (q2 <= 1.21 * k2)


def _fd_job(args):
    """Central difference of the masked L2 loss for one parameter, over the
    masked pixels whose rays pass near its surfel; None if a discrete
    decision of those pixels changes within +-h."""
    from oracle.frames import quat_frames
    from oracle.render import single_bounce
    key, comp, i = args
    base, cams, prms, rays, mask, tgt, fwd0 = (_FD[k] for k in ("base", "cams", "prms", "rays", "mask", "tgt", "fwd0"))
    tu, tv, n = (a[0] for a in quat_frames(base["rot"][:, i:i + 1]))
    p = base["pos"][:, i]
    su, sv = base["scale"][:, i]
    k2 = prms[0].k_sigma ** 2
    val = base[key][comp, i] if comp is not None else base[key][i]
    h = 1e-6 * max(1.0, abs(val))
    dL = 0.0
    for ci in range(len(cams)):
        O, W, owner = rays[ci]
        aff = np.unique(owner[_near(O, W, p, n, tu, tv, su, sv, k2)])
        if aff.size == 0:
            continue
        pix = mask[ci][aff]
        f0 = fwd0[ci]
        sig0 = signature({"branch": f0["branch"][aff], "cam": [f0["cam"][a] for a in aff],
                          "sec": [f0["sec"][a] for a in aff]})
        f = []
        for sgn in (1, -1):
            pert = {kk: vv for kk, vv in base.items()}
            arr = base[key].copy()
            if comp is not None:
                arr[comp, i] += sgn * h
            else:
                arr[i] += sgn * h
            pert[key] = arr
            out = single_bounce(Scene64(pert), cams[ci], prms[ci], pixels=pix, keep_segments=True)
            if signature(out) != sig0:
                return None
            f.append(0.5 * float(((out["L"] - tgt[ci][aff]) ** 2).sum()))
        dL += (f[0] - f[1]) / (2 * h)
    return key, comp, i, dL


@pytest.mark.slow
def test_adjoint_config2_against_finite_differences():
    """The reconstruction step at full size: 100k-surfel room, 8 cameras at
    256x256, 8 spp, L2 loss over a mask of 64 seeded pixels per camera
    against the oracle's render of the perturbed scene. The adjoint of the
    full-size call against central differences of the float64 forward on 50
    random parameters of surfels the masked pixels blend (camera and
    secondary segments), each parameter's difference taken over the masked
    pixels whose rays pass near its surfel, resampled when a discrete
    decision of those pixels changes; agreement 1e-2."""
    from oracle import Params as OParams
    from paper_2601_23065_amd.api import Params
    scene, cams, cfg = sg.config(2)
    target = sg.perturb(scene, seed=102)
    p_spp = cfg["spp"]
    prms = [OParams(spp=p_spp, seed=0, camera_id=ci) for ci in range(len(cams))]
    sc, st = Scene64(scene), Scene64(target)
    H, W = cams[0].height, cams[0].width
    rng = np.random.default_rng(302)
    masks, fwds, tgts, rays = [], [], [], []
    dL = np.zeros((len(cams), H * W, 3), dtype=np.float32)
    hit_cam, hit_sec = set(), set()
    for ci, cam in enumerate(cams):
        cand = np.sort(rng.choice(H * W, 64, replace=False))
        fwd = single_bounce(sc, cam, prms[ci], pixels=cand, keep_segments=True)
        ok = fwd["flags"] == 0
        pix = cand[ok]
        fwd = single_bounce(sc, cam, prms[ci], pixels=pix, keep_segments=True)
        tgt = single_bounce(st, cam, prms[ci], pixels=pix)["L"]
        masks.append(pix)
        fwds.append(fwd)
        tgts.append(tgt)
        dL[ci, pix] = (fwd["L"] - tgt).astype(np.float32)
        O = [fwd["O"]]
        Wd = [fwd["W"]]
        owner = [np.arange(pix.size)]
        for a, row in enumerate(fwd["sec"]):
            for g in row:
                if g is not None:
                    O.append(g.O[None])
                    Wd.append(g.W[None])
                    owner.append(np.array([a]))
                    hit_sec.update(int(h) for h in g.hits)
        rays.append((np.concatenate(O), np.concatenate(Wd), np.concatenate(owner)))
        hit_cam.update(int(h) for s in fwd["cam"] for h in s.hits)
    got, _ = _gpu_grads(scene, cams, Params(spp=p_spp, seed=0, camera_id=0), dL.reshape(len(cams), H, W, 3))
    base = {k: np.asarray(v, dtype=np.float64).copy() for k, v in scene.arrays().items()}
    _FD.update(base=base, cams=cams, prms=prms, rays=rays, mask=masks, tgt=tgts, fwd0=fwds)
    pools = (sorted(hit_cam), sorted(hit_sec - hit_cam) or sorted(hit_cam))
    jobs = []
    for j in range(160):
        k = PARAMS[rng.integers(len(PARAMS))]
        i = int(rng.choice(pools[j % 2]))
        comp = int(rng.integers(base[k].shape[0])) if base[k].ndim == 2 else None
        jobs.append((k, comp, i))
    import multiprocessing as mp
    import os
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        res = [r for r in pool.map(_fd_job, jobs, chunksize=1) if r is not None][:50]
    scale = max(np.abs(v).max() for v in got.values())
    worst = 0.0
    for k, comp, i, fd in res:
        ad = got[k][comp, i] if comp is not None else got[k][i]
        e = abs(ad - fd) / max(abs(fd), 1e-2 * scale)
        worst = max(worst, e)
        assert e <= 1e-2, (k, comp, i, ad, fd)
    print(f"{len(res)} parameters checked, worst {worst:.2e}; {len(hit_cam)} camera-hit and {len(hit_sec)} "
          f"secondary-hit surfels")
    assert len(res) == 50
