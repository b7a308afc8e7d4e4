"""Pins for the oracle's Stage-0 objective (Sec. 3.2, Eq. 4): closed forms
for one surfel, the distance normal of a tilted plane, and central
differences of the float64 forward and of the image objective."""
import numpy as np

import scenegen as sg
from oracle import Params
from oracle.stage0 import _objective, _rays, image_objective, stage0_images, stage0_objective
from oracle.tracer import Scene64

F32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)   # noqa: E731


def _one(rot=(1.0, 0.0, 0.0, 0.0), size=0.5, z=2.0, sigma=0.6, r=(0.3, 0.5, 0.9), e=0.25):
    return sg.Scene(F32([[0.0], [0.0], [z]]), F32(np.array(rot)[:, None]), F32(np.full((2, 1), size)),
                    F32([sigma]), F32(np.full((3, 1), 0.5)), F32(np.array(r)[:, None]), F32([e]),
                    bounds=(np.full(3, -3.0), np.full(3, 3.0)))


def _targets(M, rgb=0.0, normal=(0.0, 0.0, -1.0), mask=0.0):
    return {"rgb": np.full((M, 3), rgb), "normal": np.tile(np.asarray(normal, dtype=np.float64), (M, 1)),
            "mask": np.full(M, mask)}


def test_one_surfel_closed_forms():
    scene = _one()
    cam = sg.Camera((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), (0.0, 1.0, 0.0), 10.0, 1, 1)
    img, _ = stage0_images(Scene64(scene), cam, Params(spp=1))
    s = float(np.float32(0.6))
    np.testing.assert_allclose(img["Nt"][0], [0.0, 0.0, -1.0], atol=1e-15)
    np.testing.assert_allclose(img["Dt"][0], 2.0, rtol=1e-15)
    np.testing.assert_allclose(img["R"][0], s * np.array([0.3, 0.5, 0.9], dtype=np.float32).astype(np.float64),
                               rtol=1e-15)
    np.testing.assert_allclose(img["E"][0], s * float(np.float32(0.25)), rtol=1e-15)
    # L_e alone: |E - M| with M = 1
    loss, g = image_objective(img, _targets(1, mask=1.0), (0.0, 0.0, 0.0, 1.0), cam, Params(spp=1))
    assert abs(loss - (1.0 - img["E"][0])) < 1e-15 and abs(g["E"][0] + 1.0) < 1e-15


def test_distance_normal_of_a_tilted_plane():
    ang = np.deg2rad(30.0)
    rot = (np.cos(ang / 2), np.sin(ang / 2), 0.0, 0.0)      # 30 degrees about x
    scene = _one(rot=rot, size=3.0)
    cam = sg.Camera((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), (0.0, 1.0, 0.0), 20.0, 9, 7)
    prm = Params(spp=1)
    img, _ = stage0_images(Scene64(scene), cam, prm)
    assert img["hit"].all()
    q = np.asarray(rot, dtype=np.float32).astype(np.float64)
    w, x = q[0], q[1]
    n = np.array([0.0, -2 * w * x, w * w - x * x]) / (w * w + x * x)     # R(q) e_z
    n = -n if n[2] > 0 else n                                          # facing the camera at the origin
    # the distance normal of every valid pixel is the plane's normal: 1 - N_d.n = 0
    loss, _ = image_objective(img, _targets(img["Dt"].size, normal=n), (0.0, 0.0, 1.0, 0.0), cam, prm)
    assert loss < 1e-12
    # against another normal the term is 1 - cos of the angle between them
    m = np.array([0.0, 0.0, -1.0])
    loss, _ = image_objective(img, _targets(img["Dt"].size, normal=m), (0.0, 0.0, 1.0, 0.0), cam, prm)
    assert abs(loss - (1.0 - float(n @ m))) < 1e-12
    # and the shading normal of a single surfel is the same
    np.testing.assert_allclose(img["Nt"], np.tile(n, (img["Dt"].size, 1)), atol=1e-12)


def _room_case():
    scene = sg.room_scene(1500, (3.0, 2.5, 2.5), 2, seed=23, emissive_frac=0.05)
    cam = sg.Camera((0.5, 0.6, 1.2), (2.5, 1.9, 1.4), (0.0, 0.0, 1.0), 60.0, 9, 7)
    rng = np.random.default_rng(3)
    scene.radiance[:] = rng.uniform(0.05, 2.0, scene.radiance.shape).astype(np.float32)
    M = cam.width * cam.height
    nrm = rng.normal(size=(M, 3))
    targets = {"rgb": rng.uniform(0.0, 2.0, (M, 3)), "normal": nrm / np.linalg.norm(nrm, axis=1, keepdims=True),
               "mask": (rng.uniform(size=M) < 0.3).astype(np.float64)}
    return scene, cam, targets


def test_image_objective_central_differences():
    scene, cam, targets = _room_case()
    prm = Params(spp=1)
    img, _ = stage0_images(Scene64(scene), cam, prm)
    weights = (1.0, 0.5, 0.7, 0.3)
    loss, g = image_objective(img, targets, weights, cam, prm)
    rng = np.random.default_rng(4)
    for key in ("Nt", "Dt", "R", "E"):
        a = np.asarray(img[key], dtype=np.float64)
        ok = np.repeat(img["hit"], a.size // img["hit"].size)
        if key == "R":
            ok &= a.ravel() > 1e-2      # PQ is smooth away from 0 (its slope is unbounded there)
        for k in rng.choice(np.nonzero(ok)[0], 4, replace=False):
            h = 1e-6 * max(1.0, abs(a.flat[k]))
            ip, im = dict(img), dict(img)
            ip[key], im[key] = a.copy(), a.copy()
            ip[key].flat[k] += h
            im[key].flat[k] -= h
            fd = (image_objective(ip, targets, weights, cam, prm)[0] - image_objective(im, targets, weights, cam, prm)[0]) / (2 * h)
            assert abs(fd - g[key].flat[k]) <= 1e-6 * max(1.0, abs(g[key].flat[k])), (key, k, fd, g[key].flat[k])


def test_parameter_gradient_central_differences():
    scene, cam, targets = _room_case()
    prm = Params(spp=1)
    weights = (1.0, 0.5, 0.7, 0.3)
    sc = Scene64(scene)
    loss, grads, _, fwd = stage0_objective(scene, cam, prm, targets, weights)
    img0, segs0 = fwd
    sig0 = [tuple(s.hits.tolist()) for s in segs0]
    O, W = _rays(cam, prm)
    import torch
    # the orientation decisions of the base point, held fixed
    _, flip0 = _objective(*(torch.as_tensor(img0[k]) for k in ("Nt", "Dt", "R", "E")), img0["hit"], O, W, targets,
                          weights, cam)
    hit_idx = np.unique(np.concatenate([s.hits for s in segs0 if s.hits.size]))
    rng = np.random.default_rng(8)
    checked = 0
    for key, comps in (("pos", 3), ("rot", 4), ("scale", 2), ("opacity", 0), ("radiance", 3), ("emissive", 0)):
        for _ in range(3):
            i = int(rng.choice(hit_idx))
            c = int(rng.integers(comps)) if comps else None
            base = getattr(scene, key)
            h = 1e-6 * max(1.0, abs(float(base[c, i] if c is not None else base[i])))
            vals = []
            for sgn in (1.0, -1.0):
                arr = scene.arrays()
                a = np.asarray(arr[key], dtype=np.float64).copy()
                if c is None:
                    a[i] += sgn * h
                else:
                    a[c, i] += sgn * h
                arr = {k: np.asarray(v, dtype=np.float64) for k, v in arr.items()}
                arr[key] = a
                img, segs = stage0_images(arr, cam, prm)
                if [tuple(s.hits.tolist()) for s in segs] != sig0:
                    break
                vals.append(float(_objective(*(torch.as_tensor(img[k]) for k in ("Nt", "Dt", "R", "E")), img["hit"],
                                             O, W, targets, weights, cam, flip=flip0)[0]))
            if len(vals) < 2:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            g = float(grads[key][c, i] if c is not None else grads[key][i])
            assert abs(fd - g) <= 1e-5 * max(1.0, abs(g)) + 1e-7, (key, i, c, fd, g)
            checked += 1
    assert checked >= 12


def test_objective_gradient_is_the_images_vjp_of_its_image_gradient():
    from oracle.stage0 import images_vjp
    scene, cam, targets = _room_case()
    prm = Params(spp=1)
    weights = (1.0, 0.5, 0.7, 0.3)
    _, grads, dimg, fwd = stage0_objective(scene, cam, prm, targets, weights)
    g2 = images_vjp(scene, cam, prm, dimg, fwd=fwd)
    for k in grads:
        np.testing.assert_allclose(g2[k], grads[k], rtol=1e-10, atol=1e-14)
    assert np.abs(grads["pos"]).max() > 0 and np.abs(grads["emissive"]).max() > 0
