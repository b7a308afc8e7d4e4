"""Pins for the oracle's single-bounce gradient: closed forms for one
surfel and central finite differences of the float64 forward pass on random
parameters whose discrete signature is unchanged within +-h."""
import numpy as np
import pytest

import scenegen as sg
from oracle import Params
from oracle.grad import PARAMS, signature, single_bounce_grad
from oracle.render import single_bounce
from oracle.tracer import Scene64


def _f64(scene):
    return {k: np.asarray(v, dtype=np.float64).copy() for k, v in scene.arrays().items()}


def test_single_surfel_emitter_closed_form():
    # one emissive surfel facing the camera: L = R = sigma g r, so
    # dL_c/dr_c = sigma g and dL/dsigma = g r
    f = np.float32
    s = dict(pos=f([[0.0], [0.0], [2.0]]), rot=f([[1.0], [0.0], [0.0], [0.0]]), scale=f([[0.5], [0.25]]),
             opacity=f([0.6]), albedo=f([[0.3], [0.3], [0.3]]), radiance=f([[2.0], [3.0], [4.0]]),
             emissive=f([1.0]))
    cam = sg.Camera((0.125, 0.0625, 0.0), (0.125, 0.0625, 1.0), (0.0, 1.0, 0.0), 20.0, 1, 1)
    prm = Params(spp=2)
    g, L, fwd = single_bounce_grad(s, cam, prm, pixels=np.array([0]), dL_dI=np.ones((1, 3)))
    assert fwd["branch"][0] == 1
    u, v = 0.125 / 0.5, 0.0625 / 0.25
    gg = np.exp(-0.5 * (u * u + v * v))
    sig = float(np.float32(0.6))
    np.testing.assert_allclose(L[0], sig * gg * np.array([2.0, 3.0, 4.0]), rtol=1e-12)
    np.testing.assert_allclose(g["radiance"][:, 0], sig * gg, rtol=1e-12)
    np.testing.assert_allclose(g["opacity"][0], gg * 9.0, rtol=1e-12)
    # d/ds_u of g = g u^2 / s_u (u = x / s_u)
    np.testing.assert_allclose(g["scale"][0, 0], sig * 9.0 * gg * u * u / 0.5, rtol=1e-10)
    assert np.all(g["albedo"] == 0)


def _fd_check(scene32, cam, prm, pixels, n_params, seed, rtol):
    rng = np.random.default_rng(seed)
    base = _f64(scene32)
    c = rng.uniform(-1, 1, (pixels.size, 3))
    g, L, fwd = single_bounce_grad(base, cam, prm, pixels, dL_dI=c)
    sig0 = signature(fwd)
    hit = set()
    for s in fwd["cam"]:
        hit.update(s.hits.tolist())
    for row in fwd["sec"]:
        for x in row:
            if x is not None:
                hit.update(x.hits.tolist())
    hit = sorted(hit)
    checked, tries = 0, 0
    while checked < n_params and tries < 10 * n_params:
        tries += 1
        k = PARAMS[rng.integers(len(PARAMS))]
        i = int(rng.choice(hit))
        comp = int(rng.integers(base[k].shape[0])) if base[k].ndim == 2 else None
        val = base[k][comp, i] if comp is not None else base[k][i]
        h = 1e-6 * max(1.0, abs(val))
        vals = []
        same = True
        for sgn in (1, -1):
            pert = {kk: vv.copy() for kk, vv in base.items()}
            if comp is not None:
                pert[k][comp, i] += sgn * h
            else:
                pert[k][i] += sgn * h
            out = single_bounce(Scene64(pert), cam, prm, pixels=pixels, keep_segments=True)
            same &= signature(out) == sig0
            vals.append(float((out["L"] * c).sum()))
        if not same:
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        ad = g[k][comp, i] if comp is not None else g[k][i]
        scale = max(abs(fd), abs(ad), 1e-3 * np.abs(np.concatenate([v.ravel() for v in g.values()])).max())
        assert abs(fd - ad) <= rtol * scale, (k, comp, i, fd, ad)
        checked += 1
    assert checked == n_params


def test_fd_cloud():
    scene, cams, _ = sg.config(1)
    cam = cams[0]
    rng = np.random.default_rng(1)
    pixels = rng.choice(cam.width * cam.height, 40, replace=False)
    _fd_check(scene, cam, Params(spp=4), pixels, 30, seed=5, rtol=1e-5)


def test_fd_room_with_bounce_chain():
    scene = sg.room_scene(6000, (3.0, 2.5, 2.5), 2, seed=41, emissive_frac=0.03)
    cam = sg.Camera((0.5, 0.6, 1.2), (2.5, 1.9, 1.9), (0.0, 0.0, 1.0), 75.0, 24, 18)
    rng = np.random.default_rng(2)
    pixels = rng.choice(cam.width * cam.height, 30, replace=False)
    _fd_check(scene, cam, Params(spp=3, seed=4), pixels, 30, seed=6, rtol=1e-5)


def test_detach_bounce_matches_albedo_gradient():
    # the albedo gradient does not depend on the bounce chain
    scene, cams, _ = sg.config(1)
    pixels = np.arange(0, 4096, 97)
    c = np.random.default_rng(0).uniform(-1, 1, (pixels.size, 3))
    g1, _, _ = single_bounce_grad(_f64(scene), cams[0], Params(spp=4), pixels, dL_dI=c)
    g2, _, _ = single_bounce_grad(_f64(scene), cams[0], Params(spp=4, detach_bounce=True), pixels, dL_dI=c)
    np.testing.assert_allclose(g1["albedo"], g2["albedo"], rtol=1e-12, atol=1e-15)
    assert np.abs(g1["pos"] - g2["pos"]).max() > 0
