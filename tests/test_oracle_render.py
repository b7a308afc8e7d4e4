"""Pins for the oracle's renderers: a white-furnace enclosure (closed form),
a quadrature of the single-bounce integral for one emitter over one receiver,
and the identities that tie path tracing to the 0-bounce and single-bounce
estimators, linearity in radiance, and zero albedo."""
import math

import numpy as np
import pytest
from scipy import integrate

import scenegen as sg
from oracle import Params, philox
from oracle.frames import cosine_direction
from oracle.render import path_trace, single_bounce, zero_bounce
from oracle.tracer import Scene64


def test_white_furnace_closed_form():
    # every segment ends inside 12 coplanar layers (A >= 1 - T_min), each
    # with radiance E and albedo rho; in additive mode a path's value is
    # E * sum_{k<=D} A_k prod_{j<k} (A_j rho), between the bounds below
    E, rho, D = 1.0, 0.5, 6
    scene = sg.furnace_scene(n_layers=12, radiance=E, albedo=rho)
    cam = sg.Camera((0.1, -0.2, 0.05), (1.0, 0.3, 0.2), (0.0, 0.0, 1.0), 90.0, 6, 6)
    prm = Params(spp=3, max_depth=D, rr_start=0, additive=True, t_min=1e-6)
    out = path_trace(Scene64(scene), cam, prm, keep_segments=True)
    vals = out["value"]
    rho32 = float(np.float32(rho))
    lo = E * (1 - 1e-4) * sum(((1 - 1e-4) * rho32) ** k for k in range(D + 1))
    hi = E * sum(rho32 ** k for k in range(D + 1))
    assert np.all(out["nseg"] == D + 1)
    assert vals.min() >= lo - 1e-12 and vals.max() <= hi + 1e-12
    closed = E * (1 - rho32 ** (D + 1)) / (1 - rho32)
    np.testing.assert_allclose(vals, closed, rtol=1e-4 * D)
    for row in out["segments"]:
        for path in row:
            assert all(s.A >= 1 - 1e-4 for s in path)
    # with Russian roulette and a deep limit the mean approaches E / (1 - rho)
    prm_rr = Params(spp=64, max_depth=40, rr_start=2, additive=True, t_min=1e-6)
    o = path_trace(Scene64(scene), cam, prm_rr)["value"][..., 0].ravel()
    se = o.std() / math.sqrt(o.size)
    assert abs(o.mean() - E / (1 - rho32)) < 4 * se + 1e-3


def _emitter_over_receiver():
    # receiver: huge surfel in z = 0, facing +z; emitter: surfel in z = 1 facing
    # -z, turned about z by the quaternion (3, 0, 0, 1) (t_u = (0.8, 0.6, 0))
    f = np.float32
    s = dict(pos=f([[0.0, 0.1], [0.0, -0.05], [0.0, 1.0]]),
             rot=f([[1.0, 0.0], [0.0, 1.0], [0.0, 3.0], [0.0, 0.0]]),  # 2nd: 180deg about x, then about z
             scale=f([[50.0, 0.3], [50.0, 0.2]]), opacity=f([0.999, 0.8]),
             albedo=f([[0.5, 0.5], [0.5, 0.5], [0.5, 0.5]]),
             radiance=f([[0.0, 5.0], [0.0, 4.0], [0.0, 3.0]]), emissive=f([0.0, 1.0]))
    return s


def test_single_bounce_quadrature():
    scene = _emitter_over_receiver()
    sc = Scene64(scene)
    # the emitter's frame from its quaternion (x = 3, y = 1 after a half turn
    # about x): check it is the plane z = 1 with normal -z
    assert np.allclose(sc.n[1], [0, 0, -1])
    tu, tv = sc.tu[1], sc.tv[1]
    su, sv, sig, r = float(np.float32(0.3)), float(np.float32(0.2)), float(np.float32(0.8)), np.array([5.0, 4.0, 3.0])
    ctr = np.array([float(np.float32(0.1)), float(np.float32(-0.05)), 1.0])
    cam = sg.Camera((3.0, 0.0, 0.5), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 10.0, 1, 1)
    S = 20000
    prm = Params(spp=S)
    out = single_bounce(sc, cam, prm)
    assert out["branch"][0] == 2
    # per-sample values in closed form: the direction meets z = 1 at y, whose
    # coordinates in the emitter frame give alpha
    u0, u1, _, _ = philox.uniforms(np.zeros(S, dtype=np.int64), np.arange(S), 0, 0, 0)
    d = cosine_direction(np.tile([0.0, 0.0, 1.0], (S, 1)), u0, u1)
    y = d / d[:, 2:3] - ctr[None, :]
    a, b = y @ tu / su, y @ tv / sv
    q2 = a * a + b * b
    al = np.where(q2 <= 9, sig * np.exp(-0.5 * q2), 0.0)
    np.testing.assert_allclose(out["R1"][0, :, 0], al * r[0], rtol=1e-9, atol=1e-12)
    # E[R1] = int sigma g r cos/pi dw = int_plane sigma g r h^2 / (pi |x|^4) dA (h = 1)
    def f(bb, aa):
        x = ctr + aa * su * tu + bb * sv * tv
        return sig * math.exp(-0.5 * (aa * aa + bb * bb)) / (math.pi * (x @ x) ** 2) * su * sv
    I, err = integrate.dblquad(f, -3, 3, lambda aa: -math.sqrt(max(9 - aa * aa, 0)),
                               lambda aa: math.sqrt(max(9 - aa * aa, 0)), epsabs=1e-11, epsrel=1e-10)
    R1 = out["R1"][0, :, 0] / r[0]
    se = R1.std() / math.sqrt(S)
    assert abs(R1.mean() - I) < 4 * se
    # the pixel value is P0 * mean(R1)
    np.testing.assert_allclose(out["L"][0], out["cam"][0].P * out["R1"][0].mean(axis=0), rtol=1e-12)


@pytest.fixture(scope="module")
def small_room():
    s = sg.room_scene(12000, (3.0, 2.5, 2.5), 3, seed=31, emissive_frac=0.02)
    cam = sg.Camera((0.4, 0.4, 1.0), (1.6, 1.3, 2.4), (0.0, 0.0, 1.0), 80.0, 10, 8)
    return s, Scene64(s), cam


def test_pt_depth0_is_emitter_part_of_zero_bounce(small_room):
    s, sc, cam = small_room
    prm = Params(spp=1, max_depth=0)
    pt = path_trace(sc, cam, prm, keep_segments=True)
    R0, segs = zero_bounce(sc, cam, prm)
    em = np.array([g.E > prm.tau_E for g in segs])
    np.testing.assert_allclose(pt["value"][:, 0], np.where(em[:, None], R0, 0.0), rtol=1e-13, atol=0)
    assert em.any() and (~em).any()


def test_pt_depth1_equals_single_bounce_on_emitter_secondaries(small_room):
    s, sc, cam = small_room
    prm = Params(spp=6, max_depth=1, rr_start=0)
    pt = path_trace(sc, cam, prm)
    sb = single_bounce(sc, cam, prm, keep_segments=True)
    n_em = 0
    for i in range(sb["pixels"].size):
        for j in range(prm.spp):
            if sb["branch"][i] == 0:
                assert np.all(pt["value"][i, j] == 0)
            elif sb["branch"][i] == 1:
                np.testing.assert_allclose(pt["value"][i, j], sb["L"][i], rtol=1e-13)
            else:
                g = sb["sec"][i][j]
                if g.E > prm.tau_E:
                    n_em += 1
                    np.testing.assert_allclose(pt["value"][i, j], sb["cam"][i].P * g.R, rtol=1e-12)
                else:
                    assert np.all(pt["value"][i, j] == 0)
    assert n_em > 0


def test_pt_linear_in_radiance_and_zero_albedo(small_room):
    s, sc, cam = small_room
    prm = Params(spp=4, max_depth=4, rr_start=2)
    base = path_trace(sc, cam, prm)["value"]
    s2 = s.copy()
    s2.radiance = (s.radiance * np.float32(4.0)).astype(np.float32)   # exact in float32
    scaled = path_trace(Scene64(s2), cam, prm)["value"]
    np.testing.assert_allclose(scaled, 4.0 * base, rtol=1e-13, atol=0)
    s3 = s.copy()
    s3.albedo = np.zeros_like(s.albedo)
    z = path_trace(Scene64(s3), cam, prm)["value"]
    d0 = path_trace(sc, cam, Params(spp=4, max_depth=0))["value"]
    np.testing.assert_allclose(z, d0, rtol=1e-13, atol=0)
    assert base.sum() > z.sum() > 0
