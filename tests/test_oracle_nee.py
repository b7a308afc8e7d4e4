"""Pins for the oracle's emitter sampling with multiple importance sampling:
the light pdf integrates to one, light samples reproduce the emitters' solid
angle and the selection and point distributions, the estimator reaches the
single-bounce integral of one emitter over one receiver (quadrature), has the
plain path tracer's mean on a room, and equals it when no vertex is reached."""
import math

import numpy as np
import pytest
from scipy import integrate

import scenegen as sg
from oracle import Params
from oracle.nee import Emitters, path_trace_nee
from oracle.render import path_trace, zero_bounce
from oracle.tracer import Scene64
from tests.test_oracle_render import _emitter_over_receiver


def _panel_scene():
    """Four emitters of different sizes and orientations, two overlapping,
    one seen edge-on from the origin's side, plus one non-emitter."""
    f = np.float32
    rng = np.random.default_rng(5)
    q = rng.normal(size=(4, 5))
    q[:, 0] = (1.0, 0.0, 0.0, 0.0)
    q[:, 1] = (1.0, 0.0, 0.0, 0.0)
    return dict(pos=f([[0.0, 0.1, -0.8, 0.9, 0.0], [0.0, 0.05, 0.3, -0.7, 0.5], [1.0, 1.1, 0.6, 0.4, 2.0]]),
                rot=f(q), scale=f([[0.3, 0.2, 0.1, 0.25, 0.5], [0.2, 0.3, 0.15, 0.05, 0.5]]),
                opacity=f([0.8, 0.6, 0.9, 0.7, 0.9]),
                albedo=f(np.full((3, 5), 0.5)),
                radiance=f([[5.0, 1.0, 2.0, 0.0, 1.0], [4.0, 1.0, 2.0, 0.0, 1.0], [3.0, 1.0, 2.0, 0.0, 1.0]]),
                emissive=f([1.0, 0.5, 1.0, 0.8, 0.0]))


def _sphere(n, rng):
    d = rng.normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


@pytest.mark.parametrize("cell", [0.0, 0.5])
def test_light_pdf_integrates_to_one(cell):
    em = Emitters(Scene64(_panel_scene()), 0.1, cell=cell)
    assert em.count == 4 and (cell == 0 or em.Wc.size == 3)
    rng = np.random.default_rng(1)
    for X in ([0.0, 0.0, 0.0], [0.3, -0.2, 0.8], [0.0, 0.0, 1.5]):
        vals = []
        for _ in range(8):
            W = _sphere(50000, rng)
            vals.append(4.0 * np.pi * em.pdf(np.tile(X, (W.shape[0], 1)), W)[0])
        v = np.concatenate(vals)
        se = v.std() / math.sqrt(v.size)
        print(f"X={X}: {v.mean():.5f} +- {se:.5f}")
        assert abs(v.mean() - 1.0) < 5 * se + 1e-3


@pytest.mark.parametrize("cell", [0.0, 0.5])
def test_light_samples_cover_the_emitters_solid_angle(cell):
    sc = Scene64(_panel_scene())
    em = Emitters(sc, 0.1, cell=cell)
    rng = np.random.default_rng(2)
    X = np.array([0.2, -0.1, 0.1])
    n = 400000
    u0, u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n), rng.random(n)
    j, y, _ = em.sample(u0, u1, u2, u3, np.tile(X, (n, 1)))
    # selection frequencies: w_j / W, or with cells I_c(X) / sum I times w_j / W_c
    freq = np.bincount(j, minlength=em.count) / n
    if cell > 0:
        I, S = em.importance(X)
        p = I[0, em.cell_of] / S[0] * em.w / em.Wc[em.cell_of]
        # hand check of the importance: W_c over the squared distance to the cell centre, floored at c^2
        m = (np.floor(em.p[0] / cell) + 0.5) * cell
        assert abs(I[0, em.cell_of[0]] - em.Wc[em.cell_of[0]] / max(np.sum((X - m) ** 2), cell * cell)) < 1e-15
    else:
        p = em.w / em.W
    assert abs(p.sum() - 1.0) < 1e-12
    assert np.all(np.abs(freq - p) <= 5 * np.sqrt(p * (1 - p) / n))
    # points are uniform on the k_sigma ellipse: (u^2 + v^2) / k^2 ~ U(0, 1)
    dy = y - em.p[j]
    q2 = ((dy * em.tu[j]).sum(1) / em.su[j]) ** 2 + ((dy * em.tv[j]).sum(1) / em.sv[j]) ** 2
    assert np.all(q2 <= 9.0 * (1 + 1e-12))
    assert abs((q2 / 9.0).mean() - 0.5) < 5 * math.sqrt(1 / 12 / n)
    assert np.all(np.abs((dy * em.n[j]).sum(1)) < 1e-12)
    # E[1 / p_l] over light samples is the solid angle crossed by some emitter
    W = (y - X) / np.linalg.norm(y - X, axis=1, keepdims=True)
    pl = em.pdf(np.tile(X, (n, 1)), W)[0]
    assert np.all(pl > 0)
    inv = 1.0 / pl
    Wu = _sphere(n, rng)
    cov = 4.0 * np.pi * (em.pdf(np.tile(X, (n, 1)), Wu)[0] > 0)
    se = math.sqrt(inv.var() / n + cov.var() / n)
    print(f"E[1/p_l] {inv.mean():.5f}  solid angle {cov.mean():.5f} +- {se:.5f}")
    assert abs(inv.mean() - cov.mean()) < 5 * se


def test_single_bounce_quadrature_with_mis():
    """One emitter (e = 1) over one receiver, max_depth 1: the path value is
    P times the integral of cos/pi alpha r over the directions where the
    emitter passes the emitter test (alpha > tau_E)."""
    scene = _emitter_over_receiver()
    sc = Scene64(scene)
    tu, tv = sc.tu[1], sc.tv[1]
    su, sv, sig = float(np.float32(0.3)), float(np.float32(0.2)), float(np.float32(0.8))
    ctr = np.array([float(np.float32(0.1)), float(np.float32(-0.05)), 1.0])
    cam = sg.Camera((3.0, 0.0, 0.5), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 10.0, 1, 1)
    S = 6000
    prm = Params(spp=S, max_depth=1, rr_start=0)
    out = path_trace_nee(sc, cam, prm)
    plain = path_trace(sc, cam, prm)
    assert np.all(out["flags"] == 0)
    c2 = 2.0 * math.log(sig / prm.tau_E)          # alpha > tau_E  <=>  u^2 + v^2 < c2

    def f(th, rr):
        a, b = rr * math.cos(th), rr * math.sin(th)
        x = ctr + a * su * tu + b * sv * tv
        return sig * math.exp(-0.5 * rr * rr) / (math.pi * (x @ x) ** 2) * su * sv * rr
    I, _ = integrate.dblquad(f, 0.0, math.sqrt(c2), 0.0, 2.0 * math.pi, epsabs=1e-12, epsrel=1e-10)
    # the camera segment's P (receiver, opacity 0.999, albedo 0.5)
    P0 = float(np.float32(0.999)) * float(np.float32(0.5))
    v = out["value"][0, :, 0] / (P0 * 5.0)
    vp = plain["value"][0, :, 0] / (P0 * 5.0)
    se = v.std() / math.sqrt(S)
    print(f"quadrature {I:.6e}  mis {v.mean():.6e} +- {se:.1e}  plain {vp.mean():.6e} +- "
          f"{vp.std() / math.sqrt(S):.1e}")
    assert abs(v.mean() - I) < 4 * se
    assert v.std() < 0.7 * vp.std()


@pytest.mark.parametrize("cell", [0.0, 1.0])
def test_mis_mean_equals_plain_mean_on_a_room(cell):
    scene = sg.room_scene(3000, (3.0, 2.5, 2.5), 3, seed=31, emissive_frac=0.05)
    sc = Scene64(scene)
    cam = sg.Camera((0.4, 0.4, 1.0), (1.6, 1.3, 2.4), (0.0, 0.0, 1.0), 80.0, 8, 6)
    prm = Params(spp=1, max_depth=3, rr_start=2, seed=4)
    _, segs = zero_bounce(sc, cam, prm)
    # pixels whose camera segment reflects
    pix = np.array([i for i, g in enumerate(segs) if g.hit and g.E <= prm.tau_E and g.flags == 0])[[0, 15, 30]]
    S = 800
    em = Emitters(sc, 0.1, cell=cell)
    a = path_trace_nee(sc, cam, Params(spp=S, max_depth=3, rr_start=2, seed=4), em=em, pixels=pix)
    b = path_trace(sc, cam, Params(spp=S, max_depth=3, rr_start=2, seed=4), pixels=pix)
    for i in range(pix.size):
        va, vb = a["value"][i].sum(-1), b["value"][i].sum(-1)
        se = math.sqrt(va.var() / S + vb.var() / S)
        print(f"pixel {pix[i]}: mis {va.mean():.5f} (sd {va.std():.3f})  plain {vb.mean():.5f} "
              f"(sd {vb.std():.3f})")
        assert abs(va.mean() - vb.mean()) < 5 * se + 1e-6
        assert (va > 0).mean() >= (vb > 0).mean() and va.std() < vb.std()


def test_no_vertex_equals_plain():
    scene = sg.room_scene(2000, (3.0, 2.5, 2.5), 3, seed=31, emissive_frac=0.02)
    sc = Scene64(scene)
    cam = sg.Camera((0.4, 0.4, 1.0), (1.6, 1.3, 2.4), (0.0, 0.0, 1.0), 80.0, 8, 6)
    prm = Params(spp=2, max_depth=0)
    a = path_trace_nee(sc, cam, prm)
    b = path_trace(sc, cam, prm)
    np.testing.assert_array_equal(a["value"], b["value"])
    assert np.any(a["value"] > 0)
