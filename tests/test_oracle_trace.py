"""Pins for the oracle's tracer: one surfel's hit in closed form, misses at
each rejection rule, a coplanar stack whose transmittance and stopping index
are closed forms, the compositing identities of front-to-back blending, and
an independent pure-Python per-ray loop on tiny random scenes."""
import math

import numpy as np
import pytest

import scenegen as sg
from oracle import Params
from oracle.tracer import Scene64, trace, composite_list


def _scene(pos, rot, scale, opacity, albedo=None, radiance=None, emissive=None):
    n = len(opacity)
    f = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return dict(pos=f(np.array(pos).T), rot=f(np.array(rot).T), scale=f(np.array(scale).T), opacity=f(opacity),
                albedo=f(np.array(albedo if albedo is not None else [[0.5, 0.5, 0.5]] * n).T),
                radiance=f(np.array(radiance if radiance is not None else [[0.0, 0.0, 0.0]] * n).T),
                emissive=f(emissive if emissive is not None else [0.0] * n))


def _qz(theta):
    return [math.cos(theta / 2), 0.0, 0.0, math.sin(theta / 2)]


def test_single_surfel_closed_form():
    # surfel in the plane z = 5 turned about z by the quaternion (3, 0, 0, 1)
    # (exact in float32; cos = 0.8, sin = 0.6 after normalisation); the ray
    # from the origin aims at p + a t_u + b t_v, so t = |x|, u = a / s_u and
    # v = b / s_v exactly
    su, sv, sig = 0.25, 0.125, 0.75
    a, b = 0.3, -0.2
    p = np.array([0.5, -0.25, 5.0])
    tu = np.array([0.8, 0.6, 0.0])
    tv = np.array([-0.6, 0.8, 0.0])
    x = p + a * tu + b * tv
    sc = Scene64(_scene([p], [[3.0, 0.0, 0.0, 1.0]], [[su, sv]], [sig], albedo=[[0.2, 0.4, 0.6]],
                        radiance=[[3.0, 2.0, 1.0]], emissive=[0.25]))
    w = x / np.linalg.norm(x)
    seg = trace(sc, np.zeros((1, 3)), w[None], Params())[0]
    u, v = a / su, b / sv
    g = math.exp(-0.5 * (u * u + v * v))
    al = sig * g
    assert list(seg.hits) == [0]
    assert seg.t[0] == pytest.approx(np.linalg.norm(x), rel=1e-9)
    assert seg.alpha[0] == pytest.approx(al, rel=1e-9)
    assert seg.A == pytest.approx(al, rel=1e-9)
    np.testing.assert_allclose(seg.R, al * np.array([3.0, 2.0, 1.0]), rtol=1e-9)
    np.testing.assert_allclose(seg.P, al * np.array([0.2, 0.4, 0.6]), rtol=1e-7)
    assert seg.E == pytest.approx(0.25 * al, rel=1e-9)
    assert seg.Dt == pytest.approx(np.linalg.norm(x), rel=1e-9)
    np.testing.assert_allclose(seg.Nt, [0, 0, -1], atol=1e-12)     # turned toward the origin
    # from the far side the normal flips to +z
    seg2 = trace(sc, np.array([[x[0], x[1], 9.0]]), np.array([[0.0, 0.0, -1.0]]), Params())[0]
    np.testing.assert_allclose(seg2.Nt, [0, 0, 1], atol=1e-12)
    assert seg2.t[0] == pytest.approx(4.0, rel=1e-9)


def test_rejections():
    p = [0.0, 0.0, 2.0]
    sc = Scene64(_scene([p], [[1, 0, 0, 0]], [[0.1, 0.1]], [0.9]))
    prm = Params()
    O = np.zeros((1, 3))
    # just inside and just outside the 3-sigma rim along t_u
    for off, hit in ((0.2999, True), (0.3001, False)):
        x = np.array([off, 0.0, 2.0])
        assert trace(sc, O, (x / np.linalg.norm(x))[None], prm)[0].hit == hit
    # behind the origin, and closer than t_min
    assert not trace(sc, O, np.array([[0.0, 0.0, -1.0]]), prm)[0].hit
    assert not trace(sc, np.array([[0.0, 0.0, 2.0 - 5e-4]]), np.array([[0.0, 0.0, 1.0]]), prm)[0].hit
    assert trace(sc, np.array([[0.0, 0.0, 2.0 - 2e-3]]), np.array([[0.0, 0.0, 1.0]]), prm)[0].hit
    # parallel to the plane
    assert not trace(sc, np.array([[-1.0, 0.0, 2.0]]), np.array([[1.0, 0.0, 0.0]]), prm)[0].hit
    # zero opacity is treated as deleted
    sc0 = Scene64(_scene([p], [[1, 0, 0, 0]], [[0.1, 0.1]], [0.0]))
    assert not trace(sc0, O, np.array([[0.0, 0.0, 1.0]]), prm)[0].hit


def test_coplanar_stack_order_and_stop():
    # 9 coplanar surfels with the same centre: g = 1 on the axis, alpha = sigma
    # = 0.9, so T_i = 0.1^i: T_4 = 1e-4 is not below T_min, T_5 = 1e-5 is, and
    # exactly 5 hits are blended, in index order
    n = 9
    sc = Scene64(_scene([[0.0, 0.0, 3.0]] * n, [_qz(0.1 * i) for i in range(n)], [[0.2, 0.3]] * n,
                        [0.9] * n, albedo=[[0.1 * i, 0.5, 0.5] for i in range(n)]))
    seg = trace(sc, np.zeros((1, 3)), np.array([[0.0, 0.0, 1.0]]), Params())[0]
    assert list(seg.hits) == [0, 1, 2, 3, 4]
    assert seg.n_acc == n
    s32 = float(np.float32(0.9))
    assert seg.T == pytest.approx((1 - s32) ** 5, rel=1e-12)
    assert seg.Dt == pytest.approx(3.0, rel=1e-12)
    w = s32 * (1 - s32) ** np.arange(5)
    rho0 = np.array([float(np.float32(0.1 * i)) for i in range(5)])
    assert seg.P[0] == pytest.approx(float(np.sum(w * rho0)), rel=1e-12)
    # exact (t, index) order gives the same list for exact ties
    seg0 = trace(sc, np.zeros((1, 3)), np.array([[0.0, 0.0, 1.0]]), Params(depth_quantum=0.0))[0]
    assert list(seg0.hits) == [0, 1, 2, 3, 4]


def test_compositing_identities():
    rng = np.random.default_rng(3)
    for _ in range(50):
        k = rng.integers(1, 30)
        al = rng.uniform(0.01, 0.99, k)
        vals = rng.uniform(-1, 1, (k, 3))
        V, w, Ts, stop = composite_list(al, vals, 1e-4)
        assert w.sum() + Ts[-1] == pytest.approx(1.0, abs=1e-14)         # telescoping
        Vc, _, Tc, _ = composite_list(al, np.ones((k, 1)) * 2.5, 1e-4)
        assert Vc[0] == pytest.approx(2.5 * (1 - Tc[-1]), rel=1e-13)     # constant v -> A v
        # transmittance after all hits does not depend on their order
        perm = rng.permutation(k)
        _, _, T1, _ = composite_list(al, vals, 0.0)
        _, _, T2, _ = composite_list(al[perm], vals[perm], 0.0)
        assert T1[-1] == pytest.approx(T2[-1], rel=1e-12)
        # split associativity: V = V_front + T_front V_back
        j = int(rng.integers(0, k))
        Vall, _, _, _ = composite_list(al, vals, 0.0)
        Vf, _, Tf, _ = composite_list(al[:j], vals[:j], 0.0) if j else (np.zeros(3), None, [1.0], 0)
        Vb, _, _, _ = composite_list(al[j:], vals[j:], 0.0)
        np.testing.assert_allclose(Vall, Vf + (Tf[-1] if j else 1.0) * Vb, atol=1e-14)


def _slow_trace(scene, o, w, prm):
    """Independent per-ray loop: plain Python floats, one surfel at a time."""
    pos, rot, sc_, op = scene["pos"], scene["rot"], scene["scale"], scene["opacity"]
    hits = []
    for i in range(op.shape[0]):
        qw, qx, qy, qz = (float(v) for v in rot[:, i])
        nq = math.sqrt(qw * qw + qx * qx + qy * qy + qz * qz)
        qw, qx, qy, qz = qw / nq, qx / nq, qy / nq, qz / nq
        tu = (1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy + qw * qz), 2 * (qx * qz - qw * qy))
        tv = (2 * (qx * qy - qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz + qw * qx))
        nn = (tu[1] * tv[2] - tu[2] * tv[1], tu[2] * tv[0] - tu[0] * tv[2], tu[0] * tv[1] - tu[1] * tv[0])
        p = [float(v) for v in pos[:, i]]
        den = sum(w[c] * nn[c] for c in range(3))
        if abs(den) <= 1e-12 or float(op[i]) == 0:
            continue
        t = sum((p[c] - o[c]) * nn[c] for c in range(3)) / den
        x = [o[c] + t * w[c] - p[c] for c in range(3)]
        u = sum(x[c] * tu[c] for c in range(3)) / float(sc_[0, i])
        v = sum(x[c] * tv[c] for c in range(3)) / float(sc_[1, i])
        if t > prm.t_min and u * u + v * v <= prm.k_sigma ** 2:
            hits.append((math.floor(t / prm.depth_quantum), i, float(op[i]) * math.exp(-0.5 * (u * u + v * v))))
    hits.sort()
    out, T = [], 1.0
    for _, i, a in hits:
        out.append(i)
        T *= 1 - a
        if T < prm.T_min:
            break
    return out, 1 - T if out else 0.0


def test_against_per_ray_loop():
    prm = Params()
    for seed in range(4):
        scene = sg.cloud_scene(50, seed=100 + seed).arrays()
        scene["scale"] = scene["scale"] * np.float32(5.0)
        sc = Scene64(scene)
        cam = sg.Camera((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0, 12, 12)
        from oracle.frames import camera_rays
        px, py = np.meshgrid(np.arange(12), np.arange(12))
        O, W = camera_rays(cam, px.ravel(), py.ravel())
        segs = trace(sc, O, W, prm)
        nhit = 0
        for o, w, seg in zip(O, W, segs):
            ref, A = _slow_trace(scene, o, w, prm)
            assert list(seg.hits) == ref
            assert seg.A == pytest.approx(A, abs=1e-12)
            nhit += bool(ref)
        assert nhit > 20
