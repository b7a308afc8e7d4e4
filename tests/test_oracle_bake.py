"""Pins for the oracle's light baking (Sec. 3.4, Eq. 10): SMPTE ST 2084
reference values, derivatives against central differences, the adjoint
identity that linearity in r gives, a hand-computed weight sum, and Adam's
first step in closed form."""
import os

import numpy as np

import scenegen as sg
from oracle import Params
from oracle.bake import adam_step, bake_loss, pq, pq_grad, zero_bounce_radiance_grad
from oracle.render import zero_bounce
from oracle.tracer import Scene64


def test_pq_reference_values():
    # ST 2084 code values for 1, 10, 100, 1000 and 10000 cd/m^2 (tests/golden),
    # and the curve's offset at zero, c1^m2
    ref = np.loadtxt(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "pq_st2084.txt"))
    L, N = ref[:, 0], ref[:, 1]
    assert L.size == 5
    np.testing.assert_allclose(pq(L), N, atol=6e-5)
    assert abs(pq(10000.0) - 1.0) < 1e-15
    assert abs(pq(0.0) - (3424.0 / 4096.0) ** (2523.0 / 4096.0 * 128.0)) < 1e-20
    assert np.all(np.diff(pq(np.linspace(0.0, 20.0, 200))) > 0)


def test_pq_grad_central_differences():
    L = np.array([1e-3, 0.05, 0.7, 3.0, 18.0, 250.0])
    h = 1e-6 * L
    fd = (pq(L + h) - pq(L - h)) / (2 * h)
    np.testing.assert_allclose(pq_grad(L), fd, rtol=1e-6)
    assert pq_grad(-1.0) == 0.0


def test_bake_loss_gradient_central_differences():
    rng = np.random.default_rng(3)
    L0 = rng.uniform(0.01, 5.0, (4, 5, 3))
    Lpt = rng.uniform(0.01, 5.0, (4, 5, 3))
    loss, g = bake_loss(L0, Lpt)
    assert np.isclose(loss, np.abs(pq(L0) - pq(Lpt)).mean())
    for k in rng.choice(L0.size, 12, replace=False):
        e = np.zeros(L0.size)
        h = 1e-7 * L0.flat[k]
        e[k] = h
        fd = (bake_loss(L0 + e.reshape(L0.shape), Lpt)[0] - bake_loss(L0 - e.reshape(L0.shape), Lpt)[0]) / (2 * h)
        assert abs(fd - g.flat[k]) <= 1e-6 * abs(g.flat[k]) + 1e-12


def _stack3():
    # three axis-aligned surfels on the z axis at z = 1, 2, 3, seen head-on
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)   # noqa: E731
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 2.0, 3.0]])
    rot = np.zeros((4, 3))
    rot[0] = 1.0
    sigma = np.array([0.5, 0.25, 0.75])
    return sg.Scene(f32(pos), f32(rot), f32(np.full((2, 3), 0.1)), f32(sigma), f32(np.full((3, 3), 0.5)),
                    f32(np.ones((3, 3))), f32(np.zeros(3)), bounds=(np.full(3, -1.0), np.full(3, 4.0))), sigma


def test_radiance_grad_hand_weights():
    scene, sigma = _stack3()
    cam = sg.Camera((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), (0.0, 1.0, 0.0), 10.0, 1, 1)
    dL = np.array([[0.3, -1.0, 2.0]])
    g = zero_bounce_radiance_grad(Scene64(scene), cam, Params(spp=1), dL)
    # the pixel-centre ray hits each centre (u = v = 0, alpha = sigma) in z order
    s = sigma.astype(np.float32).astype(np.float64)
    w = np.array([s[0], (1 - s[0]) * s[1], (1 - s[0]) * (1 - s[1]) * s[2]])
    np.testing.assert_allclose(g, w[:, None] * dL, rtol=1e-14, atol=1e-16)


def test_radiance_grad_adjoint_identity():
    # L_o^0 is linear in r, so <dL, L_o^0(r)> = <grad, r> for every r
    scene = sg.room_scene(3000, (3.0, 2.5, 2.5), 2, seed=17, emissive_frac=0.05)
    cam = sg.Camera((0.4, 0.5, 1.1), (2.4, 1.8, 1.6), (0.0, 0.0, 1.0), 70.0, 10, 8)
    prm = Params(spp=1)
    rng = np.random.default_rng(5)
    sc = Scene64(scene)
    sc.r = rng.uniform(0.0, 3.0, sc.r.shape)
    dL = rng.uniform(-1.0, 1.0, (cam.width * cam.height, 3))
    L0, _ = zero_bounce(sc, cam, prm)
    g = zero_bounce_radiance_grad(sc, cam, prm, dL)
    lhs = float((dL * L0).sum())
    rhs = float((g * sc.r).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    assert np.count_nonzero(g.sum(axis=1)) > 10


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(9)
    r = rng.uniform(1.0, 2.0, 50)
    g = rng.uniform(-1.0, 1.0, 50)
    r1, m, v = adam_step(r, g, np.zeros(50), np.zeros(50), 1, 0.01)
    # m_hat = g, v_hat = g^2: the first step is -lr sign(g)
    np.testing.assert_allclose(r1, r - 0.01 * np.sign(g), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
    # the clamp at zero
    r2, _, _ = adam_step(np.full(3, 0.005), np.ones(3), np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.all(r2 == 0.0)
