"""Pins for the oracle's frames: closed-form rotations, the pinhole camera's
geometry, the hemisphere frame and the cosine-weighted sampler's moments."""
import numpy as np

import scenegen as sg
from oracle import philox
from oracle.frames import quat_frames, camera_rays, camera_basis, hemisphere_frame, cosine_direction


def test_rotation_about_z():
    th = np.array([0.0, 0.3, 1.0, 2.5, -1.2])
    q = np.stack([np.cos(th / 2), 0 * th, 0 * th, np.sin(th / 2)])
    tu, tv, n = quat_frames(q * 3.7)           # any norm
    np.testing.assert_allclose(tu, np.stack([np.cos(th), np.sin(th), 0 * th], 1), atol=1e-15)
    np.testing.assert_allclose(tv, np.stack([-np.sin(th), np.cos(th), 0 * th], 1), atol=1e-15)
    np.testing.assert_allclose(n, np.tile([0.0, 0, 1], (th.size, 1)), atol=1e-15)


def test_rotation_about_x_quarter_turn():
    # +90 deg about x: e_y -> e_z, e_z -> -e_y
    q = np.array([[np.cos(np.pi / 4)], [np.sin(np.pi / 4)], [0.0], [0.0]])
    tu, tv, n = quat_frames(q)
    np.testing.assert_allclose(tu[0], [1, 0, 0], atol=1e-15)
    np.testing.assert_allclose(tv[0], [0, 0, 1], atol=1e-15)
    np.testing.assert_allclose(n[0], [0, -1, 0], atol=1e-15)


def test_generator_quaternions_reproduce_face_normals():
    s = sg.room_scene(2000, seed=9, n_boxes=3)
    tu, tv, n = quat_frames(s.rot)
    # every generated normal is axis aligned to float32 precision
    assert np.all(np.abs(np.abs(n).max(axis=1) - 1) < 1e-6)
    np.testing.assert_allclose(np.einsum("ij,ij->i", tu, tv), 0, atol=1e-12)


def test_camera_geometry():
    cam = sg.Camera((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0, 64, 48)
    eye, right, up, fwd = camera_basis(cam)
    np.testing.assert_allclose(fwd, [0, 0, 1])
    np.testing.assert_allclose(np.cross(right, up), -fwd, atol=1e-15)
    # the rays through the two central pixel columns/rows are symmetric
    o, d = camera_rays(cam, np.array([31, 32]), np.array([23, 24]))
    np.testing.assert_allclose(d[0] @ right, -(d[1] @ right), atol=1e-15)
    np.testing.assert_allclose(d[0] @ up, -(d[1] @ up), atol=1e-15)
    # a pixel at the top edge's centre column sees half the vertical fov
    # minus half a pixel: tan(angle) = tan(30deg) * (1 - 1/H)
    cam2 = sg.Camera((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 0.0, 1.0), 60.0, 65, 49)
    o, d = camera_rays(cam2, np.array([32]), np.array([0]))
    ang = np.arctan2(d[0, 2], d[0, 0])
    np.testing.assert_allclose(np.tan(ang), np.tan(np.pi / 6) * (1 - 1 / 49), rtol=1e-14)
    assert abs(d[0, 1]) < 1e-15
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1, atol=1e-15)


def test_hemisphere_frame_orthonormal_and_continuous_on_axes():
    rng = np.random.default_rng(0)
    n = rng.standard_normal((1000, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    axes = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    n = np.concatenate([n, axes])
    b1, b2, mlen = hemisphere_frame(n)
    for a, b in ((b1, b2), (b1, n), (b2, n)):
        np.testing.assert_allclose(np.einsum("ij,ij->i", a, b), 0, atol=1e-12)
    for a in (b1, b2):
        np.testing.assert_allclose(np.linalg.norm(a, axis=1), 1, atol=1e-12)
    np.testing.assert_allclose(np.einsum("ij,ij->i", np.cross(b1, b2), n), 1, atol=1e-12)
    # axis-aligned normals are far from the frame's only singularity (n = +-h)
    assert mlen[-6:].min() > 0.5
    eps = 1e-7       # continuity: a tiny tilt of a wall normal barely moves the frame
    t1, _, _ = hemisphere_frame(np.array([[1.0, eps, 0.0]]) / np.linalg.norm([1.0, eps, 0.0]))
    np.testing.assert_allclose(t1[0], b1[-6], atol=1e-6)


def test_cosine_sampler_moments():
    M = 400_000
    u0, u1, _, _ = philox.uniforms(np.arange(M), 0, 0, 0, 11)
    for nrm in ([0.0, 0.0, 1.0], [0.3, -0.5, 0.8]):
        nv = np.array(nrm) / np.linalg.norm(nrm)
        d = cosine_direction(np.tile(nv, (M, 1)), u0, u1)
        np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1, atol=1e-12)
        c = d @ nv
        assert c.min() >= 0
        se = np.sqrt(1 / 18 / M)                       # Var[cos] = 1/2 - 4/9
        assert abs(c.mean() - 2 / 3) < 4 * se
        se2 = np.sqrt((1 / 3 - 1 / 4) / M)             # Var[cos^2] = 1/3 - 1/4
        assert abs((c * c).mean() - 0.5) < 4 * se2
        h, _ = np.histogram(c * c, bins=40, range=(0, 1))  # cos^2 ~ U(0,1)
        e = M / 40
        assert ((h - e) ** 2 / e).sum() < 85           # 39 dof
        # azimuth uniform about the normal
        b1, b2, _ = hemisphere_frame(np.tile(nv, (M, 1)))
        phi = np.arctan2(np.einsum("ij,ij->i", d, b2), np.einsum("ij,ij->i", d, b1))
        h, _ = np.histogram(phi, bins=36, range=(-np.pi, np.pi))
        e = M / 36
        assert ((h - e) ** 2 / e).sum() < 80
