"""Pins for the oracle's geometric edits: selection on hand-placed centres,
rigid motions in closed form, the frame identity and the tree cost of
hand-built trees."""
import numpy as np

from oracle.edits import frames, quat_mul, rigid, rotation_matrix, sah_cost, select_box


def test_select_box_hand_placed():
    pos = np.array([[0.0, 1.0, 0.5, 1.0000001, -0.1, 0.5],
                    [0.0, 1.0, 0.5, 0.5, 0.5, 0.5],
                    [0.0, 1.0, 0.5, 0.5, 0.5, 1.0]], dtype=np.float32)
    # closed box: the corners and the face are inside, just outside is not
    np.testing.assert_array_equal(select_box(pos, (0, 0, 0), (1, 1, 1)), [0, 1, 2, 5])
    assert select_box(pos, (2, 2, 2), (3, 3, 3)).size == 0


def test_rigid_quarter_turns_and_inverse():
    rng = np.random.default_rng(2)
    pos = rng.uniform(-1, 1, (3, 5))
    rot = rng.normal(size=(4, 5))
    rot /= np.linalg.norm(rot, axis=0)
    h = np.sqrt(0.5)
    # a quarter turn about z through the origin maps (x, y, z) to (-y, x, z)
    p1, q1 = rigid(pos, rot, np.arange(5), (h, 0.0, 0.0, h), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    np.testing.assert_allclose(p1, np.stack([-pos[1], pos[0], pos[2]]), atol=1e-15)
    # about x through the pivot (0, 1, 0), then moved by t: (x, y, z) -> (x, 1 - z, y - 1) + t
    t = np.array([0.5, -2.0, 3.0])
    p2, _ = rigid(pos, rot, np.arange(5), (h, h, 0.0, 0.0), (0.0, 1.0, 0.0), t)
    np.testing.assert_allclose(p2, np.stack([pos[0], 1.0 - pos[2], pos[1] - 1.0]) + t[:, None], atol=1e-15)
    # r then its inverse (w, -x, -y, -z) about the same pivot gives back the input (q up to sign)
    r = rng.normal(size=4)
    r /= np.linalg.norm(r)
    pv = (0.3, -0.2, 0.7)
    p3, q3 = rigid(pos, rot, np.arange(5), r, pv, (0.0, 0.0, 0.0))
    p4, q4 = rigid(p3, q3, np.arange(5), r * np.array([1, -1, -1, -1]), pv, (0.0, 0.0, 0.0))
    np.testing.assert_allclose(p4, pos, atol=1e-14)
    np.testing.assert_allclose(q4, rot, atol=1e-14)
    # untouched surfels stay put
    p5, q5 = rigid(pos, rot, np.array([1, 3]), r, pv, t)
    np.testing.assert_array_equal(p5[:, [0, 2, 4]], pos[:, [0, 2, 4]])
    np.testing.assert_array_equal(q5[:, [0, 2, 4]], rot[:, [0, 2, 4]])


def test_frame_identity():
    # the frame of r (x) q is R(r) applied to the frame of q
    rng = np.random.default_rng(3)
    q = rng.normal(size=(4, 6))
    r = rng.normal(size=4)
    r /= np.linalg.norm(r)
    tu, tv, n = frames(q)
    tu2, tv2, n2 = frames(quat_mul(r[:, None], q))
    R = rotation_matrix(r)
    np.testing.assert_allclose(tu2, tu @ R.T, atol=1e-14)
    np.testing.assert_allclose(tv2, tv @ R.T, atol=1e-14)
    np.testing.assert_allclose(n2, n @ R.T, atol=1e-14)


def test_sah_cost_hand_trees():
    unit = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])           # area 6
    half = np.array([[0.0, 0.0, 0.0], [0.5, 1.0, 1.0]])           # area 4
    # one root with two children of half the unit cube: 1 + (4 + 4) / 6
    assert abs(sah_cost([half, half + [[0.5, 0, 0], [0.5, 0, 0]]], unit) - (1 + 8 / 6)) < 1e-15
    # a flat child (zero thickness) has the area of its two faces
    flat = np.array([[0.0, 0.0, 0.5], [1.0, 1.0, 0.5]])
    assert abs(sah_cost([flat], unit) - (1 + 2 / 6)) < 1e-15
