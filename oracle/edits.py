"""Geometric scene edits (Sec. 1 and Sec. 5: moving, importing and deleting
objects), float64.

* select_box: the surfels whose centre lies in the closed box [lo, hi],
  compared in float32 as the centres are stored, ascending.
* rigid: the rigid motion p' = R(r) (p - pivot) + pivot + t of the centres and
  q' = r (x) q (Hamilton product, r a unit quaternion) of the orientations,
  so that the frame of q' is R(r) applied to the frame of q; scales,
  opacity and the attributes are unchanged.
* delete: opacity 0 (the tracer skips such surfels).
* duplicate: the selected surfels' full records, moved by a rigid motion,
  appended after the scene's (a new scene of n + count surfels).
* sah_cost: the surface-area cost of a 4-wide tree, 1 + the sum over every
  node of the areas of its children's boxes, divided by the area of the
  root's box: the expected number of box tests of a random ray that crosses
  the root (up to the cost ratio of a box and a surfel test).

Pinned by tests/test_oracle_edits.py: a hand-placed selection with centres
on the box faces; rotations by a quarter turn about z and about x in
closed form, r followed by its inverse giving back the input, the frame
identity R(r (x) q) = R(r) R(q), and translations; the cost of hand-built
trees.
"""
import numpy as np

from .frames import quat_frames


def select_box(pos, lo, hi):
    p = np.asarray(pos, dtype=np.float32)
    lo = np.asarray(lo, dtype=np.float32)[:, None]
    hi = np.asarray(hi, dtype=np.float32)[:, None]
    return np.nonzero(np.all((p >= lo) & (p <= hi), axis=0))[0]


def quat_mul(a, b):
    """Hamilton product a (x) b of quaternions (w, x, y, z) along axis 0."""
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.array([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def rotation_matrix(r):
    """R(r) of a unit quaternion r = (w, x, y, z)."""
    w, x, y, z = np.asarray(r, dtype=np.float64) / np.linalg.norm(r)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def rigid(pos, rot, idx, r, pivot, t):
    """Centres [3, n] and quaternions [4, n] (float64) after moving the
    surfels idx by the rigid motion (r unit, pivot, t)."""
    pos = np.asarray(pos, dtype=np.float64).copy()
    rot = np.asarray(rot, dtype=np.float64).copy()
    r = np.asarray(r, dtype=np.float64) / np.linalg.norm(r)
    R = rotation_matrix(r)
    pv = np.asarray(pivot, dtype=np.float64)[:, None]
    pos[:, idx] = R @ (pos[:, idx] - pv) + pv + np.asarray(t, dtype=np.float64)[:, None]
    rot[:, idx] = quat_mul(r[:, None], rot[:, idx])
    return pos, rot


def frames(rot):
    return quat_frames(rot)


def sah_cost(child_boxes, root_box):
    """child_boxes: [m, 2, 3] (lo, hi) of every child of every node; root_box
    [2, 3]. Returns 1 + sum of child areas / root area."""
    def area(b):
        e = np.maximum(b[..., 1, :] - b[..., 0, :], 0.0)
        return 2.0 * (e[..., 0] * e[..., 1] + e[..., 1] * e[..., 2] + e[..., 2] * e[..., 0])
    cb = np.asarray(child_boxes, dtype=np.float64)
    return 1.0 + float(area(cb).sum()) / float(area(np.asarray(root_box, dtype=np.float64)))
