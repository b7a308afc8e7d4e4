"""Frames and directions, float64.

* quat_frames: a surfel's tangent axes t_u, t_v are the first two columns of
  the rotation matrix of its normalised quaternion (w, x, y, z; Hamilton
  convention), and its normal is t_u x t_v (Sec. 3.1, Eq. 1 and the traced
  normal of Eq. 3). Pinned by closed-form rotations (tests/test_oracle_frames).
* camera_rays: pinhole camera with vertical field of view through pixel
  centres, row 0 at the top. Eye, look-at, up and field of view are float32
  values (the camera record), upcast exactly. The camera basis is fwd = normalize(look_at -
  eye), right = normalize(fwd x up), up' = right x fwd. Pinned by
  symmetry and angle checks.
* hemisphere_frame / cosine_direction: the paper samples the new direction in
  the hemisphere about the traced normal (Sec. 3.1 "Light Bouncing") with
  cosine weighting (appendix, "Path Tracing"). The frame is Gram-Schmidt of
  the fixed helper h = normalize(1, 2, 3) against the normal, b1 =
  normalize(h - (h.N)N), b2 = N x b1, which is continuous for the
  axis-aligned normals of room scenes; the direction is Malley's method
  r = sqrt(u0), phi = 2 pi u1. Pinned by sampler moments and orthonormality.
"""
import numpy as np

HELPER = np.array([1.0, 2.0, 3.0]) / np.sqrt(14.0)


def quat_frames(rot):
    """rot: [4,N] (w,x,y,z), any nonzero norm -> t_u, t_v, n each [N,3]."""
    q = np.asarray(rot, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=0, keepdims=True)
    w, x, y, z = q
    tu = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y + w * z), 2 * (x * z - w * y)], axis=1)
    tv = np.stack([2 * (x * y - w * z), 1 - 2 * (x * x + z * z), 2 * (y * z + w * x)], axis=1)
    n = np.cross(tu, tv)
    return tu, tv, n


def _f32(v):
    """Camera parameters are float32 values (the renderers' camera record)."""
    return np.asarray(v, dtype=np.float32).astype(np.float64)


def camera_basis(cam):
    eye = _f32(cam.eye)
    fwd = _f32(cam.look_at) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, _f32(cam.up))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    return eye, right, up, fwd


def camera_rays(cam, px, py, jitter=None):
    """Origins [M,3] and unit directions [M,3] for pixel coordinates px, py
    (integer arrays). jitter: optional (jx, jy) in [0,1) replacing the 0.5
    pixel-centre offset."""
    eye, right, up, fwd = camera_basis(cam)
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    ox, oy = (0.5, 0.5) if jitter is None else jitter
    tan_h = np.tan(np.deg2rad(float(_f32(cam.vfov_deg))) * 0.5)
    aspect = cam.width / cam.height
    nx = (2.0 * (px + ox) / cam.width - 1.0) * tan_h * aspect
    ny = (1.0 - 2.0 * (py + oy) / cam.height) * tan_h
    d = nx[:, None] * right[None, :] + ny[:, None] * up[None, :] + fwd[None, :]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(eye, d.shape).copy()
    return o, d


def hemisphere_frame(nrm):
    """nrm: [M,3] unit -> b1, b2 [M,3], and |h - (h.N)N| (singular near 0)."""
    m = HELPER[None, :] - (nrm @ HELPER)[:, None] * nrm
    mlen = np.linalg.norm(m, axis=1)
    b1 = m / mlen[:, None]
    b2 = np.cross(nrm, b1)
    return b1, b2, mlen


def cosine_direction(nrm, u0, u1):
    """Cosine-weighted direction about unit normals nrm [M,3]; pdf = cos/pi."""
    b1, b2, _ = hemisphere_frame(nrm)
    r = np.sqrt(u0)
    phi = 2.0 * np.pi * u1
    return ((r * np.cos(phi))[:, None] * b1 + (r * np.sin(phi))[:, None] * b2
            + np.sqrt(1.0 - u0)[:, None] * nrm)
