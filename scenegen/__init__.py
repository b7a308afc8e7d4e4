"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws scenes, cameras, rays and request streams. It holds none of
the rendering method's arithmetic: no frames, no intersections, no
compositing and no sampling of bounce directions. Both the FP64 oracle and the
GPU path read the same float32 arrays produced here.

Scenes stand in for the paper's captured indoor datasets (FIPT, Eyeful Tower,
Blender scenes; Sec. 5 "Datasets"), which are not available: a cloud of random
2D Gaussians, and axis-aligned rooms whose walls, floor, ceiling and furniture
boxes are tiled with coplanar surfels, with a small fraction of emissive
ceiling-panel surfels. Scale (1e5 to 5e6 Gaussians) follows the paper's
200k-1M Gaussians (Sec. 5 "Implementation Details"); layer depth is tuned so
composited hits per ray land near the 63-79 the paper's appendix reports.

Surfel arrays are component-major float32 (SoA):
  pos [3,N], rot [4,N] quaternion (w,x,y,z), scale [2,N] (s_u, s_v),
  opacity [N], albedo [3,N], radiance [3,N], emissive [N].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Scene", "Camera", "cloud_scene", "room_scene", "multiroom_scene",
    "interior_cameras", "perturb", "random_rays", "config", "arrivals",
    "quat_from_axes", "furnace_scene",
]


@dataclass
class Scene:
    pos: np.ndarray
    rot: np.ndarray
    scale: np.ndarray
    opacity: np.ndarray
    albedo: np.ndarray
    radiance: np.ndarray
    emissive: np.ndarray
    boxes: list = field(default_factory=list)      # furniture (lo, hi) pairs, float64
    bounds: tuple = None                            # room extent (lo, hi), float64

    @property
    def n(self) -> int:
        return int(self.opacity.shape[0])

    def arrays(self) -> dict:
        return dict(pos=self.pos, rot=self.rot, scale=self.scale, opacity=self.opacity,
                    albedo=self.albedo, radiance=self.radiance, emissive=self.emissive)

    def copy(self) -> "Scene":
        return Scene(**{k: v.copy() for k, v in self.arrays().items()},
                     boxes=list(self.boxes), bounds=self.bounds)

    def save(self, path: str) -> None:
        np.savez(path, **self.arrays())

    @staticmethod
    def load(path: str) -> "Scene":
        with np.load(path, allow_pickle=False) as z:
            return Scene(**{k: np.ascontiguousarray(z[k]) for k in
                            ("pos", "rot", "scale", "opacity", "albedo", "radiance", "emissive")})


@dataclass
class Camera:
    eye: tuple
    look_at: tuple
    up: tuple
    vfov_deg: float
    width: int
    height: int


# ---------------------------------------------------------------------------
# orientation helpers (input construction only)
# ---------------------------------------------------------------------------

def quat_from_axes(tu: np.ndarray, tv: np.ndarray, n: np.ndarray) -> np.ndarray:
    """Unit quaternion (w,x,y,z) of the rotation whose matrix has columns
    (tu, tv, n). Inputs are float64 [M,3]; output float64 [4,M].

    Shepperd's branch on the largest of (trace, diagonal) keeps it stable.
    """
    m00, m11, m22 = tu[:, 0], tv[:, 1], n[:, 2]
    m01, m02 = tv[:, 0], n[:, 0]
    m10, m12 = tu[:, 1], n[:, 1]
    m20, m21 = tu[:, 2], tv[:, 2]
    tr = m00 + m11 + m22
    q = np.zeros((4, tu.shape[0]))
    c0 = tr > 0
    c1 = (~c0) & (m00 >= m11) & (m00 >= m22)
    c2 = (~c0) & (~c1) & (m11 >= m22)
    c3 = (~c0) & (~c1) & (~c2)
    s = np.sqrt(np.maximum(tr[c0] + 1.0, 1e-300)) * 2
    q[:, c0] = np.stack([0.25 * s, (m21[c0] - m12[c0]) / s, (m02[c0] - m20[c0]) / s, (m10[c0] - m01[c0]) / s])
    s = np.sqrt(np.maximum(1.0 + m00[c1] - m11[c1] - m22[c1], 1e-300)) * 2
    q[:, c1] = np.stack([(m21[c1] - m12[c1]) / s, 0.25 * s, (m01[c1] + m10[c1]) / s, (m02[c1] + m20[c1]) / s])
    s = np.sqrt(np.maximum(1.0 + m11[c2] - m00[c2] - m22[c2], 1e-300)) * 2
    q[:, c2] = np.stack([(m02[c2] - m20[c2]) / s, (m01[c2] + m10[c2]) / s, 0.25 * s, (m12[c2] + m21[c2]) / s])
    s = np.sqrt(np.maximum(1.0 + m22[c3] - m00[c3] - m11[c3], 1e-300)) * 2
    q[:, c3] = np.stack([(m10[c3] - m01[c3]) / s, (m02[c3] + m20[c3]) / s, (m12[c3] + m21[c3]) / s, 0.25 * s])
    return q / np.linalg.norm(q, axis=0, keepdims=True)


def _loguniform(rng, lo, hi, size):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


# ---------------------------------------------------------------------------
# scenes
# ---------------------------------------------------------------------------

def cloud_scene(n: int = 2000, seed: int = 1, emissive_frac: float = 0.01) -> Scene:
    """Random cloud: centres U[-1,1]^3, Haar-uniform rotations (normalised 4-D
    standard normal), scales log-uniform [0.02, 0.1], opacity U[0.5, 0.99],
    albedo U[0.1, 0.8]^3, 1% emitters with radiance U[1,10]^3 and e=1."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-1.0, 1.0, (3, n))
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    scale = _loguniform(rng, 0.02, 0.1, (2, n))
    opacity = rng.uniform(0.5, 0.99, n)
    albedo = rng.uniform(0.1, 0.8, (3, n))
    n_e = max(1, int(round(emissive_frac * n)))
    em_idx = rng.choice(n, n_e, replace=False)
    radiance = np.zeros((3, n))
    radiance[:, em_idx] = rng.uniform(1.0, 10.0, (3, n_e))
    emissive = np.zeros(n)
    emissive[em_idx] = 1.0
    return Scene(_f32(pos), _f32(q), _f32(scale), _f32(opacity), _f32(albedo), _f32(radiance), _f32(emissive),
                 bounds=(np.array([-1.0, -1, -1]), np.array([1.0, 1, 1])))


class _Faces:
    """Planar rectangles: origin o, edge vectors e1, e2, unit normal nrm,
    the axis the plane is normal to, and an optional rectangular hole in
    (a, b) face coordinates."""

    def __init__(self):
        self.items = []

    def add(self, o, e1, e2, nrm, hole=None):
        o, e1, e2, nrm = (np.asarray(v, dtype=np.float64) for v in (o, e1, e2, nrm))
        axis = int(np.argmax(np.abs(nrm)))
        area = np.linalg.norm(e1) * np.linalg.norm(e2)
        if hole is not None:
            (a0, a1), (b0, b1) = hole
            area -= (a1 - a0) * (b1 - b0) * area
        self.items.append((o, e1, e2, nrm, axis, area, hole))

    def areas(self):
        return np.array([it[5] for it in self.items])


def _room_faces(faces: _Faces, lo, hi, skip_x_lo=False, skip_x_hi=False):
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    L = np.array(hi) - np.array(lo)
    faces.add((x0, y0, z0), (L[0], 0, 0), (0, L[1], 0), (0, 0, 1))      # floor
    faces.add((x0, y0, z1), (L[0], 0, 0), (0, L[1], 0), (0, 0, -1))     # ceiling
    faces.add((x0, y0, z0), (L[0], 0, 0), (0, 0, L[2]), (0, 1, 0))      # y = y0
    faces.add((x0, y1, z0), (L[0], 0, 0), (0, 0, L[2]), (0, -1, 0))     # y = y1
    if not skip_x_lo:
        faces.add((x0, y0, z0), (0, L[1], 0), (0, 0, L[2]), (1, 0, 0))
    if not skip_x_hi:
        faces.add((x1, y0, z0), (0, L[1], 0), (0, 0, L[2]), (-1, 0, 0))


def _box_faces(faces: _Faces, lo, hi):
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    w, d, h = x1 - x0, y1 - y0, z1 - z0
    faces.add((x0, y0, z1), (w, 0, 0), (0, d, 0), (0, 0, 1))            # top
    faces.add((x0, y0, z0), (w, 0, 0), (0, 0, h), (0, -1, 0))
    faces.add((x0, y1, z0), (w, 0, 0), (0, 0, h), (0, 1, 0))
    faces.add((x0, y0, z0), (0, d, 0), (0, 0, h), (-1, 0, 0))
    faces.add((x1, y0, z0), (0, d, 0), (0, 0, h), (1, 0, 0))


def _sample_on_faces(rng, faces: _Faces, count: int, face_idx=None):
    """Centres uniform on the faces (area-proportional), each surfel exactly on
    its face plane in float32, normal = face normal, in-plane angle U[0,2pi)."""
    areas = faces.areas()
    counts = rng.multinomial(count, areas / areas.sum())
    P, TU, TV, NN = [], [], [], []
    for (o, e1, e2, nrm, axis, _area, hole), c in zip(faces.items, counts):
        if c == 0:
            continue
        a = rng.uniform(0, 1, c)
        b = rng.uniform(0, 1, c)
        if hole is not None:
            (a0, a1), (b0, b1) = hole
            bad = (a >= a0) & (a <= a1) & (b >= b0) & (b <= b1)
            while bad.any():
                a[bad] = rng.uniform(0, 1, bad.sum())
                b[bad] = rng.uniform(0, 1, bad.sum())
                bad = (a >= a0) & (a <= a1) & (b >= b0) & (b <= b1)
        p = o[None, :] + a[:, None] * e1[None, :] + b[:, None] * e2[None, :]
        p[:, axis] = np.float32(o[axis])        # exactly on the plane
        u1 = e1 / np.linalg.norm(e1)
        u2 = np.cross(nrm, u1)                  # (u1, u2, nrm) right-handed
        phi = rng.uniform(0, 2 * np.pi, c)
        tu = np.cos(phi)[:, None] * u1 + np.sin(phi)[:, None] * u2
        tv = np.cross(np.broadcast_to(nrm, tu.shape), tu)
        P.append(p)
        TU.append(tu)
        TV.append(tv)
        NN.append(np.broadcast_to(nrm, tu.shape))
    return np.concatenate(P), np.concatenate(TU), np.concatenate(TV), np.concatenate(NN)


def _furniture(rng, lo, hi, n_boxes, margin=0.3):
    boxes = []
    for _ in range(n_boxes):
        w, d = rng.uniform(0.4, 1.6, 2)
        h = rng.uniform(0.4, 1.2)
        cx = rng.uniform(lo[0] + margin + w / 2, hi[0] - margin - w / 2)
        cy = rng.uniform(lo[1] + margin + d / 2, hi[1] - margin - d / 2)
        b_lo = np.array([cx - w / 2, cy - d / 2, lo[2]], dtype=np.float32).astype(np.float64)
        b_hi = np.array([cx + w / 2, cy + d / 2, lo[2] + h], dtype=np.float32).astype(np.float64)
        boxes.append((b_lo, b_hi))
    return boxes


def _panels(rooms, n_panels, ceiling_drop=0.01, pw=1.2, pd=0.6):
    """Emitter panels on a regular grid per room ceiling, normal -z."""
    faces = _Faces()
    per_room = [n_panels // len(rooms) + (1 if i < n_panels % len(rooms) else 0) for i in range(len(rooms))]
    for (lo, hi), k in zip(rooms, per_room):
        if k == 0:
            continue
        Lx, Ly = hi[0] - lo[0], hi[1] - lo[1]
        nx = max(1, int(math.ceil(math.sqrt(k * Lx / Ly))))
        ny = max(1, int(math.ceil(k / nx)))
        z = float(np.float32(hi[2] - ceiling_drop))
        placed = 0
        for j in range(ny):
            for i in range(nx):
                if placed == k:
                    break
                cx = lo[0] + (i + 0.5) * Lx / nx
                cy = lo[1] + (j + 0.5) * Ly / ny
                faces.add((cx - pw / 2, cy - pd / 2, z), (pw, 0, 0), (0, pd, 0), (0, 0, -1))
                placed += 1
    return faces


def _assemble(rng, faces_ne, n_ne, faces_em, n_em, boxes, bounds):
    P, TU, TV, _ = _sample_on_faces(rng, faces_ne, n_ne)
    Pe, TUe, TVe, _ = _sample_on_faces(rng, faces_em, n_em)
    n = n_ne + n_em
    pos = np.concatenate([P, Pe])
    q = quat_from_axes(np.concatenate([TU, TUe]), np.concatenate([TV, TVe]),
                       np.cross(np.concatenate([TU, TUe]), np.concatenate([TV, TVe])))
    scale = _loguniform(rng, 0.01, 0.05, (2, n))
    opacity = rng.uniform(0.6, 0.99, n)
    albedo = rng.uniform(0.05, 0.9, (3, n))
    radiance = np.zeros((3, n))
    emissive = np.zeros(n)
    radiance[:, n_ne:] = rng.uniform(5.0, 20.0, n_em)[None, :]
    emissive[n_ne:] = 1.0
    perm = rng.permutation(n)                  # indices carry no face grouping
    return Scene(_f32(pos[perm].T), _f32(q[:, perm]), _f32(scale[:, perm]), _f32(opacity[perm]),
                 _f32(albedo[:, perm]), _f32(radiance[:, perm]), _f32(emissive[perm]),
                 boxes=boxes, bounds=bounds)


def _n_panels(n_em, mean_area=0.0175, layers=10.0, panel_area=0.72):
    return max(1, int(round(n_em * mean_area / layers / panel_area)))


def room_scene(n: int, size=(6.0, 4.0, 3.0), n_boxes: int = 12, seed: int = 2,
               emissive_frac: float = 0.005) -> Scene:
    """One axis-aligned room [0,Lx]x[0,Ly]x[0,Lz], z up, inward normals, with
    furniture boxes (5 faces, outward normals) and emissive ceiling panels."""
    rng = np.random.default_rng(seed)
    lo, hi = np.zeros(3), np.array(size, dtype=np.float64)
    boxes = _furniture(rng, lo, hi, n_boxes)
    faces = _Faces()
    _room_faces(faces, lo, hi)
    for b in boxes:
        _box_faces(faces, *b)
    n_em = max(1, int(round(emissive_frac * n)))
    em = _panels([(lo, hi)], _n_panels(n_em))
    return _assemble(rng, faces, n - n_em, em, n_em, boxes, (lo, hi))


def multiroom_scene(n: int, n_rooms: int = 3, size=(8.0, 6.0, 3.0), boxes_per_room: int = 40,
                    seed: int = 4, emissive_frac: float = 0.005, door=((2.5, 3.5), (0.0, 2.0))) -> Scene:
    """Rooms along x sharing walls at x = k*Lx; each shared wall is double
    sided (two coplanar faces, opposite normals) with a doorway y in door[0],
    z in door[1]."""
    rng = np.random.default_rng(seed)
    Lx, Ly, Lz = size
    rooms = [(np.array([k * Lx, 0.0, 0.0]), np.array([(k + 1) * Lx, Ly, Lz])) for k in range(n_rooms)]
    faces = _Faces()
    boxes = []
    for k, (lo, hi) in enumerate(rooms):
        _room_faces(faces, lo, hi, skip_x_lo=k > 0, skip_x_hi=k < n_rooms - 1)
        boxes += _furniture(rng, lo, hi, boxes_per_room)
    (ya, yb), (za, zb) = door
    hole = ((ya / Ly, yb / Ly), (za / Lz, zb / Lz))
    for k in range(1, n_rooms):
        x = k * Lx
        faces.add((x, 0, 0), (0, Ly, 0), (0, 0, Lz), (-1, 0, 0), hole=hole)
        faces.add((x, 0, 0), (0, Ly, 0), (0, 0, Lz), (1, 0, 0), hole=hole)
    for b in boxes:
        _box_faces(faces, *b)
    n_em = max(1, int(round(emissive_frac * n)))
    em = _panels(rooms, _n_panels(n_em))
    return _assemble(rng, faces, n - n_em, em, n_em, boxes,
                     (rooms[0][0], rooms[-1][1]))


def furnace_scene(n_layers: int = 12, radiance: float = 1.0, albedo: float = 0.5, half: float = 1.0,
                  scale: float = 2.0, opacity: float = 0.99) -> Scene:
    """Closed cube [-half, half]^3 whose six faces each carry n_layers coplanar
    surfels centred on the face, large enough that every point of every face
    is covered by all layers with high response; inward normals. Every surfel
    has radiance = `radiance` (grey), albedo = `albedo`, e = 1."""
    faces = []
    for axis in range(3):
        for sgn in (-1.0, 1.0):
            nrm = np.zeros(3)
            nrm[axis] = -sgn
            c = np.zeros(3)
            c[axis] = sgn * half
            faces.append((c, nrm))
    P, TU, TV = [], [], []
    for li in range(n_layers):
        for c, nrm in faces:
            helper = np.array([1.0, 0, 0]) if abs(nrm[0]) < 0.5 else np.array([0, 1.0, 0])
            tu = helper - nrm * np.dot(helper, nrm)
            tu /= np.linalg.norm(tu)
            ang = 2 * np.pi * li / n_layers
            tu2 = np.cos(ang) * tu + np.sin(ang) * np.cross(nrm, tu)
            P.append(c)
            TU.append(tu2)
            TV.append(np.cross(nrm, tu2))
    P, TU, TV = np.array(P), np.array(TU), np.array(TV)
    q = quat_from_axes(TU, TV, np.cross(TU, TV))
    n = P.shape[0]
    return Scene(_f32(P.T), _f32(q), _f32(np.full((2, n), scale)), _f32(np.full(n, opacity)),
                 _f32(np.full((3, n), albedo)), _f32(np.full((3, n), radiance)), _f32(np.ones(n)),
                 bounds=(np.full(3, -half), np.full(3, half)))


# ---------------------------------------------------------------------------
# cameras, rays, perturbation, request streams
# ---------------------------------------------------------------------------

def interior_cameras(scene: Scene, count: int, width: int, height: int, seed: int,
                     vfov: float = 60.0, clearance: float = 0.2) -> list:
    """Cameras at uniform interior positions (0.5 m from walls, z in [1, 2]),
    rejected within `clearance` of a furniture box; yaw U[0,2pi), pitch
    U[-15deg, 15deg]; up = +z."""
    rng = np.random.default_rng(seed)
    lo, hi = scene.bounds
    cams = []
    while len(cams) < count:
        p = rng.uniform([lo[0] + 0.5, lo[1] + 0.5, 1.0], [hi[0] - 0.5, hi[1] - 0.5, 2.0])
        if any(np.all(p >= b[0] - clearance) and np.all(p <= b[1] + clearance) for b in scene.boxes):
            continue
        yaw = rng.uniform(0, 2 * np.pi)
        pitch = np.deg2rad(rng.uniform(-15, 15))
        d = np.array([np.cos(pitch) * np.cos(yaw), np.cos(pitch) * np.sin(yaw), np.sin(pitch)])
        cams.append(Camera(tuple(map(float, p)), tuple(map(float, p + d)), (0.0, 0.0, 1.0), vfov, width, height))
    return cams


def perturb(scene: Scene, seed: int = 102, sigma: float = 0.01) -> Scene:
    """Target scene for the reconstruction loss: additive N(0, sigma^2) on
    centre, quaternion, albedo, opacity and emitter radiance; multiplicative
    exp(N(0, sigma^2)) on scales; clamps opacity to [0, 0.99], albedo to
    [0, 1], radiance >= 0; e unchanged."""
    rng = np.random.default_rng(seed)
    s = scene.copy()
    n = s.n
    s.pos = _f32(s.pos + sigma * rng.standard_normal((3, n)))
    s.rot = _f32(s.rot + sigma * rng.standard_normal((4, n)))
    s.scale = _f32(s.scale * np.exp(sigma * rng.standard_normal((2, n))))
    s.opacity = _f32(np.clip(s.opacity + sigma * rng.standard_normal(n), 0.0, 0.99))
    s.albedo = _f32(np.clip(s.albedo + sigma * rng.standard_normal((3, n)), 0.0, 1.0))
    em = s.emissive > 0
    r = s.radiance.astype(np.float64)
    r[:, em] = np.maximum(r[:, em] + sigma * rng.standard_normal((3, int(em.sum()))), 0.0)
    s.radiance = _f32(r)
    return s


def random_rays(scene: Scene, count: int, seed: int, inset: float = 0.05):
    """Rays with origins uniform inside the scene bounds (shrunk by `inset`)
    and directions uniform on the sphere. Returns float32 origin [3,M] and
    unit direction [3,M] (normalised in float64, then rounded)."""
    rng = np.random.default_rng(seed)
    lo, hi = scene.bounds
    o = rng.uniform(np.asarray(lo) + inset, np.asarray(hi) - inset, (count, 3)).T
    d = rng.standard_normal((3, count))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    return _f32(o), _f32(d)


def config(k: int, n_override: int | None = None):
    """The five benchmark configurations (scene seed = k):
      1: 2,000-surfel cloud, one 64x64 camera at (0,0,-3), 4 spp.
      2: 100k-surfel 6x4x3 m room, 12 boxes, 8 interior 256x256 cameras, 8 spp.
      3: 1M-surfel 8x6x3 m room, 40 boxes, one 1024x768 camera, 64 spp, depth 5.
      4: 5M surfels, three 8x6x3 m rooms with doorways, 120 boxes, 1920x1080,
         256 spp in 16-spp passes, depth 8.
      5: 3M-surfel resident room for serving.
    Returns (scene, cameras, params dict)."""
    if k == 1:
        sc = cloud_scene(n_override or 2000, seed=1)
        cams = [Camera((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0, 64, 64)]
        return sc, cams, dict(spp=4, max_depth=1, rr_start=3)
    if k == 2:
        sc = room_scene(n_override or 100_000, (6.0, 4.0, 3.0), 12, seed=2)
        cams = interior_cameras(sc, 8, 256, 256, seed=22)
        return sc, cams, dict(spp=8, max_depth=1, rr_start=3)
    if k == 3:
        sc = room_scene(n_override or 1_000_000, (8.0, 6.0, 3.0), 40, seed=3)
        cams = [Camera((1.0, 3.0, 1.6), (8.0, 3.0, 1.2), (0.0, 0.0, 1.0), 60.0, 1024, 768)]
        return sc, cams, dict(spp=64, max_depth=5, rr_start=3)
    if k == 4:
        sc = multiroom_scene(n_override or 5_000_000, seed=4)
        cams = [Camera((14.0, 3.0, 1.6), (2.0, 3.0, 1.0), (0.0, 0.0, 1.0), 60.0, 1920, 1080)]
        return sc, cams, dict(spp=256, max_depth=8, rr_start=3, pass_spp=16)
    if k == 5:
        sc = room_scene(n_override or 3_000_000, (8.0, 6.0, 3.0), 40, seed=5)
        return sc, [], dict(max_depth=5, rr_start=3)
    raise ValueError(f"unknown config {k}")


def arrivals(scene: Scene, n_requests: int, rate_hz: float, seed: int = 505, edit_frac: float = 0.05,
             resolutions=((256, 256), (512, 512), (1024, 768), (1920, 1080)), spps=(16, 64, 256),
             edit_sizes=(1_000, 50_000)):
    """Poisson request stream: list of dicts with arrival time t (s) and either
    kind='render' (camera, spp) or kind='edit' (op, surfel indices, value)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    cams = interior_cameras(scene, n_requests, 16, 16, seed=seed + 1)
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        if rng.uniform() < edit_frac:
            cnt = int(rng.integers(edit_sizes[0], edit_sizes[1] + 1))
            cnt = min(cnt, scene.n)
            idx = np.sort(rng.choice(scene.n, cnt, replace=False)).astype(np.int32)
            if rng.uniform() < 0.5:
                out.append(dict(t=t, kind="edit", op="scale_radiance", idx=idx,
                                value=(0.0, 0.0, 0.0) if rng.uniform() < 0.5 else (1.0, 1.0, 1.0)))
            else:
                out.append(dict(t=t, kind="edit", op="set_albedo", idx=idx,
                                value=tuple(map(float, rng.uniform(0.05, 0.9, 3)))))
        else:
            w, h = resolutions[int(rng.integers(len(resolutions)))]
            c = cams[i]
            out.append(dict(t=t, kind="render", camera=Camera(c.eye, c.look_at, c.up, c.vfov_deg, w, h),
                            spp=int(spps[int(rng.integers(len(spps)))])))
    return out
