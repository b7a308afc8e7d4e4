"""Shared test helpers: the comparison measure and scene upload."""
import numpy as np


def rel_err(a, b, mask=None):
    """|a - b| / max(|b|, 1e-2 * RMS(b over the compared set)), elementwise."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if mask is not None:
        a, b = a[mask], b[mask]
    if b.size == 0:
        return np.zeros(0)
    rms = np.sqrt(np.mean(b * b))
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-2 * rms + 1e-30)


def gpu_scene(scene):
    from paper_2601_23065_amd.api import Scene
    return Scene(scene.arrays() if hasattr(scene, "arrays") else scene)


def oracle_params(p):
    """oracle Params from the binding's Params."""
    from oracle import Params
    return Params(spp=p.spp, max_depth=p.max_depth, rr_start=p.rr_start, tau_E=p.tau_E, T_min=p.T_min,
                  t_min=p.t_min, k_sigma=p.k_sigma, depth_quantum=p.depth_quantum, seed=p.seed,
                  camera_id=p.camera_id, jitter=bool(p.flags & 1), additive=bool(p.flags & 2),
                  detach_bounce=bool(p.flags & 4))


def coplanar_stack(layers, seed):
    """`layers` surfels on z = 0 with centres within 0.02 of the origin,
    axis-aligned, scales 0.2, opacity 0.02 (T stays above T_min through 300
    of them), random albedo and radiance, all emissive."""
    import scenegen as sg
    rng = np.random.default_rng(seed)
    pos = np.zeros((3, layers))
    pos[:2] = rng.uniform(-0.02, 0.02, (2, layers))
    rot = np.zeros((4, layers))
    rot[0] = 1.0
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)   # noqa: E731
    return sg.Scene(f32(pos), f32(rot), f32(np.full((2, layers), 0.2)), f32(np.full(layers, 0.02)),
                    f32(rng.uniform(0.1, 0.8, (3, layers))), f32(rng.uniform(1.0, 10.0, (3, layers))),
                    f32(np.ones(layers)), bounds=(np.full(3, -1.0), np.full(3, 1.0)))
