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
