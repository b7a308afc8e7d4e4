"""Parity of the single-bounce render (Eq. 5-7) and the path tracer (Eq. 9)
with the FP64 oracle, per pixel and per sample on unflagged entries, plus
the GPU-only invariants: split-pass invariance of the fixed-point
accumulators and a white furnace against its closed form."""
import numpy as np
import pytest
import torch

import scenegen as sg
from oracle.render import path_trace as o_path_trace
from oracle.render import single_bounce as o_single_bounce
from oracle.tracer import Scene64
from tests._util import coplanar_stack, gpu_scene, oracle_params, rel_err

pytestmark = pytest.mark.gpu


def test_single_bounce_config1_full_image():
    from paper_2601_23065_amd.api import BVH, Params, render_single_bounce
    scene, cams, cfg = sg.config(1)
    p = Params(spp=cfg["spp"])
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    rgb = render_single_bounce(bvh, gs, cams, p)[0].cpu().numpy().reshape(-1, 3)
    ref = o_single_bounce(Scene64(scene), cams[0], oracle_params(p))
    ok = ref["flags"] == 0
    err = rel_err(rgb, ref["L"], np.broadcast_to(ok[:, None], rgb.shape))
    print(f"pixels={ok.size} unflagged={ok.mean():.3f} max_err={err.max():.2e} branches={np.bincount(ref['branch'])}")
    assert ok.mean() >= 0.98
    assert err.max() <= 1e-4
    # miss pixels are exactly zero, emitter pixels carry R
    miss = ref["branch"] == 0
    assert np.all(rgb[miss] == 0)


def _small_room():
    scene = sg.room_scene(16000, (3.0, 2.5, 2.5), 3, seed=31, emissive_frac=0.02)
    cam = sg.Camera((0.4, 0.4, 1.0), (1.6, 1.3, 2.4), (0.0, 0.0, 1.0), 80.0, 20, 14)
    return scene, cam


@pytest.mark.parametrize("jitter", [False, True])
def test_single_bounce_room_per_sample(jitter):
    from paper_2601_23065_amd import JITTER
    from paper_2601_23065_amd.api import BVH, Params, render_single_bounce
    scene, cam = _small_room()
    p = Params(spp=3, camera_id=7, seed=123, flags=JITTER if jitter else 0)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    rgb, state = render_single_bounce(bvh, gs, [cam], p, keep_state=True)
    npix = cam.width * cam.height
    r1 = state[npix * 28:].view(torch.float64).view(npix, p.spp, 3).cpu().numpy()
    st = state[:npix * 28].view(npix, 28).cpu().numpy()
    ref = o_single_bounce(Scene64(scene), cam, oracle_params(p))
    ok = ref["flags"] == 0
    assert ok.mean() >= 0.98
    np.testing.assert_array_equal(st[:, 25].astype(int)[ok], ref["branch"][ok])
    e1 = rel_err(r1, ref["R1"], np.broadcast_to(ok[:, None, None], r1.shape))
    eL = rel_err(rgb[0].cpu().numpy().reshape(-1, 3), ref["L"], np.broadcast_to(ok[:, None], (npix, 3)))
    print(f"unflagged={ok.mean():.3f} R1 err={e1.max():.2e} L err={eL.max():.2e}")
    assert e1.max() <= 1e-4 and eL.max() <= 1e-4


def _pt_per_sample(bvh, gs, cam, p, samples):
    from paper_2601_23065_amd.api import path_trace
    out = []
    for s in samples:
        acc = path_trace(bvh, gs, cam, p, sample_begin=s, sample_count=1)
        out.append(acc.cpu().numpy().reshape(-1, 3).astype(np.float64) / 2.0 ** 32)
    return np.stack(out, axis=1)          # [pix, S, 3]


def test_path_trace_room_per_sample():
    from paper_2601_23065_amd.api import BVH, Params
    scene, cam = _small_room()
    p = Params(spp=4, max_depth=5, rr_start=3, camera_id=3, seed=99)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    got = _pt_per_sample(bvh, gs, cam, p, range(p.spp))
    ref = o_path_trace(Scene64(scene), cam, oracle_params(p))
    ok = ref["flags"] == 0
    err = rel_err(got, ref["value"], np.broadcast_to(ok[..., None], got.shape))
    print(f"paths={ok.size} unflagged={ok.mean():.3f} err={err.max():.2e} nonzero={np.mean(ref['value'].sum(-1) > 0):.3f}")
    assert ok.mean() >= 0.98
    assert err.max() <= 1e-4


def _cloud():
    return (sg.cloud_scene(2000, seed=1, emissive_frac=0.3),
            sg.Camera((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0, 24, 18))


@pytest.mark.parametrize("case", ["exact_t_order", "k2_Tmin1e-3_tmin1e-2"])
def test_path_trace_other_readings_per_sample(case):
    """The readings exposed as parameters: exact (t, index) order instead of
    the depth quantum (on the cloud: coplanar walls would leave every order
    to rounding); a 2-sigma extent with other stopping and minimum-hit
    distances (on the room). Every path against the oracle with the same
    parameters."""
    from paper_2601_23065_amd.api import BVH, Params
    if case == "exact_t_order":
        scene, cam = _cloud()
        kw = dict(depth_quantum=0.0)
    else:
        scene, cam = _small_room()
        kw = dict(k_sigma=2.0, T_min=1e-3, t_min=1e-2)
    p = Params(spp=2, max_depth=4, rr_start=2, seed=17, **kw)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    got = _pt_per_sample(bvh, gs, cam, p, range(p.spp))
    ref = o_path_trace(Scene64(scene), cam, oracle_params(p))
    ok = ref["flags"] == 0
    err = rel_err(got, ref["value"], np.broadcast_to(ok[..., None], got.shape))
    print(f"{case}: paths={ok.size} unflagged={ok.mean():.3f} err={err.max():.2e} "
          f"nonzero={np.mean(ref['value'].sum(-1) > 0):.3f}")
    assert ok.mean() >= 0.98 and err.max() <= 1e-4
    assert np.mean(ref["value"].sum(-1) > 0) > 0.05


def test_path_trace_jittered_camera_rays_per_sample():
    """EAG_JITTER: camera rays jittered inside the pixel by Philox segment
    word 0xffffffff; every path against the oracle."""
    from paper_2601_23065_amd import JITTER
    from paper_2601_23065_amd.api import BVH, Params
    scene, cam = _small_room()
    p = Params(spp=3, max_depth=4, rr_start=2, camera_id=1, seed=7, flags=JITTER)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    got = _pt_per_sample(bvh, gs, cam, p, range(p.spp))
    prm = oracle_params(p)
    assert prm.jitter
    ref = o_path_trace(Scene64(scene), cam, prm)
    ok = ref["flags"] == 0
    err = rel_err(got, ref["value"], np.broadcast_to(ok[..., None], got.shape))
    print(f"paths={ok.size} unflagged={ok.mean():.3f} err={err.max():.2e}")
    assert ok.mean() >= 0.98 and err.max() <= 1e-4
    # the jitter moves the camera rays: sample 0 differs from the pixel-centre render
    centre = _pt_per_sample(bvh, gs, cam, Params(spp=1, max_depth=4, rr_start=2, camera_id=1, seed=7), [0])
    assert not np.array_equal(centre[:, 0], got[:, 0])


def test_progressive_passes_are_exact():
    from paper_2601_23065_amd.api import BVH, Params, path_trace
    scene, cam = _small_room()
    p = Params(spp=8, max_depth=4, rr_start=2)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    one = path_trace(bvh, gs, cam, p, 0, 8)
    acc = None
    for s0 in (0, 2, 3, 7):
        acc = path_trace(bvh, gs, cam, p, s0, {0: 2, 2: 1, 3: 4, 7: 1}[s0], accum=acc)
    assert torch.equal(one, acc)
    again = path_trace(bvh, gs, cam, p, 0, 8)
    assert torch.equal(one, again)


def test_white_furnace_gpu():
    from paper_2601_23065_amd import ADDITIVE_EMISSION
    from paper_2601_23065_amd.api import BVH, Params, path_trace, resolve
    E, rho, D = 1.0, 0.5, 6
    scene = sg.furnace_scene(n_layers=12, radiance=E, albedo=rho)
    cam = sg.Camera((0.1, -0.2, 0.05), (1.0, 0.3, 0.2), (0.0, 0.0, 1.0), 90.0, 32, 32)
    p = Params(spp=4, max_depth=D, rr_start=0, flags=ADDITIVE_EMISSION, t_min=1e-4)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    img = resolve(path_trace(bvh, gs, cam, p), p.spp).cpu().numpy()
    rho32 = float(np.float32(rho))
    closed = E * (1 - rho32 ** (D + 1)) / (1 - rho32)
    err = np.abs(img - closed) / closed
    print(f"furnace max rel err {err.max():.2e}")
    assert err.max() <= 1e-4 * (D + 1)


@pytest.mark.parametrize("layers", [100, 300])
def test_path_trace_deep_coplanar_stack(layers):
    """Coplanar surfels stacked on z = 0, deeper than the k-buffer: with 100
    the later rounds come from the per-lane hit list, with 300 one depth
    bucket holds more keys than the list, which overflows, and the rounds fall
    back to traversal. Opacity 0.02 keeps T above T_min through the whole
    stack, and random radiance makes the pixel depend on the blending order
    (the surfel index within the bucket)."""
    from paper_2601_23065_amd.api import BVH, Params
    scene = coplanar_stack(layers, 61 + layers)
    cam = sg.Camera((0.0, 0.0, -2.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 5.0, 8, 8)
    p = Params(spp=2, max_depth=0, rr_start=0, seed=3)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    got = _pt_per_sample(bvh, gs, cam, p, range(p.spp))
    ref = o_path_trace(Scene64(scene), cam, oracle_params(p))
    ok = ref["flags"] == 0
    err = rel_err(got, ref["value"], np.broadcast_to(ok[..., None], got.shape))
    print(f"layers={layers} paths={ok.size} unflagged={ok.mean():.3f} err={err.max():.2e} "
          f"mean={ref['value'].mean():.3f}")
    assert ok.mean() >= 0.98
    assert err.max() <= 1e-4
    # every camera ray blends the whole stack, 16 keys per k-buffer round
    from paper_2601_23065_amd.api import path_trace
    c = torch.zeros(6, dtype=torch.int64, device="cuda")
    path_trace(bvh, gs, cam, p, counters=c)
    seg, _, rounds, _, hits, _ = c.tolist()
    assert seg == ok.size
    assert hits == seg * layers
    assert rounds >= seg * -(-layers // 16)


def test_side_stream_equals_current_stream():
    """Every call given a stream other than torch's current one: the BVH
    built, the accumulator created and cleared, and the paths traced on a
    side stream, and a single-bounce render there, equal the same calls on
    the current stream bit for bit."""
    from paper_2601_23065_amd.api import BVH, Params, path_trace, render_single_bounce
    scene, cam = _small_room()
    p = Params(spp=4, max_depth=4, rr_start=2, seed=12)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    ref_pt = path_trace(bvh, gs, cam, p)
    ref_sb = render_single_bounce(bvh, gs, [cam], p)
    side = torch.cuda.Stream()
    bvh_side = BVH(gs, stream=side)
    pt = path_trace(bvh_side, gs, cam, p, stream=side)
    sb = render_single_bounce(bvh_side, gs, [cam], p, stream=side)
    side.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(pt, ref_pt) and int(pt.abs().sum()) > 0
    assert torch.equal(sb, ref_sb)
