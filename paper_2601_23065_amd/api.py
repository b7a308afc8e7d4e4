"""Python binding of the surfel tracing library: torch tensors for device
memory and streams, the C ABI for every computation.

All tensors passed in are float32 CUDA (HIP) tensors in the component-major
layouts of include/eag.h. Nothing here computes on the scene: a missing or
failing library raises.
"""
from __future__ import annotations

import ctypes as C
import functools
import inspect
from dataclasses import dataclass, fields

import torch

from . import _lib as L

_GEOM = ("pos", "rot", "scale", "opacity")
_ATTR = ("albedo", "radiance", "emissive")
_SHAPES = {"pos": 3, "rot": 4, "scale": 2, "opacity": 0, "albedo": 3, "radiance": 3, "emissive": 0}


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _streamed(fn):
    """Run a binding function on its `stream` argument when one is given.

    The library launches on that stream, so the work torch has queued on its
    current stream (the caller's inputs, and the zero fills of tensors made
    here) must come first: the stream waits for the current one. The body
    then runs with the stream current, so workspaces, accumulators and
    temporaries made here are allocated and cleared on it, and the caching
    allocator does not hand their memory to other streams while the
    library's kernels may still use it. Without a stream, everything runs on
    torch's current stream."""
    sig = inspect.signature(fn)

    @functools.wraps(fn)
    def run(*args, **kwargs):
        stream = sig.bind_partial(*args, **kwargs).arguments.get("stream")
        if stream is None:
            return fn(*args, **kwargs)
        stream.wait_stream(torch.cuda.current_stream(stream.device))
        with torch.cuda.stream(stream):
            return fn(*args, **kwargs)
    return run


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _bytes(nbytes, device):
    return torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)


def _aligned(buf):
    """256-byte aligned view start of a uint8 buffer."""
    p = buf.data_ptr()
    off = (-p) % 256
    return C.c_void_p(p + off), buf.numel() - off


@dataclass
class Params:
    """Mirror of eag_trace_params (defaults = eag_default_params)."""
    spp: int = 4
    max_depth: int = 5
    rr_start: int = 3
    tau_E: float = 0.1
    T_min: float = 1e-4
    t_min: float = 1e-3
    k_sigma: float = 3.0
    depth_quantum: float = 2.0 ** -13
    kbuf: int = 16
    camera_id: int = 0
    seed: int = 0
    flags: int = 0

    def c(self):
        p = L.TraceParams()
        for f in fields(self):
            setattr(p, f.name, getattr(self, f.name))
        return p


def camera_struct(cam):
    """cam: object with eye, look_at, up, vfov_deg, width, height."""
    c = L.Camera()
    c.eye[:] = [float(v) for v in cam.eye]
    c.look_at[:] = [float(v) for v in cam.look_at]
    c.up[:] = [float(v) for v in cam.up]
    c.vfov_deg = float(cam.vfov_deg)
    c.width = int(cam.width)
    c.height = int(cam.height)
    return c


class Scene:
    """Device-resident surfel arrays (float32, component-major)."""

    def __init__(self, arrays: dict, device="cuda"):
        self.t = {}
        n = None
        for k in _GEOM + _ATTR:
            v = torch.as_tensor(arrays[k], dtype=torch.float32).to(device).contiguous()
            if _SHAPES[k]:
                assert v.dim() == 2 and v.shape[0] == _SHAPES[k], (k, tuple(v.shape))
                m = v.shape[1]
            else:
                assert v.dim() == 1, k
                m = v.shape[0]
            n = m if n is None else n
            assert m == n, f"{k} has {m} surfels, expected {n}"
            self.t[k] = v
        self.n = n
        self.device = torch.device(device)

    def __getattr__(self, k):
        t = self.__dict__.get("t", {})
        if k in t:
            return t[k]
        raise AttributeError(k)

    def c(self, overrides: dict | None = None):
        s = L.Surfels()
        s.n = self.n
        for k in _GEOM + _ATTR:
            setattr(s, k, _ptr((overrides or {}).get(k, self.t[k])))
        return s

    def attrs_c(self):
        a = L.SurfelAttrs()
        a.n = self.n
        a.albedo, a.radiance, a.emissive = _ptr(self.t["albedo"]), _ptr(self.t["radiance"]), _ptr(self.t["emissive"])
        return a


class BVH:
    """Linear BVH over a Scene; owns its device memory as a torch tensor."""

    @_streamed
    def __init__(self, scene: Scene, stream=None):
        lib = L.load()
        self.scene = scene
        n = scene.n
        self.mem = _bytes(lib.eag_bvh_bytes(n), scene.device)
        ws = _bytes(lib.eag_build_workspace_bytes(n), scene.device)
        h = C.c_void_p()
        mp, mb = _aligned(self.mem)
        wp, wb = _aligned(ws)
        sc = scene.c()
        L.check(lib.eag_build_bvh(C.byref(sc), mp, mb, wp, wb, _stream(stream), C.byref(h)))
        self.h = h
        self._ws = ws
        self.cost_at_build = self.sah_cost(stream)   # for the refit-or-rebuild policy (update_bvh)

    @_streamed
    def refit(self, scene: Scene | None = None, stream=None):
        lib = L.load()
        scene = scene or self.scene
        wp, wb = _aligned(self._ws)
        sc = scene.c()
        L.check(lib.eag_refit_bvh(self.h, C.byref(sc), wp, wb, _stream(stream)))

    @_streamed
    def sah_cost(self, stream=None):
        """The tree's surface-area cost (a device float64 scalar)."""
        cost = torch.empty((), dtype=torch.float64, device=self.scene.device)
        wp, wb = _aligned(self._ws)
        L.check(L.load().eag_bvh_sah_cost(self.h, _ptr(cost), wp, wb, _stream(stream)))
        return cost

    def info(self):
        i = L.BvhInfo()
        L.check(L.load().eag_bvh_get_info(self.h, C.byref(i)))
        return i

    def __del__(self):
        try:
            if getattr(self, "h", None):
                L.load().eag_bvh_destroy(self.h)
                self.h = None
        except Exception:
            pass


@_streamed
def trace_rays(bvh: BVH, scene: Scene, params: Params, origins, dirs, max_hits: int = 0, stream=None,
               stats=None):
    """origins, dirs: [3, M] float32 device tensors. Returns out [12, M]
    (Nt, Dt, R, E, P, A) and, if max_hits > 0, (hit_idx [M, max_hits],
    hit_count [M]). stats: optional int32 [M, 3] device tensor receiving
    (k-buffer rounds, candidate tests, nodes visited) per ray."""
    lib = L.load()
    m = origins.shape[1]
    dev = scene.device
    out = torch.empty((12, m), dtype=torch.float32, device=dev)
    hits = torch.full((m, max(max_hits, 1)), -1, dtype=torch.int32, device=dev) if max_hits > 0 else None
    cnt = torch.zeros(m, dtype=torch.int32, device=dev) if max_hits > 0 else None
    ws = _bytes(lib.eag_trace_workspace_bytes(scene.n), dev)
    wp, wb = _aligned(ws)
    p = params.c()
    sc = scene.c()
    origins = origins.to(torch.float64).contiguous()
    dirs = dirs.to(torch.float64).contiguous()
    L.check(lib.eag_trace_rays(bvh.h, C.byref(sc), C.byref(p), m, _ptr(origins),
                               _ptr(dirs), _ptr(out), _ptr(hits), _ptr(cnt), max_hits, _ptr(stats),
                               wp, wb, _stream(stream)))
    return (out, hits, cnt) if max_hits > 0 else out


def init():
    """eag_init on the current device: set-up for trace_rays_noalloc."""
    L.check(L.load().eag_init())


def trace_rays_noalloc(bvh: BVH, scene: Scene, params: Params, origins, dirs, out, hits=None, counts=None,
                       stats=None, stream=None):
    """eag_trace_rays_noalloc: as trace_rays, with every buffer the caller's
    (origins, dirs: contiguous float64 [3, M]; out: float32 [12, M]; hits:
    optional int32 [M, max_hits]; counts: int32 [M]; stats: int32 [M, 3])
    and nothing allocated, here or in the library (after init() on this
    device). At most 2^18 surfels."""
    p = params.c()
    sc = scene.c()
    max_hits = hits.shape[1] if hits is not None else 0
    s = stream if stream is not None else torch.cuda.current_stream()
    L.check(L.load().eag_trace_rays_noalloc(bvh.h, C.byref(sc), C.byref(p), origins.shape[1], _ptr(origins),
                                            _ptr(dirs), _ptr(out), _ptr(hits), _ptr(counts), max_hits, _ptr(stats),
                                            C.c_void_p(s.cuda_stream)))
    return out


def _cams(cams):
    arr = (L.Camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = camera_struct(c)
    return arr


@_streamed
def render_single_bounce(bvh: BVH, scene: Scene, cams, params: Params, keep_state: bool = False, stream=None,
                         overrides=None):
    """Returns rgb [n_cams, H, W, 3] and, if keep_state, the forward state."""
    lib = L.load()
    ca = _cams(cams)
    p = params.c()
    H, W = cams[0].height, cams[0].width
    dev = scene.device
    rgb = torch.empty((len(cams), H, W, 3), dtype=torch.float32, device=dev)
    state = None
    if keep_state:
        state = torch.empty(lib.eag_fwd_state_floats(ca, len(cams), C.byref(p)), dtype=torch.float32, device=dev)
    ws = _bytes(lib.eag_render_workspace_bytes(scene.n, ca, len(cams), C.byref(p)), dev)
    wp, wb = _aligned(ws)
    sc = scene.c(overrides)
    L.check(lib.eag_render_single_bounce(bvh.h, C.byref(sc), ca, len(cams), C.byref(p), _ptr(rgb), _ptr(state),
                                         wp, wb, _stream(stream)))
    return (rgb, state) if keep_state else rgb


@_streamed
def single_bounce_backward(bvh: BVH, scene: Scene, cams, params: Params, dL_drgb, state, grads: dict | None = None,
                           stream=None, overrides=None):
    """Accumulates gradients into `grads` (zeroed tensors are created if
    None) and returns them."""
    lib = L.load()
    ca = _cams(cams)
    p = params.c()
    dev = scene.device
    if grads is None:
        grads = {k: torch.zeros_like(scene.t[k]) for k in ("pos", "rot", "scale", "opacity", "albedo", "radiance")}
    g = L.SurfelGrads()
    for k in ("pos", "rot", "scale", "opacity", "albedo", "radiance"):
        setattr(g, k, _ptr(grads[k]))
    ws = _bytes(lib.eag_backward_workspace_bytes(scene.n, ca, len(cams), C.byref(p)), dev)
    wp, wb = _aligned(ws)
    sc = scene.c(overrides)
    L.check(lib.eag_single_bounce_backward(bvh.h, C.byref(sc), ca, len(cams), C.byref(p),
                                           _ptr(dL_drgb.contiguous()), _ptr(state), C.byref(g), wp, wb,
                                           _stream(stream)))
    return grads


class SingleBounceRender(torch.autograd.Function):
    """Differentiable single-bounce render: forward and backward both run in
    the HIP library; the BVH must match the geometry passed in (build or
    refit it outside)."""

    @staticmethod
    def forward(ctx, pos, rot, scale, opacity, albedo, radiance, emissive, bvh, scene, cams, params):
        ov = dict(pos=pos.detach(), rot=rot.detach(), scale=scale.detach(), opacity=opacity.detach(),
                  albedo=albedo.detach(), radiance=radiance.detach(), emissive=emissive.detach())
        rgb, state = render_single_bounce(bvh, scene, cams, params, keep_state=True, overrides=ov)
        ctx.save_for_backward(state)
        ctx.extra = (bvh, scene, cams, params, ov)
        return rgb

    @staticmethod
    def backward(ctx, d_rgb):
        (state,) = ctx.saved_tensors
        bvh, scene, cams, params, ov = ctx.extra
        grads = {k: torch.zeros_like(ov[k]) for k in ("pos", "rot", "scale", "opacity", "albedo", "radiance")}
        single_bounce_backward(bvh, scene, cams, params, d_rgb, state, grads, overrides=ov)
        return (grads["pos"], grads["rot"], grads["scale"], grads["opacity"], grads["albedo"], grads["radiance"],
                None, None, None, None, None)


@_streamed
def path_trace(bvh: BVH, scene: Scene, cam, params: Params, sample_begin: int = 0, sample_count: int | None = None,
               accum=None, counters=None, stream=None, ws=None):
    """Adds samples [sample_begin, sample_begin + sample_count) into the int64
    fixed-point accumulator [H, W, 3] (created if None) and returns it."""
    lib = L.load()
    dev = scene.device
    sample_count = params.spp if sample_count is None else sample_count
    if accum is None:
        accum = torch.zeros((cam.height, cam.width, 3), dtype=torch.int64, device=dev)
    if ws is None:
        ws = _bytes(lib.eag_path_trace_workspace_bytes(scene.n), dev)
    wp, wb = _aligned(ws)
    c = camera_struct(cam)
    p = params.c()
    sc = scene.c()
    L.check(lib.eag_path_trace(bvh.h, C.byref(sc), C.byref(c), C.byref(p), sample_begin, sample_count, _ptr(accum),
                               _ptr(counters), wp, wb, _stream(stream)))
    return accum


class Emitters:
    """Emitter table of a Scene for emitter sampling with multiple importance
    sampling (built for params.tau_E and params.k_sigma); owns its device
    memory. Rebuild it after editing the scene. cell: 0 selects emitters by
    power, a power of two selects by cells of that size weighted by their
    power over the squared distance to the vertex."""

    @_streamed
    def __init__(self, scene: Scene, params: Params, cell: float = 0.0, stream=None):
        lib = L.load()
        self.scene = scene
        n = scene.n
        self.mem = _bytes(lib.eag_emitters_bytes(n), scene.device)
        ws = _bytes(lib.eag_emitters_workspace_bytes(n), scene.device)
        h = C.c_void_p()
        mp, mb = _aligned(self.mem)
        wp, wb = _aligned(ws)
        sc = scene.c()
        p = params.c()
        L.check(lib.eag_build_emitters(C.byref(sc), C.byref(p), float(cell), mp, mb, wp, wb, _stream(stream),
                                       C.byref(h)))
        self.h = h

    def info(self):
        """(number of emitters, total selection weight W)."""
        n = C.c_int64()
        w = C.c_double()
        L.check(L.load().eag_emitters_get_info(self.h, C.byref(n), C.byref(w), None))
        return int(n.value), float(w.value)

    def cells(self):
        """Cells of the selection by cells (0 for selection by power)."""
        c = C.c_int32()
        L.check(L.load().eag_emitters_get_info(self.h, None, None, C.byref(c)))
        return int(c.value)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                L.load().eag_emitters_destroy(self.h)
                self.h = None
        except Exception:
            pass


@_streamed
def path_trace_mis(bvh: BVH, scene: Scene, emitters: Emitters, cam, params: Params, sample_begin: int = 0,
                   sample_count: int | None = None, accum=None, counters=None, stream=None, ws=None):
    """path_trace with emitter sampling combined by multiple importance
    sampling; same accumulator and sample ranges (ws: path_trace_mis_workspace)."""
    lib = L.load()
    dev = scene.device
    sample_count = params.spp if sample_count is None else sample_count
    if accum is None:
        accum = torch.zeros((cam.height, cam.width, 3), dtype=torch.int64, device=dev)
    c = camera_struct(cam)
    p = params.c()
    if ws is None:
        ws = _bytes(lib.eag_path_trace_mis_workspace_bytes(scene.n, C.byref(c), C.byref(p)), dev)
    wp, wb = _aligned(ws)
    sc = scene.c()
    L.check(lib.eag_path_trace_mis(bvh.h, C.byref(sc), emitters.h, C.byref(c), C.byref(p), sample_begin,
                                   sample_count, _ptr(accum), _ptr(counters), wp, wb, _stream(stream)))
    return accum


def path_trace_mis_workspace(scene: Scene, cam, params: Params):
    c = camera_struct(cam)
    p = params.c()
    return _bytes(L.load().eag_path_trace_mis_workspace_bytes(scene.n, C.byref(c), C.byref(p)), scene.device)


def path_trace_workspace(scene: Scene):
    return _bytes(L.load().eag_path_trace_workspace_bytes(scene.n), scene.device)


@_streamed
def resolve(accum, total_spp: int, stream=None):
    """float32 image [H, W, 3] = accum / (2^32 * total_spp)."""
    rgb = torch.empty(accum.shape, dtype=torch.float32, device=accum.device)
    L.check(L.load().eag_accum_resolve(_ptr(accum), accum.numel() // 3, int(total_spp), _ptr(rgb), _stream(stream)))
    return rgb


@_streamed
def apply_edit(scene: Scene, kind: int, idx, value, stream=None):
    """In-place attribute edit of the scene's arrays; idx: int32 device tensor."""
    e = L.Edit()
    e.kind = int(kind)
    idx = idx.to(torch.int32).contiguous()
    e.idx = _ptr(idx)
    e.count = idx.numel()
    vals = [float(v) for v in value]
    e.value[:] = vals + [0.0] * (12 - len(vals))
    a = scene.attrs_c()
    L.check(L.load().eag_apply_edit(C.byref(e), C.byref(a), _stream(stream)))


def _f3(v, k=3):
    return (C.c_float * k)(*[float(x) for x in v])


def _out(scene: Scene):
    o = L.SurfelsOut()
    o.n = scene.n
    for k in _GEOM + _ATTR:
        setattr(o, k, _ptr(scene.t[k]))
    return o


@_streamed
def select_box(scene: Scene, lo, hi, stream=None):
    """int32 device tensor of the surfels whose centre lies in [lo, hi]
    (reads the count back: a synchronisation)."""
    lib = L.load()
    idx = torch.empty(scene.n, dtype=torch.int32, device=scene.device)
    count = torch.zeros((), dtype=torch.int64, device=scene.device)
    ws = _bytes(lib.eag_select_workspace_bytes(scene.n), scene.device)
    wp, wb = _aligned(ws)
    sc = scene.c()
    L.check(lib.eag_select_box(C.byref(sc), _f3(lo), _f3(hi), _ptr(idx), _ptr(count), wp, wb, _stream(stream)))
    return idx[:int(count)]


@_streamed
def move_surfels(scene: Scene, idx, r=(1.0, 0.0, 0.0, 0.0), pivot=(0.0, 0.0, 0.0), t=(0.0, 0.0, 0.0), stream=None):
    """In place: p -> R(r)(p - pivot) + pivot + t, q -> r (x) q for the surfels idx."""
    idx = idx.to(torch.int32).contiguous()
    o = _out(scene)
    L.check(L.load().eag_move_surfels(C.byref(o), _ptr(idx), idx.numel(), _f3(r, 4), _f3(pivot), _f3(t),
                                      _stream(stream)))


@_streamed
def delete_surfels(scene: Scene, idx, stream=None):
    """In place: opacity 0 for the surfels idx."""
    idx = idx.to(torch.int32).contiguous()
    o = _out(scene)
    L.check(L.load().eag_delete_surfels(C.byref(o), _ptr(idx), idx.numel(), _stream(stream)))


@_streamed
def duplicate_surfels(scene: Scene, idx, r=(1.0, 0.0, 0.0, 0.0), pivot=(0.0, 0.0, 0.0), t=(0.0, 0.0, 0.0),
                      stream=None):
    """A new Scene: the surfels of `scene`, then moved copies of the surfels idx."""
    idx = idx.to(torch.int32).contiguous()
    m = scene.n + idx.numel()
    arrays = {k: torch.empty(((_SHAPES[k],) if _SHAPES[k] else ()) + (m,), dtype=torch.float32, device=scene.device)
              for k in _GEOM + _ATTR}
    dst = Scene(arrays, device=scene.device)
    o = _out(dst)
    sc = scene.c()
    L.check(L.load().eag_duplicate_surfels(C.byref(sc), _ptr(idx), idx.numel(), C.byref(o), _f3(r, 4), _f3(pivot),
                                           _f3(t), _stream(stream)))
    return dst


@_streamed
def update_bvh(bvh: BVH, scene: Scene, max_cost_ratio: float = 1.25, stream=None):
    """Refit-or-rebuild policy after geometric edits: a changed surfel count
    needs a build; otherwise the tree is refitted, and rebuilt when its
    surface-area cost has grown past max_cost_ratio times the cost of its
    last build. Returns (bvh, rebuilt)."""
    if scene.n != bvh.scene.n:
        return BVH(scene, stream), True
    bvh.refit(scene, stream)
    ratio = float(bvh.sah_cost(stream)) / float(bvh.cost_at_build)
    if ratio > max_cost_ratio:
        return BVH(scene, stream), True
    return bvh, False


@_streamed
def render_stage0(bvh: BVH, scene: Scene, cams, params: Params, ws=None, stream=None):
    """Stage-0 images [n_cams, H, W, 8] (Nt, Dt, R, E) and the forward state
    the backward needs."""
    lib = L.load()
    ca = _cams(cams)
    H, W = cams[0].height, cams[0].width
    images = torch.empty((len(cams), H, W, L.STAGE0_FLOATS), dtype=torch.float32, device=scene.device)
    state = torch.empty(len(cams) * H * W * L.FWD_PIXEL_FLOATS, dtype=torch.float32, device=scene.device)
    ws = _bytes(lib.eag_stage0_workspace_bytes(scene.n, ca, len(cams)), scene.device) if ws is None else ws
    wp, wb = _aligned(ws)
    sc = scene.c()
    L.check(lib.eag_render_stage0(bvh.h, C.byref(sc), ca, len(cams), C.byref(params.c()), _ptr(images), _ptr(state),
                                  wp, wb, _stream(stream)))
    return images, state


@_streamed
def stage0_loss(images, rgb_gt, normal_mono, mask, cams, params: Params, weights=(1.0, 1.0, 1.0, 1.0), stream=None):
    """(loss as a device float64 scalar, d loss / d images) of Eq. 4."""
    lib = L.load()
    ca = _cams(cams)
    ws = _bytes(lib.eag_stage0_loss_workspace_bytes(ca, len(cams)), images.device)
    wp, wb = _aligned(ws)
    d = torch.empty_like(images)
    loss = torch.empty((), dtype=torch.float64, device=images.device)
    w = (C.c_float * 4)(*[float(x) for x in weights])
    L.check(lib.eag_stage0_loss(_ptr(images.contiguous()), _ptr(rgb_gt.contiguous()), _ptr(normal_mono.contiguous()),
                                _ptr(mask.contiguous()), ca, len(cams), C.byref(params.c()), w, _ptr(d), _ptr(loss),
                                wp, wb, _stream(stream)))
    return loss, d


@_streamed
def stage0_backward(bvh: BVH, scene: Scene, cams, params: Params, d_images, state, grads: dict | None = None, ws=None,
                    stream=None):
    """Accumulates d<d_images, images>/d(pos, rot, scale, opacity, radiance,
    emissive) into `grads` (zeroed tensors are created if None)."""
    lib = L.load()
    ca = _cams(cams)
    if grads is None:
        grads = {k: torch.zeros_like(scene.t[k]) for k in ("pos", "rot", "scale", "opacity", "radiance", "emissive")}
    g = L.SurfelGrads()
    for k in ("pos", "rot", "scale", "opacity", "radiance"):
        setattr(g, k, _ptr(grads[k]))
    g.albedo = C.c_void_p(0)
    ws = _bytes(lib.eag_stage0_workspace_bytes(scene.n, ca, len(cams)), scene.device) if ws is None else ws
    wp, wb = _aligned(ws)
    sc = scene.c()
    L.check(lib.eag_stage0_backward(bvh.h, C.byref(sc), ca, len(cams), C.byref(params.c()),
                                    _ptr(d_images.contiguous()), _ptr(state), C.byref(g), _ptr(grads["emissive"]), wp,
                                    wb, _stream(stream)))
    return grads


def bake_workspace(scene: Scene, cams):
    return _bytes(L.load().eag_bake_workspace_bytes(scene.n, _cams(cams), len(cams)), scene.device)


@_streamed
def render_zero_bounce(bvh: BVH, scene: Scene, cams, params: Params, ws=None, stream=None):
    """0-bounce images [n_cams, H, W, 3]: R composited along each camera ray."""
    lib = L.load()
    ca = _cams(cams)
    rgb = torch.empty((len(cams), cams[0].height, cams[0].width, 3), dtype=torch.float32, device=scene.device)
    ws = bake_workspace(scene, cams) if ws is None else ws
    wp, wb = _aligned(ws)
    sc = scene.c()
    L.check(lib.eag_render_zero_bounce(bvh.h, C.byref(sc), ca, len(cams), C.byref(params.c()), _ptr(rgb), wp, wb,
                                       _stream(stream)))
    return rgb


@_streamed
def zero_bounce_backward(bvh: BVH, scene: Scene, cams, params: Params, dL_drgb, grad_radiance=None, ws=None,
                         stream=None):
    """grad_radiance [3, n] += d<dL_drgb, 0-bounce image>/d radiance."""
    lib = L.load()
    ca = _cams(cams)
    if grad_radiance is None:
        grad_radiance = torch.zeros_like(scene.t["radiance"])
    ws = bake_workspace(scene, cams) if ws is None else ws
    wp, wb = _aligned(ws)
    sc = scene.c()
    L.check(lib.eag_zero_bounce_backward(bvh.h, C.byref(sc), ca, len(cams), C.byref(params.c()),
                                         _ptr(dL_drgb.contiguous()), _ptr(grad_radiance), wp, wb, _stream(stream)))
    return grad_radiance


@_streamed
def bake_loss(rgb, target, stream=None):
    """(loss as a device float64 scalar, dloss/drgb) of mean |PQ(rgb) - PQ(target)|."""
    rgb, target = rgb.contiguous(), target.contiguous()
    dL = torch.empty_like(rgb)
    loss = torch.empty((), dtype=torch.float64, device=rgb.device)
    L.check(L.load().eag_bake_loss(_ptr(rgb), _ptr(target), rgb.numel(), _ptr(dL), _ptr(loss), _stream(stream)))
    return loss, dL


@dataclass
class Adam:
    """Mirror of eag_adam."""
    lr: float = 0.01
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15

    def c(self):
        a = L.Adam()
        a.lr, a.beta1, a.beta2, a.eps = self.lr, self.beta1, self.beta2, self.eps
        return a


@_streamed
def adam_step(param, grad, m, v, adam: Adam, step: int, stream=None):
    """In-place projected Adam update of param (m, v: moment tensors)."""
    L.check(L.load().eag_adam_step(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(), C.byref(adam.c()),
                                   int(step), _stream(stream)))


class Baker:
    """Light baking (Eq. 10) of the scene's radiance into its 0-bounce image
    against target images [n_cams, H, W, 3]; step() runs one iteration
    (render, loss, radiance gradient, Adam update of scene.radiance in place)
    and returns the loss before the update as a device float64 scalar."""

    def __init__(self, bvh: BVH, scene: Scene, cams, params: Params, targets, adam: Adam | None = None):
        self.bvh, self.scene, self.cams, self.params = bvh, scene, list(cams), params
        self.targets = targets.contiguous()
        self.adam = adam or Adam()
        self.m = torch.zeros_like(scene.t["radiance"])
        self.v = torch.zeros_like(scene.t["radiance"])
        self.ws = bake_workspace(scene, self.cams)
        self.loss = torch.zeros((), dtype=torch.float64, device=scene.device)
        self.steps = 0

    @_streamed
    def step(self, stream=None):
        lib = L.load()
        self.steps += 1
        wp, wb = _aligned(self.ws)
        sc = self.scene.c()
        L.check(lib.eag_bake_step(self.bvh.h, C.byref(sc), _cams(self.cams), len(self.cams), C.byref(self.params.c()),
                                  _ptr(self.targets), _ptr(self.scene.t["radiance"]), _ptr(self.m), _ptr(self.v),
                                  C.byref(self.adam.c()), self.steps, _ptr(self.loss), wp, wb, _stream(stream)))
        return self.loss


class Server:
    """Continuous-batching render server over a resident scene (eag_serve_*).

    arena_bytes: device memory for the scene copy, BVH, attribute versions
    and the request pool (per request: H*W*24 bytes of fixed-point
    accumulator). The arena is one torch tensor owned by this object."""

    def __init__(self, scene: Scene, arena_bytes: int, max_live_requests: int = 8,
                 paths_per_launch: int = 1 << 22, stream=None):
        lib = L.load()
        need = lib.eag_serve_arena_bytes(scene.n, 3, 0)
        self.arena = _bytes(max(int(arena_bytes), need), scene.device)
        ap, ab = _aligned(self.arena)
        cfg = L.ServerConfig()
        cfg.arena, cfg.arena_bytes = ap, ab
        cfg.max_live_requests = int(max_live_requests)
        cfg.paths_per_launch = int(paths_per_launch)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=scene.device)
        cfg.stream = C.c_void_p(self.stream.cuda_stream)
        sc = scene.c()
        h = C.c_void_p()
        L.check(lib.eag_serve_create(C.byref(sc), C.byref(cfg), C.byref(h)))
        self.h = h
        self.device = scene.device
        self._keep = {}

    def submit(self, cam, params: Params, out=None):
        """Queue a path-tracing request; returns (ticket, output tensor)."""
        if out is None:
            out = torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device=self.device)
        r = L.Request()
        r.cam = camera_struct(cam)
        r.params = params.c()
        r.out_rgb = _ptr(out)
        t = C.c_uint64()
        L.check(L.load().eag_serve_submit(self.h, C.byref(r), C.byref(t)))
        self._keep[t.value] = out
        return t.value, out

    def edit(self, kind: int, idx, value):
        """Queue an attribute edit, or EDIT_TRANSFORM with value = r (4),
        pivot (3), t (3); idx: surfel indices (any int sequence or tensor),
        held on the device until the edit is done. Returns its ticket."""
        idx = torch.as_tensor(idx, dtype=torch.int32).to(self.device).contiguous()
        # the server reads idx on its stream: the upload must come first
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        idx.record_stream(self.stream)
        e = L.Edit()
        e.kind = int(kind)
        e.idx = _ptr(idx)
        e.count = idx.numel()
        vals = [float(v) for v in value]
        e.value[:] = vals + [0.0] * (12 - len(vals))
        t = C.c_uint64()
        L.check(L.load().eag_serve_edit(self.h, C.byref(e), C.byref(t)))
        self._keep[t.value] = idx
        return t.value

    def transform(self, idx, r=(1.0, 0.0, 0.0, 0.0), pivot=(0.0, 0.0, 0.0), t=(0.0, 0.0, 0.0)):
        """Queue a rigid motion of the surfels idx (p -> R(r)(p - pivot) +
        pivot + t, q -> r (x) q) with a BVH refit; it waits for the requests
        submitted before it. Returns its ticket."""
        from ._lib import EDIT_TRANSFORM
        return self.edit(EDIT_TRANSFORM, idx, list(r) + list(pivot) + list(t))

    def poll(self, ticket: int):
        """Returns None while running, else a dict with status and times."""
        res = L.Result()
        st = L.load().eag_serve_poll(self.h, ticket, C.byref(res))
        if st == L.EAG_NOT_READY:
            return None
        self._keep.pop(ticket, None)   # the server no longer reads the buffers it was given
        return dict(status=st, version=res.scene_version, t_submit=res.t_submit, t_admit=res.t_admit,
                    t_done=res.t_done, paths=res.paths)

    def wait(self, ticket: int, timeout: float = 120.0):
        import time
        t0 = time.time()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.time() - t0 > timeout:
                raise TimeoutError(f"ticket {ticket} not done after {timeout} s")
            time.sleep(0.0005)

    def cancel(self, ticket: int):
        L.check(L.load().eag_serve_cancel(self.h, ticket))

    def close(self):
        if getattr(self, "h", None):
            h, self.h = self.h, None
            L.check(L.load().eag_serve_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
