// C ABI of the library: argument validation, workspace carving and error
// conversion. Every entry point catches everything and returns a status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "eag_internal.h"
#include "eag_render.h"

namespace eag {

namespace {
thread_local std::string g_last_error;

eag_status set_error(eag_status s, const std::string& m) {
  g_last_error = m;
  return s;
}

template <class F>
eag_status guarded(F&& f) {
  try {
    check_device_status();
    f();
    return EAG_OK;
  } catch (const Error& e) {
    return set_error(e.status, e.msg);
  } catch (const std::bad_alloc&) {
    return set_error(EAG_ERR_INTERNAL, "host allocation failed");
  } catch (...) {
    return set_error(EAG_ERR_INTERNAL, "unexpected exception");
  }
}

int bits_for(int64_t n) {
  int b = 1;
  while ((int64_t(1) << b) < n) ++b;
  return b;
}

bool is_pow2_or_zero(float x) {
  if (x == 0.0f) return true;
  if (!(x > 0.0f) || !std::isfinite(x)) return false;
  int e = 0;
  return std::frexp(x, &e) == 0.5f;
}
}  // namespace

void fail(eag_status s, const std::string& msg) { throw Error{s, msg}; }
void set_last_error(const std::string& msg) { g_last_error = msg; }

void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(EAG_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Errors that only a kernel can see reach the host through one word of
// mapped host memory per process: a kernel stores its code there, and the
// next call into the library reports and clears it (calls stay
// asynchronous; the report comes one call late, as for other device errors).
namespace {
std::mutex g_status_mu;
unsigned int* g_status = nullptr;
}  // namespace

unsigned int* device_status_word() {
  std::lock_guard<std::mutex> g(g_status_mu);
  if (!g_status) {
    void* p = nullptr;
    check_hip(hipHostMalloc(&p, 256, hipHostMallocMapped), "status word");
    g_status = static_cast<unsigned int*>(p);
    __atomic_store_n(g_status, 0u, __ATOMIC_SEQ_CST);
  }
  return g_status;
}

bool device_status_allocated() {
  std::lock_guard<std::mutex> g(g_status_mu);
  return g_status != nullptr;
}

void check_device_status() {
  unsigned int* w = g_status;
  if (!w) return;
  const unsigned int code = __atomic_exchange_n(w, 0u, __ATOMIC_SEQ_CST);
  if (code & EAG_DEVICE_KEY_RANGE)
    fail(EAG_ERR_DEVICE, "an earlier launch met a hit beyond the order key's last depth bucket "
                         "(max_bucket * depth_quantum): raise depth_quantum; its results are invalid");
  if (code & EAG_DEVICE_SORT_RANGE)
    fail(EAG_ERR_DEVICE, "an earlier radix sort computed an output position out of range (an internal error); "
                         "its results are invalid");
  if (code) fail(EAG_ERR_DEVICE, "an earlier launch reported a device error");
}

void bvh_sync_host(eag_bvh* b) {
  check_hip(hipEventSynchronize(b->built), "bvh build wait");
  BvhHeader h;
  check_hip(hipMemcpy(&h, b->hdr, sizeof(h), hipMemcpyDeviceToHost), "bvh header read");
  for (int a = 0; a < 3; ++a) {
    b->lo[a] = header_float(h.blo[a]);
    b->hi[a] = header_float(h.bhi[a]);
  }
  b->max_depth = h.max_depth;
  b->n_nodes4 = h.n_nodes4;
  b->depth4 = h.depth4;
}

void validate_params(const eag_trace_params* p) {
  if (!p) fail(EAG_ERR_INVALID_ARGUMENT, "params is null");
  if (p->kbuf != KBUF) fail(EAG_ERR_INVALID_ARGUMENT, "kbuf must be 16");
  if (p->spp < 1) fail(EAG_ERR_INVALID_ARGUMENT, "spp must be >= 1");
  if (p->max_depth < 0 || p->max_depth > 64) fail(EAG_ERR_INVALID_ARGUMENT, "max_depth must be in [0, 64]");
  if (p->rr_start < 0) fail(EAG_ERR_INVALID_ARGUMENT, "rr_start must be >= 0");
  if (!(p->T_min > 0.0f && p->T_min < 1.0f)) fail(EAG_ERR_INVALID_ARGUMENT, "T_min must be in (0, 1)");
  if (!(p->t_min >= 0.0f) || !std::isfinite(p->t_min)) fail(EAG_ERR_INVALID_ARGUMENT, "t_min must be >= 0");
  if (!(p->k_sigma > 0.0f) || !std::isfinite(p->k_sigma)) fail(EAG_ERR_INVALID_ARGUMENT, "k_sigma must be > 0");
  if (!std::isfinite(p->tau_E)) fail(EAG_ERR_INVALID_ARGUMENT, "tau_E must be finite");
  if (!is_pow2_or_zero(p->depth_quantum))
    fail(EAG_ERR_INVALID_ARGUMENT, "depth_quantum must be 0 or a power of two");
}

TraceSetup trace_setup(const eag_bvh* b, const eag_trace_params* p) {
  TraceSetup ts;
  ts.idx_bits = b->idx_bits;
  const int bucket_bits = 64 - 2 * ts.idx_bits;
  if (p->depth_quantum == 0.0f) {
    if (bucket_bits < 32) fail(EAG_ERR_INVALID_ARGUMENT, "depth_quantum = 0 (exact t order) needs n <= 65536");
    ts.max_bucket = 0xffffffffu;
    ts.inv_dq = 0.0;
  } else {
    // A distance beyond the last bucket (max_bucket * depth_quantum) is
    // detected by the kernels (device status), not here: the scene's extent
    // lives on the device, and the calls do not wait for it.
    ts.max_bucket = bucket_bits >= 32 ? 0xffffffffu : ((1u << bucket_bits) - 1u);
    ts.inv_dq = 1.0 / (double)p->depth_quantum;
  }
  // (the traversal stack holds 3 entries per level of any tree the build
  // can make: STACK_SIZE covers the deepest)
  return ts;
}

CamDev make_cam(const eag_camera& c, uint32_t id) {
  if (c.width < 1 || c.height < 1) fail(EAG_ERR_INVALID_ARGUMENT, "camera size must be >= 1");
  if ((int64_t)c.width * c.height > (int64_t(1) << 31)) fail(EAG_ERR_INVALID_ARGUMENT, "camera too large");
  if (!(c.vfov_deg > 0.0f && c.vfov_deg < 180.0f)) fail(EAG_ERR_INVALID_ARGUMENT, "vfov must be in (0, 180)");
  double e[3], f[3], u[3];
  for (int a = 0; a < 3; ++a) {
    e[a] = c.eye[a];
    f[a] = (double)c.look_at[a] - c.eye[a];
    u[a] = c.up[a];
  }
  const double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(fl > 0)) fail(EAG_ERR_INVALID_ARGUMENT, "camera eye equals look_at");
  for (double& v : f) v /= fl;
  double r[3] = {f[1] * u[2] - f[2] * u[1], f[2] * u[0] - f[0] * u[2], f[0] * u[1] - f[1] * u[0]};
  const double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (!(rl > 1e-12)) fail(EAG_ERR_INVALID_ARGUMENT, "camera up is parallel to the view direction");
  for (double& v : r) v /= rl;
  const double up2[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
  const double th = std::tan(c.vfov_deg * M_PI / 360.0);
  const double aspect = (double)c.width / (double)c.height;
  CamDev d;
  for (int a = 0; a < 3; ++a) {
    d.eye[a] = e[a];
    d.right[a] = r[a] * th * aspect;
    d.up[a] = up2[a] * th;
    d.fwd[a] = f[a];
  }
  d.width = c.width;
  d.height = c.height;
  d.id = id;
  d.pad = 0;
  return d;
}

}  // namespace eag

using namespace eag;

namespace {

// Render / trace workspace: attribute records plus per-call buffers.
struct RenderWs {
  Attr* attrs;
  float* state;
  double* r1;
  float* adj;                 // per-sample dL/dX, dL/dNt of the adjoint
  double* gacc;               // double gradient accumulators of the adjoint
  GradRecs grecs;             // per-hit gradient records of the secondary adjoint
  unsigned long long* work;
  uint64_t* hitlist;          // path tracing: HL_CAP keys per lane of the persistent grid
  size_t bytes;
};

// records: the backward's per-hit gradient records, for camera batches of
// n_pix_batch pixels (the forward needs none).
RenderWs render_ws(void* base, int64_t n, int64_t n_pix, int64_t spp, bool own_state, int64_t hl_lanes = 0,
                   int64_t n_pix_batch = 0, bool records = false) {
  Carver c(base, ~size_t(0));
  RenderWs w;
  w.attrs = c.take<Attr>(n);
  w.state = own_state ? c.take<float>(n_pix * EAG_FWD_PIXEL_FLOATS) : nullptr;
  w.r1 = own_state ? c.take<double>(n_pix * spp * 3) : nullptr;
  w.adj = own_state ? c.take<float>(n_pix * spp * 12) : nullptr;   // 6 doubles per sample
  w.gacc = own_state ? c.take<double>(grad_accum_doubles(n)) : nullptr;
  std::memset(&w.grecs, 0, sizeof(w.grecs));
  if (own_state && records) {
    // sized for the largest camera batch of one launch
    GradRecs& g = w.grecs;
    // (at least one chunk per wave of the persistent grid)
    const int64_t want = grad_rec_capacity(std::min<int64_t>(n_pix, n_pix_batch) * spp);
    g.n_chunks = std::max<int64_t>(std::max<int64_t>(1, hl_lanes / 64), (want + REC_CHUNK - 1) / REC_CHUNK);
    const int64_t cap = g.n_chunks * REC_CHUNK;
    g.chunk_used = c.take<uint32_t>(g.n_chunks);
    g.rec = c.take<float>((size_t)cap * 16);
    g.idx = c.take<uint32_t>(cap);
    g.order = c.take<uint32_t>(cap);
    g.cnt = c.take<uint32_t>(n);
    g.cursor = c.take<uint32_t>(n);
    g.off = c.take<uint32_t>(n);
    g.scan_bytes = grad_rec_scan_bytes(n);
    g.scan_tmp = c.take<char>(g.scan_bytes);
  }
  w.work = c.take<unsigned long long>(8);
  w.hitlist = hl_lanes > 0 ? c.take<uint64_t>((size_t)hl_lanes * HL_CAP) : nullptr;
  w.bytes = c.bytes();
  return w;
}

void check_cams(const eag_camera* cams, int32_t n_cams) {
  if (!cams || n_cams < 1) fail(EAG_ERR_INVALID_ARGUMENT, "need at least one camera");
  for (int i = 1; i < n_cams; ++i)
    if (cams[i].width != cams[0].width || cams[i].height != cams[0].height)
      fail(EAG_ERR_INVALID_ARGUMENT, "all cameras of a batch must have the same size");
}

void check_bvh(const eag_bvh* b, const eag_surfels* s) {
  if (!b) fail(EAG_ERR_INVALID_ARGUMENT, "bvh is null");
  validate_surfels(s);
  if (s->n != b->n) fail(EAG_ERR_INVALID_ARGUMENT, "surfel count differs from the BVH's");
}

// Light-baking workspace: packed attributes, work counter, hit list, double
// radiance-gradient accumulators [3][n], and the image, image gradient and
// loss of eag_bake_step.
struct BakeWs {
  Attr* attrs;
  unsigned long long* work;
  uint64_t* hitlist;
  double* gacc;
  float* rgb;
  float* dL;
  double* loss;
  size_t bytes;
};

BakeWs bake_ws(void* base, int64_t n, int64_t n_values, int64_t hl_lanes) {
  Carver c(base, ~size_t(0));
  BakeWs w;
  w.attrs = c.take<Attr>(n);
  w.work = c.take<unsigned long long>(8);
  w.hitlist = c.take<uint64_t>((size_t)hl_lanes * HL_CAP);
  w.gacc = c.take<double>((size_t)n * 3);
  w.rgb = c.take<float>(n_values);
  w.dL = c.take<float>(n_values);
  w.loss = c.take<double>(1);
  w.bytes = c.bytes();
  return w;
}

// Trace setup, attributes and camera batches shared by the light-baking calls.
struct BakeCall {
  TraceCtx tc;
  SbParams sp;
  int64_t hw;
};

BakeCall bake_setup(const eag_bvh* b, const eag_surfels* s, const eag_camera* cams, int32_t n_cams,
                    const eag_trace_params* p, const BakeWs& w, hipStream_t st) {
  const TraceSetup ts = trace_setup(b, p);
  pack_attrs(s, b, w.attrs, st);
  BakeCall k;
  k.tc = make_ctx(b, w.attrs, p, ts);
  k.tc.hl = w.hitlist;
  k.sp.spp = 1;
  k.sp.flags = p->flags;
  k.sp.k0 = (uint32_t)(p->seed & 0xffffffffu);
  k.sp.k1 = (uint32_t)(p->seed >> 32);
  k.sp.tau_E = p->tau_E;
  k.hw = (int64_t)cams[0].width * cams[0].height;
  return k;
}

template <class F>
void for_camera_batches(const eag_camera* cams, int32_t n_cams, const eag_trace_params* p, F&& f) {
  for (int c0 = 0; c0 < n_cams; c0 += MAX_CAMS_PER_LAUNCH) {
    const int nc = std::min(MAX_CAMS_PER_LAUNCH, n_cams - c0);
    CamBatch cb;
    std::memset(&cb, 0, sizeof(cb));
    for (int i = 0; i < nc; ++i) cb.c[i] = make_cam(cams[c0 + i], p->camera_id + (uint32_t)(c0 + i));
    f(c0, nc, cb);
  }
}

// Stage-0 workspace: packed attributes, work counters, hit list, double
// gradient accumulators and gradient records, the camera pass's colour
// output, the loss counters and the distance-normal contributions.
struct Stage0Ws {
  Attr* attrs;
  unsigned long long* work;
  uint64_t* hitlist;
  double* gacc;
  GradRecs grecs;
  float* rgb;
  unsigned long long* counts;
  float* contrib;
  size_t bytes;
};

Stage0Ws stage0_ws(void* base, int64_t n, int64_t n_pix, int64_t n_pix_batch, int64_t hl_lanes) {
  Carver c(base, ~size_t(0));
  Stage0Ws w;
  w.attrs = c.take<Attr>(n);
  w.work = c.take<unsigned long long>(8);
  w.hitlist = c.take<uint64_t>((size_t)hl_lanes * HL_CAP);
  w.gacc = c.take<double>(grad_accum_doubles(n));
  GradRecs& g = w.grecs;
  std::memset(&g, 0, sizeof(g));
  const int64_t want = grad_rec_capacity(std::min<int64_t>(n_pix, n_pix_batch));
  g.n_chunks = std::max<int64_t>(std::max<int64_t>(1, hl_lanes / 64), (want + REC_CHUNK - 1) / REC_CHUNK);
  const int64_t cap = g.n_chunks * REC_CHUNK;
  g.chunk_used = c.take<uint32_t>(g.n_chunks);
  g.rec = c.take<float>((size_t)cap * 16);
  g.idx = c.take<uint32_t>(cap);
  g.order = c.take<uint32_t>(cap);
  g.cnt = c.take<uint32_t>(n);
  g.cursor = c.take<uint32_t>(n);
  g.off = c.take<uint32_t>(n);
  g.scan_bytes = grad_rec_scan_bytes(n);
  g.scan_tmp = c.take<char>(g.scan_bytes);
  w.rgb = c.take<float>(n_pix * 3);
  w.counts = c.take<unsigned long long>(4);
  w.contrib = c.take<float>(n_pix * 4);
  w.bytes = c.bytes();
  return w;
}

void check_adam(const eag_adam* a) {
  if (!a) fail(EAG_ERR_INVALID_ARGUMENT, "adam parameters are null");
  if (!(a->lr >= 0.0f) || !(a->beta1 >= 0.0f && a->beta1 < 1.0f) || !(a->beta2 >= 0.0f && a->beta2 < 1.0f) ||
      !(a->eps >= 0.0f))
    fail(EAG_ERR_INVALID_ARGUMENT, "adam parameters out of range (lr >= 0, 0 <= beta < 1, eps >= 0)");
}

}  // namespace

extern "C" {

const char* eag_last_error(void) { return g_last_error.c_str(); }
uint32_t eag_abi_version(void) { return EAG_ABI_VERSION; }

void eag_default_params(eag_trace_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->spp = 4;
  p->max_depth = 5;
  p->rr_start = 3;
  p->tau_E = 0.1f;
  p->T_min = 1e-4f;
  p->t_min = 1e-3f;
  p->k_sigma = 3.0f;
  p->depth_quantum = 1.0f / 8192.0f;
  p->kbuf = 16;
  p->camera_id = 0;
  p->seed = 0;
  p->flags = 0;
}

size_t eag_bvh_bytes(int64_t n) { return n < 1 ? 0 : bvh_layout(nullptr, n).bytes; }

size_t eag_build_workspace_bytes(int64_t n) {
  if (n < 1) return 0;
  try {
    return build_ws_bytes(n);
  } catch (...) {
    return 0;
  }
}

eag_status eag_build_bvh(const eag_surfels* s, void* bvh_mem, size_t bvh_bytes, void* ws, size_t ws_bytes,
                         void* stream, eag_bvh** out) {
  return guarded([&] {
    validate_surfels(s);
    if (!out) fail(EAG_ERR_INVALID_ARGUMENT, "out is null");
    if (!bvh_mem || !ws) fail(EAG_ERR_INVALID_ARGUMENT, "bvh_mem and ws must be device buffers");
    if ((reinterpret_cast<uintptr_t>(bvh_mem) & 255) || (reinterpret_cast<uintptr_t>(ws) & 255))
      fail(EAG_ERR_INVALID_ARGUMENT, "bvh_mem and ws must be 256-byte aligned");
    const BvhLayout l = bvh_layout(bvh_mem, s->n);
    if (bvh_bytes < l.bytes) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "bvh_mem too small");
    eag_bvh* b = new eag_bvh();
    b->n = s->n;
    b->idx_bits = bits_for(s->n);
    b->mem = bvh_mem;
    b->mem_bytes = bvh_bytes;
    bvh_attach(b, l);
    try {
      check_hip(hipEventCreateWithFlags(&b->built, hipEventDisableTiming), "build event");
      build_bvh(s, b, ws, ws_bytes, static_cast<hipStream_t>(stream));
    } catch (...) {
      if (b->built) (void)hipEventDestroy(b->built);
      delete b;
      throw;
    }
    *out = b;
  });
}

eag_status eag_refit_bvh(eag_bvh* b, const eag_surfels* s, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    check_bvh(b, s);
    if (!ws) fail(EAG_ERR_INVALID_ARGUMENT, "ws is null");
    refit_bvh(s, b, ws, ws_bytes, static_cast<hipStream_t>(stream));
  });
}

eag_status eag_bvh_get_info(const eag_bvh* b, eag_bvh_info* out) {
  return guarded([&] {
    if (!b || !out) fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
    // the one BVH call that waits: for the last build or refit, then reads
    // the header the device wrote
    bvh_sync_host(const_cast<eag_bvh*>(b));
    out->n = b->n;
    out->max_depth = b->max_depth;
    out->root = b->root;
    for (int a = 0; a < 3; ++a) {
      out->lo[a] = b->lo[a];
      out->hi[a] = b->hi[a];
    }
    out->nodes = b->nodes;
    out->records = b->recs;
    out->perm = b->perm;
    out->nodes4 = b->nodes4;
    out->n_nodes4 = b->n_nodes4;
    out->depth4 = b->depth4;
  });
}

void eag_bvh_destroy(eag_bvh* b) {
  if (!b) return;
  if (b->built) (void)hipEventDestroy(b->built);
  delete b;
}

size_t eag_trace_workspace_bytes(int64_t n) { return n < 1 ? 0 : render_ws(nullptr, n, 0, 0, false).bytes; }

eag_status eag_trace_rays(const eag_bvh* b, const eag_surfels* s, const eag_trace_params* p, int64_t n_rays,
                          const double* origins, const double* dirs, float* out, int32_t* hit_idx, int32_t* hit_count,
                          int32_t max_hits, int32_t* stats, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    check_bvh(b, s);
    validate_params(p);
    if (n_rays < 0) fail(EAG_ERR_INVALID_ARGUMENT, "n_rays < 0");
    if (n_rays > 0 && (!origins || !dirs || !out)) fail(EAG_ERR_INVALID_ARGUMENT, "ray or output pointer is null");
    if (hit_idx && max_hits < 1) fail(EAG_ERR_INVALID_ARGUMENT, "max_hits must be >= 1 with hit_idx");
    const RenderWs w = render_ws(ws, b->n, 0, 0, false);
    if (!ws || ws_bytes < w.bytes) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "trace workspace too small");
    if (n_rays == 0) return;
    const TraceSetup ts = trace_setup(b, p);
    hipStream_t st = static_cast<hipStream_t>(stream);
    pack_attrs(s, b, w.attrs, st);
    launch_trace_rays(b, w.attrs, p, ts, n_rays, origins, dirs, out, hit_idx, hit_count, max_hits, stats, st);
  });
}

eag_status eag_init(void) {
  return guarded([&] {
    (void)device_status_word();
    noalloc_setup_current_device();
  });
}

eag_status eag_trace_rays_noalloc(const eag_bvh* b, const eag_surfels* s, const eag_trace_params* p, int64_t n_rays,
                                  const double* origins, const double* dirs, float* out, int32_t* hit_idx,
                                  int32_t* hit_count, int32_t max_hits, int32_t* stats, void* stream) {
  return guarded([&] {
    check_bvh(b, s);
    validate_params(p);
    if (n_rays < 0) fail(EAG_ERR_INVALID_ARGUMENT, "n_rays < 0");
    if (n_rays > 0 && (!origins || !dirs || !out)) fail(EAG_ERR_INVALID_ARGUMENT, "ray or output pointer is null");
    if (hit_idx && max_hits < 1) fail(EAG_ERR_INVALID_ARGUMENT, "max_hits must be >= 1 with hit_idx");
    if (b->n > EAG_NOALLOC_MAX_SURFELS)
      fail(EAG_ERR_INVALID_ARGUMENT, "eag_trace_rays_noalloc takes at most EAG_NOALLOC_MAX_SURFELS (2^18) surfels");
    Attr* attrs = noalloc_scratch_current_device();
    if (!attrs || !device_status_allocated())
      fail(EAG_ERR_INVALID_ARGUMENT, "eag_trace_rays_noalloc needs eag_init on this device first");
    if (n_rays == 0) return;
    const TraceSetup ts = trace_setup(b, p);
    hipStream_t st = static_cast<hipStream_t>(stream);
    pack_attrs(s, b, attrs, st);   // all n records rewritten: nothing left from an earlier call is read
    launch_trace_rays(b, attrs, p, ts, n_rays, origins, dirs, out, hit_idx, hit_count, max_hits, stats, st);
  });
}

int64_t eag_fwd_state_floats(const eag_camera* cams, int32_t n_cams, const eag_trace_params* p) {
  if (!cams || n_cams < 1 || !p || p->spp < 1) return 0;
  const int64_t np = (int64_t)cams[0].width * cams[0].height * n_cams;
  return np * (EAG_FWD_PIXEL_FLOATS + 6 * (int64_t)p->spp);
}

size_t eag_render_workspace_bytes(int64_t n, const eag_camera* cams, int32_t n_cams, const eag_trace_params* p) {
  if (n < 1 || !cams || n_cams < 1 || !p || p->spp < 1) return 0;
  const int64_t np = (int64_t)cams[0].width * cams[0].height * n_cams;
  try {
    return render_ws(nullptr, n, np, p->spp, true, runner_lanes()).bytes;
  } catch (const Error& e) {
    set_error(e.status, e.msg);
    return 0;
  }
}

size_t eag_backward_workspace_bytes(int64_t n, const eag_camera* cams, int32_t n_cams, const eag_trace_params* p) {
  if (n < 1 || !cams || n_cams < 1 || !p || p->spp < 1) return 0;
  const int64_t hw = (int64_t)cams[0].width * cams[0].height;
  try {
    return render_ws(nullptr, n, hw * n_cams, p->spp, true, runner_lanes(), hw * MAX_CAMS_PER_LAUNCH, true).bytes;
  } catch (const Error& e) {
    set_error(e.status, e.msg);
    return 0;
  }
}

eag_status eag_render_single_bounce(const eag_bvh* b, const eag_surfels* s, const eag_camera* cams, int32_t n_cams,
                                    const eag_trace_params* p, float* rgb, float* fwd_state, void* ws,
                                    size_t ws_bytes, void* stream) {
  return guarded([&] {
    check_bvh(b, s);
    validate_params(p);
    check_cams(cams, n_cams);
    if (!rgb) fail(EAG_ERR_INVALID_ARGUMENT, "rgb is null");
    const int64_t hw = (int64_t)cams[0].width * cams[0].height;
    const int64_t np = hw * n_cams;
    const RenderWs w = render_ws(ws, b->n, np, p->spp, true, runner_lanes());
    if (!ws || ws_bytes < w.bytes) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "render workspace too small");
    const TraceSetup ts = trace_setup(b, p);
    hipStream_t st = static_cast<hipStream_t>(stream);
    pack_attrs(s, b, w.attrs, st);
    const TraceCtx tc = make_ctx(b, w.attrs, p, ts);
    float* state = fwd_state ? fwd_state : w.state;
    double* r1 = fwd_state ? reinterpret_cast<double*>(fwd_state + np * EAG_FWD_PIXEL_FLOATS) : w.r1;
    SbParams sp;
    sp.spp = p->spp;
    sp.flags = p->flags;
    sp.k0 = (uint32_t)(p->seed & 0xffffffffu);
    sp.k1 = (uint32_t)(p->seed >> 32);
    sp.tau_E = p->tau_E;
    for (int c0 = 0; c0 < n_cams; c0 += MAX_CAMS_PER_LAUNCH) {
      const int nc = std::min(MAX_CAMS_PER_LAUNCH, n_cams - c0);
      CamBatch cb;
      std::memset(&cb, 0, sizeof(cb));
      for (int i = 0; i < nc; ++i) cb.c[i] = make_cam(cams[c0 + i], p->camera_id + (uint32_t)(c0 + i));
      launch_single_bounce(tc, cb, hw, nc, sp, state + c0 * hw * EAG_FWD_PIXEL_FLOATS, r1 + c0 * hw * p->spp * 3,
                           rgb + c0 * hw * 3, w.work, w.hitlist, st);
    }
  });
}

eag_status eag_single_bounce_backward(const eag_bvh* b, const eag_surfels* s, const eag_camera* cams, int32_t n_cams,
                                      const eag_trace_params* p, const float* dL_drgb, const float* fwd_state,
                                      const eag_surfel_grads* grads, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    check_bvh(b, s);
    validate_params(p);
    check_cams(cams, n_cams);
    if (!dL_drgb || !fwd_state || !grads) fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
    if (!grads->pos || !grads->rot || !grads->scale || !grads->opacity || !grads->albedo || !grads->radiance)
      fail(EAG_ERR_INVALID_ARGUMENT, "a gradient pointer is null");
    const int64_t hw = (int64_t)cams[0].width * cams[0].height;
    const int64_t np = hw * n_cams;
    const RenderWs w = render_ws(ws, b->n, np, p->spp, true, runner_lanes(), hw * MAX_CAMS_PER_LAUNCH, true);
    if (!ws || ws_bytes < w.bytes) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "backward workspace too small");
    const TraceSetup ts = trace_setup(b, p);
    hipStream_t st = static_cast<hipStream_t>(stream);
    pack_attrs(s, b, w.attrs, st);
    const TraceCtx tc = make_ctx(b, w.attrs, p, ts);
    SbParams sp;
    sp.spp = p->spp;
    sp.flags = p->flags;
    sp.k0 = (uint32_t)(p->seed & 0xffffffffu);
    sp.k1 = (uint32_t)(p->seed >> 32);
    sp.tau_E = p->tau_E;
    const double* r1 = reinterpret_cast<const double*>(fwd_state + np * EAG_FWD_PIXEL_FLOATS);
    launch_grad_zero(w.gacc, b->n, st);
    for (int c0 = 0; c0 < n_cams; c0 += MAX_CAMS_PER_LAUNCH) {
      const int nc = std::min(MAX_CAMS_PER_LAUNCH, n_cams - c0);
      CamBatch cb;
      std::memset(&cb, 0, sizeof(cb));
      for (int i = 0; i < nc; ++i) cb.c[i] = make_cam(cams[c0 + i], p->camera_id + (uint32_t)(c0 + i));
      launch_single_bounce_backward(tc, *s, cb, hw, nc, sp, fwd_state + c0 * hw * EAG_FWD_PIXEL_FLOATS,
                                    r1 + c0 * hw * p->spp * 3, dL_drgb + c0 * hw * 3, w.gacc, w.adj, w.grecs,
                                    w.work, w.hitlist, st);
    }
    launch_grad_finalize(w.gacc, b->n, *grads, st);
  });
}

size_t eag_path_trace_workspace_bytes(int64_t n) {
  if (n < 1) return 0;
  try {
    return render_ws(nullptr, n, 0, 0, false, runner_lanes()).bytes;
  } catch (const Error& e) {
    set_error(e.status, e.msg);
    return 0;
  }
}

namespace {
// One request's path-tracing launch: all its work items (sample_count
// samples of every pixel, in 8x8 tiles) in slot 0.
PtLaunch single_request_launch(const CamDev& cd, const eag_camera& cam, const eag_trace_params* p, const Attr* attrs,
                               int64_t* accum, uint32_t sample_begin, uint32_t sample_count) {
  PtLaunch L;
  std::memset(&L, 0, sizeof(L));
  PtSlot& S = L.s[0];
  S.cam = cd;
  S.accum = accum;
  S.attrs = attrs;
  S.work_begin = 0;
  S.tiles_x = (cam.width + 7) / 8;
  S.tile_pixels = (int64_t)S.tiles_x * ((cam.height + 7) / 8) * 64;
  S.global_end = (int64_t)sample_count * S.tile_pixels;
  S.sample_begin = sample_begin;
  S.max_depth = p->max_depth;
  S.rr_start = p->rr_start;
  S.flags = p->flags;
  S.k0 = (uint32_t)(p->seed & 0xffffffffu);
  S.k1 = (uint32_t)(p->seed >> 32);
  S.tau_E = p->tau_E;
  L.n_slots = 1;
  L.n_work = S.global_end;
  return L;
}
}  // namespace

eag_status eag_path_trace(const eag_bvh* b, const eag_surfels* s, const eag_camera* cam, const eag_trace_params* p,
                          uint32_t sample_begin, uint32_t sample_count, int64_t* accum, uint64_t* counters, void* ws,
                          size_t ws_bytes, void* stream) {
  return guarded([&] {
    check_bvh(b, s);
    validate_params(p);
    if (!cam || !accum) fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
    if ((uint64_t)sample_begin + sample_count > 0xffffffffull) fail(EAG_ERR_INVALID_ARGUMENT, "sample range overflow");
    const RenderWs w = render_ws(ws, b->n, 0, 0, false, runner_lanes());
    if (!ws || ws_bytes < w.bytes) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "path-trace workspace too small");
    const CamDev cd = make_cam(*cam, p->camera_id);
    const TraceSetup ts = trace_setup(b, p);
    if (sample_count == 0) return;
    hipStream_t st = static_cast<hipStream_t>(stream);
    pack_attrs(s, b, w.attrs, st);
    const TraceCtx tc = make_ctx(b, w.attrs, p, ts);
    const PtLaunch L = single_request_launch(cd, *cam, p, w.attrs, accum, sample_begin, sample_count);
    launch_path_trace(tc, L, w.work, reinterpret_cast<unsigned long long*>(counters), w.hitlist, st);
  });
}

size_t eag_emitters_bytes(int64_t n) {
  if (n < 1) return 0;
  try {
    return emitters_mem_bytes(n);
  } catch (const Error& e) {
    set_error(e.status, e.msg);
    return 0;
  }
}

size_t eag_emitters_workspace_bytes(int64_t n) {
  if (n < 1) return 0;
  try {
    return emitters_ws_bytes(n);
  } catch (const Error& e) {
    set_error(e.status, e.msg);
    return 0;
  }
}

eag_status eag_build_emitters(const eag_surfels* s, const eag_trace_params* p, float cell, void* mem, size_t mem_bytes,
                              void* ws, size_t ws_bytes, void* stream, eag_emitters** out) {
  return guarded([&] {
    validate_surfels(s);
    validate_params(p);
    if (!out) fail(EAG_ERR_INVALID_ARGUMENT, "out is null");
    if (!(p->tau_E >= 0.0f)) fail(EAG_ERR_INVALID_ARGUMENT, "emitter sampling needs tau_E >= 0");
    if (!(p->k_sigma <= 3.0f)) fail(EAG_ERR_INVALID_ARGUMENT, "emitter sampling needs k_sigma <= 3");
    if (cell != 0.0f) {
      int e = 0;
      if (!(cell >= 0x1p-10f && cell <= 0x1p10f) || std::frexp(cell, &e) != 0.5f)
        fail(EAG_ERR_INVALID_ARGUMENT, "cell must be 0 or a power of two in [2^-10, 2^10]");
    }
    if (!mem || !ws) fail(EAG_ERR_INVALID_ARGUMENT, "mem and ws must be device buffers");
    if ((reinterpret_cast<uintptr_t>(mem) & 255) || (reinterpret_cast<uintptr_t>(ws) & 255))
      fail(EAG_ERR_INVALID_ARGUMENT, "mem and ws must be 256-byte aligned");
    eag_emitters* e = new eag_emitters();
    try {
      build_emitters(s, p->tau_E, p->k_sigma, cell, mem, mem_bytes, ws, ws_bytes, static_cast<hipStream_t>(stream), e);
    } catch (...) {
      delete e;
      throw;
    }
    *out = e;
  });
}

eag_status eag_emitters_get_info(const eag_emitters* em, int64_t* count, double* total_weight, int32_t* n_cells) {
  return guarded([&] {
    if (!em) fail(EAG_ERR_INVALID_ARGUMENT, "emitter table is null");
    if (count) *count = em->dev.n;
    if (total_weight) *total_weight = em->dev.W;
    if (n_cells) *n_cells = em->dev.n_cells;
  });
}

void eag_emitters_destroy(eag_emitters* em) {
  if (!em) return;
  eag_bvh_destroy(em->bvh);
  delete em;
}

size_t eag_path_trace_mis_workspace_bytes(int64_t n, const eag_camera* cam, const eag_trace_params* p) {
  if (n < 1 || !cam || !p || cam->width < 1 || cam->height < 1 || p->max_depth < 0) return 0;
  try {
    const int64_t entries = pdf_queue_entries((int64_t)cam->width * cam->height, p->max_depth, MIS_CHUNK_SPP);
    return render_ws(nullptr, n, 0, 0, false, runner_lanes()).bytes + align_up(pdf_queue_bytes(entries));
  } catch (const Error& e) {
    set_error(e.status, e.msg);
    return 0;
  }
}

eag_status eag_path_trace_mis(const eag_bvh* b, const eag_surfels* s, const eag_emitters* em, const eag_camera* cam,
                              const eag_trace_params* p, uint32_t sample_begin, uint32_t sample_count,
                              int64_t* accum, uint64_t* counters, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    check_bvh(b, s);
    validate_params(p);
    if (!cam || !accum || !em) fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
    if (em->n_src != s->n) fail(EAG_ERR_INVALID_ARGUMENT, "emitter table built for another surfel count");
    if (em->tau_E != p->tau_E || em->k_sigma != p->k_sigma)
      fail(EAG_ERR_INVALID_ARGUMENT, "emitter table built for another tau_E or k_sigma");
    if (p->flags & EAG_ADDITIVE_EMISSION)
      fail(EAG_ERR_INVALID_ARGUMENT, "emitter sampling is defined for the emitter-terminated path tracer");
    if ((uint64_t)sample_begin + sample_count > 0xffffffffull) fail(EAG_ERR_INVALID_ARGUMENT, "sample range overflow");
    const RenderWs w = render_ws(ws, b->n, 0, 0, false, runner_lanes());
    // Samples per launch: as many as the caller's queue holds, up to
    // MIS_CHUNK_SPP (the size eag_path_trace_mis_workspace_bytes returns).
    const int64_t per_sample = pdf_queue_entries((int64_t)cam->width * cam->height, p->max_depth, 1);
    uint32_t chunk = 0;
    if (ws && ws_bytes >= w.bytes) {
      for (uint32_t c = MIS_CHUNK_SPP; c >= 1 && !chunk; --c)
        if (ws_bytes - w.bytes >= align_up(pdf_queue_bytes(per_sample * c))) chunk = c;
    }
    if (!chunk)
      fail(EAG_ERR_WORKSPACE_TOO_SMALL, "path-trace workspace too small for one sample's light-pdf queue "
                                        "(eag_path_trace_mis_workspace_bytes)");
    const int64_t entries = per_sample * chunk;
    void* queue = static_cast<char*>(ws) + w.bytes;
    const CamDev cd = make_cam(*cam, p->camera_id);
    const TraceSetup ts = trace_setup(b, p);
    if (sample_count == 0) return;
    hipStream_t st = static_cast<hipStream_t>(stream);
    pack_attrs(s, b, w.attrs, st);
    const TraceCtx tc = make_ctx(b, w.attrs, p, ts);
    // launches of at most `chunk` samples, each followed by its light pdfs
    for (uint64_t c0 = 0; c0 < sample_count; c0 += chunk) {
      const uint32_t cnt = (uint32_t)std::min<uint64_t>(chunk, sample_count - c0);
      const PtLaunch L = single_request_launch(cd, *cam, p, w.attrs, accum, sample_begin + (uint32_t)c0, cnt);
      launch_path_trace_mis(tc, L, em->dev, queue, entries, w.work, reinterpret_cast<unsigned long long*>(counters),
                            w.hitlist, st);
    }
  });
}

size_t eag_bake_workspace_bytes(int64_t n, const eag_camera* cams, int32_t n_cams) {
  if (n < 1 || !cams || n_cams < 1) return 0;
  try {
    return bake_ws(nullptr, n, (int64_t)cams[0].width * cams[0].height * n_cams * 3, runner_lanes()).bytes;
  } catch (const Error& e) {
    set_error(e.status, e.msg);
    return 0;
  }
}

eag_status eag_render_zero_bounce(const eag_bvh* b, const eag_surfels* s, const eag_camera* cams, int32_t n_cams,
                                  const eag_trace_params* p, float* rgb, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    check_bvh(b, s);
    validate_params(p);
    check_cams(cams, n_cams);
    if (!rgb) fail(EAG_ERR_INVALID_ARGUMENT, "rgb is null");
    const int64_t hw = (int64_t)cams[0].width * cams[0].height;
    const BakeWs w = bake_ws(ws, b->n, hw * n_cams * 3, runner_lanes());
    if (!ws || ws_bytes < w.bytes) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "bake workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const BakeCall k = bake_setup(b, s, cams, n_cams, p, w, st);
    for_camera_batches(cams, n_cams, p, [&](int c0, int nc, const CamBatch& cb) {
      launch_zero_bounce(k.tc, cb, hw, nc, k.sp, rgb + c0 * hw * 3, w.work, w.hitlist, st);
    });
  });
}

eag_status eag_zero_bounce_backward(const eag_bvh* b, const eag_surfels* s, const eag_camera* cams, int32_t n_cams,
                                    const eag_trace_params* p, const float* dL_drgb, float* grad_radiance, void* ws,
                                    size_t ws_bytes, void* stream) {
  return guarded([&] {
    check_bvh(b, s);
    validate_params(p);
    check_cams(cams, n_cams);
    if (!dL_drgb || !grad_radiance) fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
    const int64_t hw = (int64_t)cams[0].width * cams[0].height;
    const BakeWs w = bake_ws(ws, b->n, hw * n_cams * 3, runner_lanes());
    if (!ws || ws_bytes < w.bytes) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "bake workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const BakeCall k = bake_setup(b, s, cams, n_cams, p, w, st);
    launch_zero_f64(w.gacc, b->n * 3, st);
    for_camera_batches(cams, n_cams, p, [&](int c0, int nc, const CamBatch& cb) {
      launch_zero_bounce_adj_r(k.tc, cb, hw, nc, k.sp, dL_drgb + c0 * hw * 3, w.gacc, b->n, w.work, w.hitlist, st);
    });
    launch_add_grad(w.gacc, b->n * 3, grad_radiance, st);
  });
}

eag_status eag_bake_loss(const float* rgb, const float* target, int64_t n_values, float* dL_drgb, double* loss,
                         void* stream) {
  return guarded([&] {
    if (!rgb || !target || !dL_drgb || !loss || n_values < 0) fail(EAG_ERR_INVALID_ARGUMENT, "bad loss arguments");
    launch_bake_loss(rgb, target, n_values, dL_drgb, loss, static_cast<hipStream_t>(stream));
  });
}

eag_status eag_adam_step(float* param, const float* grad, float* m, float* v, int64_t n, const eag_adam* a,
                         int32_t step, void* stream) {
  return guarded([&] {
    if (!param || !grad || !m || !v || n < 0) fail(EAG_ERR_INVALID_ARGUMENT, "bad adam arguments");
    check_adam(a);
    if (step < 1) fail(EAG_ERR_INVALID_ARGUMENT, "adam step counts from 1");
    launch_adam(param, grad, m, v, n, *a, step, static_cast<hipStream_t>(stream));
  });
}

eag_status eag_bake_step(const eag_bvh* b, const eag_surfels* s, const eag_camera* cams, int32_t n_cams,
                         const eag_trace_params* p, const float* targets, float* radiance, float* m, float* v,
                         const eag_adam* a, int32_t step, double* loss, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    check_bvh(b, s);
    validate_params(p);
    check_cams(cams, n_cams);
    check_adam(a);
    if (!targets || !radiance || !m || !v || !loss) fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
    if (radiance != s->radiance) fail(EAG_ERR_INVALID_ARGUMENT, "radiance must be the scene's radiance array");
    if (step < 1) fail(EAG_ERR_INVALID_ARGUMENT, "adam step counts from 1");
    const int64_t hw = (int64_t)cams[0].width * cams[0].height;
    const int64_t nv = hw * n_cams * 3;
    const BakeWs w = bake_ws(ws, b->n, nv, runner_lanes());
    if (!ws || ws_bytes < w.bytes) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "bake workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const BakeCall k = bake_setup(b, s, cams, n_cams, p, w, st);
    for_camera_batches(cams, n_cams, p, [&](int c0, int nc, const CamBatch& cb) {
      launch_zero_bounce(k.tc, cb, hw, nc, k.sp, w.rgb + c0 * hw * 3, w.work, w.hitlist, st);
    });
    launch_bake_loss(w.rgb, targets, nv, w.dL, loss, st);
    launch_zero_f64(w.gacc, b->n * 3, st);
    for_camera_batches(cams, n_cams, p, [&](int c0, int nc, const CamBatch& cb) {
      launch_zero_bounce_adj_r(k.tc, cb, hw, nc, k.sp, w.dL + c0 * hw * 3, w.gacc, b->n, w.work, w.hitlist, st);
    });
    launch_adam(radiance, w.gacc, m, v, b->n * 3, *a, step, st);
  });
}

size_t eag_stage0_workspace_bytes(int64_t n, const eag_camera* cams, int32_t n_cams) {
  if (n < 1 || !cams || n_cams < 1) return 0;
  try {
    const int64_t hw = (int64_t)cams[0].width * cams[0].height;
    return stage0_ws(nullptr, n, hw * n_cams, hw * MAX_CAMS_PER_LAUNCH, runner_lanes()).bytes;
  } catch (const Error& e) {
    set_error(e.status, e.msg);
    return 0;
  }
}

eag_status eag_render_stage0(const eag_bvh* b, const eag_surfels* s, const eag_camera* cams, int32_t n_cams,
                             const eag_trace_params* p, float* images, float* fwd_state, void* ws, size_t ws_bytes,
                             void* stream) {
  return guarded([&] {
    check_bvh(b, s);
    validate_params(p);
    check_cams(cams, n_cams);
    if (!images || !fwd_state) fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
    const int64_t hw = (int64_t)cams[0].width * cams[0].height;
    const Stage0Ws w = stage0_ws(ws, b->n, hw * n_cams, hw * MAX_CAMS_PER_LAUNCH, runner_lanes());
    if (!ws || ws_bytes < w.bytes) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "stage-0 workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const TraceSetup ts = trace_setup(b, p);
    pack_attrs(s, b, w.attrs, st);
    const TraceCtx tc = make_ctx(b, w.attrs, p, ts);
    SbParams sp;
    sp.spp = 1;
    sp.flags = p->flags;
    sp.k0 = (uint32_t)(p->seed & 0xffffffffu);
    sp.k1 = (uint32_t)(p->seed >> 32);
    sp.tau_E = p->tau_E;
    for_camera_batches(cams, n_cams, p, [&](int c0, int nc, const CamBatch& cb) {
      launch_camera_pass(tc, cb, hw, nc, sp, fwd_state + c0 * hw * EAG_FWD_PIXEL_FLOATS, w.rgb + c0 * hw * 3, w.work,
                         w.hitlist, st);
    });
    launch_stage0_images(fwd_state, hw * n_cams, images, st);
  });
}

eag_status eag_stage0_loss(const float* images, const float* rgb_gt, const float* normal_mono, const float* mask,
                           const eag_camera* cams, int32_t n_cams, const eag_trace_params* p, const float* weights,
                           float* d_images, double* loss, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    validate_params(p);
    check_cams(cams, n_cams);
    if (!images || !rgb_gt || !normal_mono || !mask || !weights || !d_images || !loss)
      fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
    const int64_t W = cams[0].width, H = cams[0].height, hw = W * H, np = hw * n_cams;
    // (only the counters and contributions of the workspace are used: its size depends on no scene)
    Carver c(ws, ~size_t(0));
    unsigned long long* counts = c.take<unsigned long long>(4);
    float* contrib = c.take<float>(np * 4);
    if (!ws || ws_bytes < c.bytes()) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "stage-0 loss workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    SbParams sp;
    sp.spp = 1;
    sp.flags = p->flags;
    sp.k0 = (uint32_t)(p->seed & 0xffffffffu);
    sp.k1 = (uint32_t)(p->seed >> 32);
    sp.tau_E = p->tau_E;
    const double wt[4] = {weights[0], weights[1], weights[2], weights[3]};
    launch_stage0_count(images, np, W, H, counts, loss, st);
    for_camera_batches(cams, n_cams, p, [&](int c0, int nc, const CamBatch& cb) {
      launch_stage0_loss_batch(images, rgb_gt, normal_mono, mask, cb, c0 * hw, nc * hw, W, H, sp, wt, counts,
                               contrib, d_images, loss, st);
    });
    launch_stage0_gather(contrib, np, W, H, d_images, st);
  });
}

size_t eag_stage0_loss_workspace_bytes(const eag_camera* cams, int32_t n_cams) {
  if (!cams || n_cams < 1) return 0;
  Carver c(nullptr, ~size_t(0));
  c.take<unsigned long long>(4);
  c.take<float>((int64_t)cams[0].width * cams[0].height * n_cams * 4);
  return c.bytes();
}

eag_status eag_stage0_backward(const eag_bvh* b, const eag_surfels* s, const eag_camera* cams, int32_t n_cams,
                               const eag_trace_params* p, const float* d_images, const float* fwd_state,
                               const eag_surfel_grads* grads, float* grad_emissive, void* ws, size_t ws_bytes,
                               void* stream) {
  return guarded([&] {
    check_bvh(b, s);
    validate_params(p);
    check_cams(cams, n_cams);
    if (!d_images || !fwd_state || !grads || !grad_emissive) fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
    if (!grads->pos || !grads->rot || !grads->scale || !grads->opacity || !grads->radiance)
      fail(EAG_ERR_INVALID_ARGUMENT, "a gradient pointer is null");
    const int64_t hw = (int64_t)cams[0].width * cams[0].height;
    const Stage0Ws w = stage0_ws(ws, b->n, hw * n_cams, hw * MAX_CAMS_PER_LAUNCH, runner_lanes());
    if (!ws || ws_bytes < w.bytes) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "stage-0 workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const TraceSetup ts = trace_setup(b, p);
    pack_attrs(s, b, w.attrs, st);
    const TraceCtx tc = make_ctx(b, w.attrs, p, ts);
    SbParams sp;
    sp.spp = 1;
    sp.flags = p->flags;
    sp.k0 = (uint32_t)(p->seed & 0xffffffffu);
    sp.k1 = (uint32_t)(p->seed >> 32);
    sp.tau_E = p->tau_E;
    launch_grad_zero(w.gacc, b->n, st);
    for_camera_batches(cams, n_cams, p, [&](int c0, int nc, const CamBatch& cb) {
      launch_stage0_backward(tc, *s, cb, hw, nc, sp, fwd_state + c0 * hw * EAG_FWD_PIXEL_FLOATS,
                             d_images + c0 * hw * STAGE0_FLOATS, w.gacc, w.grecs, w.work, w.hitlist, st);
    });
    launch_stage0_finalize(w.gacc, b->n, *grads, grad_emissive, st);
  });
}

size_t eag_select_workspace_bytes(int64_t n) {
  if (n < 1) return 0;
  try {
    Carver c(nullptr, ~size_t(0));
    c.take<uint32_t>(n);
    c.take<uint32_t>(n);
    c.take<char>(select_scan_bytes(n));
    return c.bytes();
  } catch (const Error& e) {
    set_error(e.status, e.msg);
    return 0;
  }
}

eag_status eag_select_box(const eag_surfels* s, const float* lo, const float* hi, int32_t* idx, int64_t* count,
                          void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    validate_surfels(s);
    if (!lo || !hi || !idx || !count) fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
    if (s->n > INT32_MAX) fail(EAG_ERR_INVALID_ARGUMENT, "selection indices are int32");
    Carver c(ws, ~size_t(0));
    uint32_t* flags = c.take<uint32_t>(s->n);
    uint32_t* scan = c.take<uint32_t>(s->n);
    const size_t tb = select_scan_bytes(s->n);
    void* tmp = c.take<char>(tb);
    if (!ws || ws_bytes < c.bytes()) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "selection workspace too small");
    launch_select_box(s->pos, s->n, lo, hi, flags, scan, tmp, tb, idx, count, static_cast<hipStream_t>(stream));
  });
}

static void check_motion(const float* r, const float* pivot, const float* t) {
  if (!r || !pivot || !t) fail(EAG_ERR_INVALID_ARGUMENT, "null motion");
  const double l = (double)r[0] * r[0] + (double)r[1] * r[1] + (double)r[2] * r[2] + (double)r[3] * r[3];
  if (!(l > 1e-20) || !std::isfinite(l)) fail(EAG_ERR_INVALID_ARGUMENT, "rotation quaternion must be non-zero");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(pivot[k]) || !std::isfinite(t[k])) fail(EAG_ERR_INVALID_ARGUMENT, "non-finite motion");
}

eag_status eag_move_surfels(const eag_surfels_out* s, const int32_t* idx, int64_t count, const float* r,
                            const float* pivot, const float* t, void* stream) {
  return guarded([&] {
    if (!s || s->n < 1 || !s->pos || !s->rot) fail(EAG_ERR_INVALID_ARGUMENT, "bad surfel arrays");
    if (count < 0 || (count > 0 && !idx)) fail(EAG_ERR_INVALID_ARGUMENT, "bad index list");
    check_motion(r, pivot, t);
    launch_move(s->pos, s->rot, s->n, idx, count, r, pivot, t, static_cast<hipStream_t>(stream));
  });
}

eag_status eag_delete_surfels(const eag_surfels_out* s, const int32_t* idx, int64_t count, void* stream) {
  return guarded([&] {
    if (!s || s->n < 1 || !s->opacity) fail(EAG_ERR_INVALID_ARGUMENT, "bad surfel arrays");
    if (count < 0 || (count > 0 && !idx)) fail(EAG_ERR_INVALID_ARGUMENT, "bad index list");
    launch_delete(s->opacity, s->n, idx, count, static_cast<hipStream_t>(stream));
  });
}

eag_status eag_duplicate_surfels(const eag_surfels* src, const int32_t* idx, int64_t count, const eag_surfels_out* dst,
                                 const float* r, const float* pivot, const float* t, void* stream) {
  return guarded([&] {
    validate_surfels(src);
    if (!dst || !dst->pos || !dst->rot || !dst->scale || !dst->opacity || !dst->albedo || !dst->radiance ||
        !dst->emissive)
      fail(EAG_ERR_INVALID_ARGUMENT, "bad destination arrays");
    if (count < 0 || (count > 0 && !idx)) fail(EAG_ERR_INVALID_ARGUMENT, "bad index list");
    if (dst->n != src->n + count) fail(EAG_ERR_INVALID_ARGUMENT, "destination must hold n + count surfels");
    check_motion(r, pivot, t);
    launch_append(*src, idx, count, *dst, r, pivot, t, static_cast<hipStream_t>(stream));
  });
}

eag_status eag_bvh_sah_cost(const eag_bvh* b, double* cost, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    if (!b || !cost) fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
    if (!ws || ws_bytes < 2 * sizeof(double)) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "tree-cost workspace too small");
    launch_sah_cost(b->nodes4, b->hdr, b->n - 1, b->root, static_cast<double*>(ws), cost,
                    static_cast<hipStream_t>(stream));
  });
}

eag_status eag_accum_resolve(const int64_t* accum, int64_t n_pixels, int32_t total_spp, float* rgb, void* stream) {
  return guarded([&] {
    if (!accum || !rgb || n_pixels < 0 || total_spp < 1) fail(EAG_ERR_INVALID_ARGUMENT, "bad resolve arguments");
    if (n_pixels == 0) return;
    launch_accum_resolve(accum, n_pixels * 3, 1.0 / (EAG_ACCUM_SCALE * (double)total_spp), rgb,
                         static_cast<hipStream_t>(stream));
  });
}

eag_status eag_apply_edit(const eag_edit* e, const eag_surfel_attrs* a, void* stream) {
  return guarded([&] {
    if (!e || !a) fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
    if (a->n < 1 || !a->albedo || !a->radiance || !a->emissive) fail(EAG_ERR_INVALID_ARGUMENT, "bad attribute arrays");
    if (e->count < 0 || (e->count > 0 && !e->idx)) fail(EAG_ERR_INVALID_ARGUMENT, "bad edit index list");
    if (e->kind < EAG_EDIT_SET_RADIANCE || e->kind > EAG_EDIT_SET_EMISSIVE)
      fail(EAG_ERR_INVALID_ARGUMENT, "bad edit kind (attribute kinds only; eag_move_surfels applies motions)");
    if (e->count == 0) return;
    launch_apply_edit(*e, *a, static_cast<hipStream_t>(stream));
  });
}

}  // extern "C"
