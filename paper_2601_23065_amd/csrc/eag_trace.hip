// Tracing of caller-supplied rays (Sec. 3.1, Eq. 1-3): one thread per ray,
// multi-round k-buffer traversal and front-to-back blending, output of the
// normalised traced quantities and, optionally, the blended hit list.
#include "eag_device.h"
#include "eag_internal.h"

#include <mutex>

// Scratch of eag_trace_rays_noalloc: the packed attribute records of a scene
// of at most EAG_NOALLOC_MAX_SURFELS surfels (32 B each, 8 MiB in all).
// Static device memory: every device the library runs on holds its own copy
// until the process ends, at its own address (looked up per device by
// eag_init), and the calls on one device share it.
static __device__ __align__(256) eag::Attr scratch[EAG_NOALLOC_MAX_SURFELS];

namespace eag {

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
Attr* g_scratch[MAX_DEVICES] = {};   // the array's device address on each device, once looked up
}  // namespace

void noalloc_setup_current_device() {
  int dev = 0;
  check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= MAX_DEVICES) fail(EAG_ERR_INVALID_ARGUMENT, "device index beyond the library's table");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch[dev]) return;
  void* ptr = nullptr;
  check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "no-alloc scratch address");
  if (!ptr) fail(EAG_ERR_DEVICE, "no-alloc scratch has no device address");
  g_scratch[dev] = static_cast<Attr*>(ptr);
}

Attr* noalloc_scratch_current_device() {
  int dev = 0;
  check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch[dev];
}

namespace {

__global__ void __launch_bounds__(256) k_trace_rays(TraceCtx tc, int64_t n_rays, const double* o, const double* d,
                                                    float* out, int32_t* hit_idx, int32_t* hit_count,
                                                    int32_t max_hits, int32_t* stats) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n_rays) return;
  const D3 O = d3(o[i], o[n_rays + i], o[2 * n_rays + i]);
  const D3 W = d3(d[i], d[n_rays + i], d[2 * n_rays + i]);
  int32_t* hl = hit_idx ? hit_idx + i * (int64_t)max_hits : nullptr;
  const SegOut s = trace_segment<Q_ALL, true>(tc, O, W, hl, max_hits);
  const double A = 1.0 - s.T;
  float v[12];
  if (s.nhits > 0 && A > 0.0) {
    const double il = 1.0 / sqrt(dot(s.N, s.N));
    v[0] = (float)(s.N.x * il); v[1] = (float)(s.N.y * il); v[2] = (float)(s.N.z * il);
    v[3] = (float)(s.D / A);
  } else {
    v[0] = v[1] = v[2] = v[3] = 0.0f;
  }
  v[4] = (float)s.R.x; v[5] = (float)s.R.y; v[6] = (float)s.R.z;
  v[7] = (float)s.E;
  v[8] = (float)s.P.x; v[9] = (float)s.P.y; v[10] = (float)s.P.z;
  v[11] = s.nhits > 0 ? (float)A : 0.0f;
#pragma unroll
  for (int k = 0; k < 12; ++k) out[k * n_rays + i] = v[k];
  if (hit_count) hit_count[i] = s.nhits;
  if (stats) {
    stats[i * 3 + 0] = s.rounds;
    stats[i * 3 + 1] = s.tests;
    stats[i * 3 + 2] = s.visits;
  }
}

}  // namespace

TraceCtx make_ctx(const eag_bvh* b, const Attr* attrs, const eag_trace_params* p, const TraceSetup& ts) {
  TraceCtx tc;
  tc.nodes = b->nodes4;
  tc.recs = b->recs;
  tc.attrs = attrs;
  tc.root = b->root;
  tc.idx_bits = ts.idx_bits;
  tc.max_bucket = ts.max_bucket;
  tc.inv_dq = ts.inv_dq;
  tc.dq = ts.inv_dq > 0.0 ? 1.0 / ts.inv_dq : 0.0;
  tc.t_min = p->t_min;
  tc.k2 = (double)p->k_sigma * (double)p->k_sigma;
  tc.T_min = p->T_min;
  tc.hl = nullptr;
  tc.status = device_status_word();
  return tc;
}

void launch_trace_rays(const eag_bvh* b, const Attr* attrs, const eag_trace_params* p, const TraceSetup& ts,
                       int64_t n_rays, const double* o, const double* d, float* out, int32_t* hit_idx,
                       int32_t* hit_count, int32_t max_hits, int32_t* stats, hipStream_t st) {
  const TraceCtx tc = make_ctx(b, attrs, p, ts);
  const unsigned g = (unsigned)((n_rays + 255) / 256);
  hipLaunchKernelGGL(k_trace_rays, dim3(g), dim3(256), 0, st, tc, n_rays, o, d, out, hit_idx, hit_count,
                     max_hits, stats);
  check_hip(hipGetLastError(), "trace_rays launch");
}

}  // namespace eag
