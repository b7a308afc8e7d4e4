// Multi-bounce diffuse path tracing (Sec. 3.4, Eq. 9) on the persistent
// segment runner (eag_runner.h): each work item is one path, traced segment
// by segment.
//
// Shading a finished segment: miss -> path ends; E > tau_E -> add beta * R,
// path ends; depth == max_depth -> discarded; otherwise beta *= P, a
// cosine-weighted direction about Nt is drawn with Philox counter (pixel,
// sample, depth, camera id), the path moves to X = O + Dt w, and Russian
// roulette (q = min(0.95, max beta), survive iff u2 < q, beta /= q) applies
// once the new depth reaches rr_start.
// One launch can serve several requests (slots), each with its own camera,
// parameters, accumulator and scene version; the server uses this to batch
// requests that are live at the same time.
//
// Work items are sample-major over 8x8 pixel tiles, so a wave's first
// segments are spatially coherent. Contributions are added to int64 fixed
// point accumulators, which makes every pixel sum independent of the order
// in which lanes finish.
#include "eag_device.h"
#include "eag_internal.h"
#include "eag_render.h"
#include "eag_runner.h"

namespace eag {

namespace {

__device__ __forceinline__ void add_fixed(int64_t* acc, float v) {
  if (v != 0.0f) {
    const long long q = (long long)rint((double)v * EAG_ACCUM_SCALE);
    atomicAdd(reinterpret_cast<unsigned long long*>(acc), (unsigned long long)q);
  }
}

// One lane's path.
struct PathSource {
  const PtLaunch* L;
  int slot;
  uint32_t pix, sample;
  int depth;
  V3 beta;

  __device__ __forceinline__ bool start(int64_t wid, TraceCtx& tcl, D3& O, D3& W) {
    int k = 0;
    while (k < L->n_slots - 1 && wid >= L->s[k].global_end) ++k;
    const PtSlot& S = L->s[k];
    const int64_t item = S.work_begin + (wid - (k ? L->s[k - 1].global_end : 0));
    const int64_t s_rel = item / S.tile_pixels;
    const int64_t tp = item - s_rel * S.tile_pixels;
    const int64_t tile = tp >> 6;
    const int within = (int)(tp & 63);
    const int x = (int)(tile % S.tiles_x) * 8 + (within & 7);
    const int y = (int)(tile / S.tiles_x) * 8 + (within >> 3);
    if (x >= S.cam.width || y >= S.cam.height) return false;
    slot = k;
    pix = (uint32_t)(y * S.cam.width + x);
    sample = S.sample_begin + (uint32_t)s_rel;
    beta = v3(1.f, 1.f, 1.f);
    depth = 0;
    tcl.attrs = S.attrs;
    O = d3(S.cam.eye[0], S.cam.eye[1], S.cam.eye[2]);
    W = pixel_dir(S.cam, pix, sample, S.flags, S.k0, S.k1);
    return true;
  }

  __device__ __forceinline__ void operator()(uint32_t, double, double, double, double, D3, D3) const {}

  __device__ __forceinline__ bool finish(const Seg<false>& s, D3& O, D3& W) {
    const PtSlot& S = L->s[slot];
    const double A = 1.0 - s.T;
    if (s.nhits == 0 || !(A > 0.0)) return false;
    const bool emit = s.E > S.tau_E;
    if ((S.flags & EAG_ADDITIVE_EMISSION) || emit) {
      int64_t* acc = S.accum + (int64_t)pix * 3;
      add_fixed(acc + 0, beta.x * s.R0);
      add_fixed(acc + 1, beta.y * s.R1);
      add_fixed(acc + 2, beta.z * s.R2);
      if (!(S.flags & EAG_ADDITIVE_EMISSION)) return false;
    }
    if (depth >= S.max_depth) return false;
    beta = v3(beta.x * s.P0, beta.y * s.P1, beta.z * s.P2);
    const uint4 w = philox(make_uint4(pix, sample, (uint32_t)depth, S.cam.id), S.k0, S.k1);
    ++depth;
    if (S.rr_start > 0 && depth >= S.rr_start) {
      const float q = fminf(0.95f, fmaxf(fmaxf(beta.x, beta.y), beta.z));
      if (!(to_unit(w.z) < q)) return false;
      const float iq = 1.0f / q;
      beta = v3(beta.x * iq, beta.y * iq, beta.z * iq);
    }
    const D3 Nt = (1.0 / sqrt(dot(s.N, s.N))) * s.N;
    const double Dt = s.D / A;
    O = d3(s.O.x + Dt * s.W.x, s.O.y + Dt * s.W.y, s.O.z + Dt * s.W.z);
    W = cosine_dir(Nt, to_unit(w.x), to_unit(w.y));
    return true;
  }
};

__global__ void __launch_bounds__(TRACE_BLOCK) k_path_trace(TraceCtx tc, PtLaunch L,
                                                            unsigned long long* work_counter,
                                                            unsigned long long* counters, uint64_t* hitlist) {
  PathSource src;
  src.L = &L;
  src.slot = 0;
  src.pix = src.sample = 0;
  src.depth = 0;
  src.beta = v3(1.f, 1.f, 1.f);
  run_segments<Q_ALL, false>(tc, src, work_counter, L.n_work, hitlist, counters);
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

__global__ void k_resolve(const int64_t* accum, int64_t n, double scale, float* rgb) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) rgb[i] = (float)((double)accum[i] * scale);
}

}  // namespace

int64_t runner_lanes() {
  int dev = 0, cus = 0;
  check_hip(hipGetDevice(&dev), "hipGetDevice");
  check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
  return (int64_t)cus * RUN_BLOCKS_PER_CU * TRACE_BLOCK;
}

void launch_zero_u64(unsigned long long* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, p, n);
}

void launch_path_trace(const TraceCtx& tc, const PtLaunch& L, unsigned long long* work_counter,
                       unsigned long long* counters, uint64_t* hitlist, hipStream_t st) {
  const unsigned blocks = (unsigned)(runner_lanes() / TRACE_BLOCK);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, work_counter, 1);
  hipLaunchKernelGGL(k_path_trace, dim3(blocks), dim3(TRACE_BLOCK), 0, st, tc, L, work_counter, counters, hitlist);
  check_hip(hipGetLastError(), "path_trace launch");
}

void launch_accum_resolve(const int64_t* accum, int64_t n_values, double scale, float* rgb, hipStream_t st) {
  hipLaunchKernelGGL(k_resolve, dim3((unsigned)((n_values + 255) / 256)), dim3(256), 0, st, accum, n_values, scale,
                     rgb);
  check_hip(hipGetLastError(), "resolve launch");
}

}  // namespace eag
