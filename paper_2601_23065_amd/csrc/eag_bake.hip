// Light baking (Sec. 3.4, "Light Baking", Eq. 10): the per-surfel radiance r
// is refitted so that the 0-bounce image (R composited along the camera ray,
// Sec. 3.2) matches path-traced renders, min_r L1(PQ(L0), PQ(Lpt)).
//
// k_zero_bounce        one work item per pixel on the persistent segment
//                      runner: the camera ray through the pixel (sample 0),
//                      blending r only; writes R.
// k_zero_bounce_adj_r  the same rays re-traced: every blended hit adds
//                      w_i dL to its surfel's radiance gradient (L0 is linear
//                      in r, with weights w_i = T_{i-1} alpha_i that do not
//                      depend on it); double atomics into the workspace.
// k_bake_loss          per value: |PQ(L0) - PQ(Lpt)| (summed per block, then
//                      one double atomic per block) and its derivative
//                      sign * PQ'(L0) / count.
// k_adam               Adam with bias correction on r, then r clamped at 0.
//
// PQ is SMPTE ST 2084 on Y = max(L, 0) / 10000 (radiance read as cd/m^2),
// its derivative taken at max(Y, 2^-24); double precision throughout.
#include "eag_device.h"
#include "eag_internal.h"
#include "eag_render.h"
#include "eag_runner.h"

#include <cmath>

namespace eag {

namespace {

constexpr double PQ_M1 = 2610.0 / 16384.0;
constexpr double PQ_M2 = 2523.0 / 4096.0 * 128.0;
constexpr double PQ_C1 = 3424.0 / 4096.0;
constexpr double PQ_C2 = 2413.0 / 4096.0 * 32.0;
constexpr double PQ_C3 = 2392.0 / 4096.0 * 32.0;
constexpr double PQ_PEAK = 10000.0;
constexpr double PQ_YMIN = 5.9604644775390625e-08;   // 2^-24

__device__ __forceinline__ double pq_curve(double L) {
  const double ym = pow(fmax(L, 0.0) / PQ_PEAK, PQ_M1);
  return pow((PQ_C1 + PQ_C2 * ym) / (1.0 + PQ_C3 * ym), PQ_M2);
}

__device__ __forceinline__ double pq_slope(double L) {
  if (L < 0.0) return 0.0;
  const double y = fmax(L / PQ_PEAK, PQ_YMIN);
  const double ym = pow(y, PQ_M1);
  const double num = PQ_C1 + PQ_C2 * ym, den = 1.0 + PQ_C3 * ym;
  const double dbase = (PQ_C2 * den - PQ_C3 * num) / (den * den);
  return PQ_M2 * pow(num / den, PQ_M2 - 1.0) * dbase * (PQ_M1 * ym / y) / PQ_PEAK;
}

struct ZeroBounceSource {
  const CamBatch* cams;
  int64_t hw;
  SbParams sp;
  float* rgb;
  int64_t item;

  __device__ __forceinline__ void operator()(uint32_t, double, double, double, double, D3, D3) const {}

  __device__ __forceinline__ bool start(int64_t wid, TraceCtx&, D3& O, D3& W) {
    item = wid;
    const CamDev& c = cams->c[wid / hw];
    O = d3(c.eye[0], c.eye[1], c.eye[2]);
    W = pixel_dir(c, (uint32_t)(wid % hw), 0, sp.flags, sp.k0, sp.k1);
    return true;
  }

  __device__ __forceinline__ bool finish(const Seg<false>& s, D3&, D3&) {
    rgb[item * 3 + 0] = s.R0;
    rgb[item * 3 + 1] = s.R1;
    rgb[item * 3 + 2] = s.R2;
    return false;
  }
};

__global__ void __launch_bounds__(TRACE_BLOCK) k_zero_bounce(TraceCtx tc, const CamBatch cams, int64_t hw,
                                                            int32_t n_cams, SbParams sp, float* rgb,
                                                            unsigned long long* work, uint64_t* hitlist) {
  ZeroBounceSource src;
  src.cams = &cams;
  src.hw = hw;
  src.sp = sp;
  src.rgb = rgb;
  src.item = 0;
  run_segments<Q_RADIANCE, false>(tc, src, work, hw * n_cams, hitlist, nullptr);
}

struct RadianceAdjSource {
  const Record* recs;
  const CamBatch* cams;
  int64_t hw;
  SbParams sp;
  const float* dL;
  double* gr;          // [3][n] double accumulators
  int64_t n;
  V3 dl;

  __device__ __forceinline__ bool start(int64_t wid, TraceCtx&, D3& O, D3& W) {
    dl = v3(dL[wid * 3 + 0], dL[wid * 3 + 1], dL[wid * 3 + 2]);
    if (dl.x == 0.0f && dl.y == 0.0f && dl.z == 0.0f) return false;   // nothing to add
    const CamDev& c = cams->c[wid / hw];
    O = d3(c.eye[0], c.eye[1], c.eye[2]);
    W = pixel_dir(c, (uint32_t)(wid % hw), 0, sp.flags, sp.k0, sp.k1);
    return true;
  }

  __device__ __forceinline__ void operator()(uint32_t pos, double, double, double w, double, D3, D3) {
    const uint32_t idx = rec_index(load_record(recs, pos));
    atomicAdd(gr + idx, w * (double)dl.x);
    atomicAdd(gr + n + idx, w * (double)dl.y);
    atomicAdd(gr + 2 * n + idx, w * (double)dl.z);
  }

  __device__ __forceinline__ bool finish(const Seg<false>&, D3&, D3&) { return false; }
};

__global__ void __launch_bounds__(TRACE_BLOCK) k_zero_bounce_adj_r(TraceCtx tc, const CamBatch cams, int64_t hw,
                                                                  int32_t n_cams, SbParams sp, const float* dL,
                                                                  double* gr, int64_t n, unsigned long long* work,
                                                                  uint64_t* hitlist) {
  RadianceAdjSource src;
  src.recs = tc.recs;
  src.cams = &cams;
  src.hw = hw;
  src.sp = sp;
  src.dL = dL;
  src.gr = gr;
  src.n = n;
  src.dl = v3(0.f, 0.f, 0.f);
  run_segments<Q_RADIANCE, false>(tc, src, work, hw * n_cams, hitlist, nullptr);
}

__global__ void __launch_bounds__(256) k_bake_loss(const float* rgb, const float* target, int64_t m, double inv_count,
                                                  float* dL, double* loss) {
  __shared__ double part[256 / 64];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double a = 0.0;
  if (i < m) {
    const double l0 = rgb[i];
    const double d = pq_curve(l0) - pq_curve((double)target[i]);
    a = fabs(d);
    const double sg = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
    dL[i] = (float)(sg * pq_slope(l0) * inv_count);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, (part[0] + part[1] + part[2] + part[3]) * inv_count);
}

template <class G>
__global__ void k_adam(float* r, const G* g, float* m, float* v, int64_t count, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = (float)g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  // c1 = 1 - b1^step, c2 = 1 - b2^step
  const float step = lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  r[i] = fmaxf(r[i] - step, 0.0f);
}

__global__ void k_add_grad(const double* acc, int64_t count, float* g) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) g[i] += (float)acc[i];
}

__global__ void k_zero_f64_b(double* p, int64_t count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

unsigned blocks_for(int64_t count) { return (unsigned)((count + 255) / 256); }

}  // namespace

void launch_zero_bounce(const TraceCtx& tc, const CamBatch& cams, int64_t hw, int32_t n_cams, const SbParams& sp,
                        float* rgb, unsigned long long* work, uint64_t* hitlist, hipStream_t st) {
  launch_zero_u64(work, 1, st);
  hipLaunchKernelGGL(k_zero_bounce, dim3((unsigned)(runner_lanes() / TRACE_BLOCK)), dim3(TRACE_BLOCK), 0, st, tc,
                     cams, hw, n_cams, sp, rgb, work, hitlist);
  check_hip(hipGetLastError(), "zero-bounce launch");
}

void launch_zero_bounce_adj_r(const TraceCtx& tc, const CamBatch& cams, int64_t hw, int32_t n_cams,
                              const SbParams& sp, const float* dL, double* gacc, int64_t n, unsigned long long* work,
                              uint64_t* hitlist, hipStream_t st) {
  launch_zero_u64(work, 1, st);
  hipLaunchKernelGGL(k_zero_bounce_adj_r, dim3((unsigned)(runner_lanes() / TRACE_BLOCK)), dim3(TRACE_BLOCK), 0, st,
                     tc, cams, hw, n_cams, sp, dL, gacc, n, work, hitlist);
  check_hip(hipGetLastError(), "zero-bounce adjoint launch");
}

void launch_zero_f64(double* p, int64_t count, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_zero_f64_b, dim3(blocks_for(count)), dim3(256), 0, st, p, count);
}

void launch_add_grad(const double* acc, int64_t count, float* g, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_add_grad, dim3(blocks_for(count)), dim3(256), 0, st, acc, count, g);
}

void launch_bake_loss(const float* rgb, const float* target, int64_t m, float* dL, double* loss, hipStream_t st) {
  launch_zero_f64(loss, 1, st);
  if (m > 0)
    hipLaunchKernelGGL(k_bake_loss, dim3(blocks_for(m)), dim3(256), 0, st, rgb, target, m, 1.0 / (double)m, dL, loss);
  check_hip(hipGetLastError(), "bake loss launch");
}

template <class G>
void launch_adam_t(float* r, const G* g, float* m, float* v, int64_t count, const eag_adam& a, int32_t step,
                   hipStream_t st) {
  const float c1 = (float)(1.0 - std::pow((double)a.beta1, step));
  const float c2 = (float)(1.0 - std::pow((double)a.beta2, step));
  if (count > 0)
    hipLaunchKernelGGL(k_adam<G>, dim3(blocks_for(count)), dim3(256), 0, st, r, g, m, v, count, a.lr, a.beta1,
                       a.beta2, a.eps, c1, c2);
  check_hip(hipGetLastError(), "adam launch");
}

void launch_adam(float* r, const double* g, float* m, float* v, int64_t count, const eag_adam& a, int32_t step,
                 hipStream_t st) {
  launch_adam_t(r, g, m, v, count, a, step, st);
}

void launch_adam(float* r, const float* g, float* m, float* v, int64_t count, const eag_adam& a, int32_t step,
                 hipStream_t st) {
  launch_adam_t(r, g, m, v, count, a, step, st);
}

}  // namespace eag
