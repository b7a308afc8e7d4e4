// Single-bounce emission-aware render (Sec. 3.3, Eq. 5-7), forward pass.
//
// k_sb_camera     one work item per pixel on the persistent segment runner:
//                 camera segment, branch (miss / emit / reflect), forward
//                 state.
// k_sb_secondary  one work item per (pixel, sample) on the persistent
//                 segment runner: cosine-sampled direction about Nt from
//                 X = O + Dt w, secondary segment blending r only (the
//                 radiance cache), R1 per sample.
// k_sb_resolve    one thread per pixel: L = P * mean_s R1 (fixed summation
//                 order, so the image does not depend on scheduling).
#include "eag_device.h"
#include "eag_internal.h"
#include "eag_render.h"
#include "eag_runner.h"

namespace eag {

namespace {

// One camera segment per pixel: the forward state and the pixel's colour
// (emitter branch) or zero (the secondary pass and the resolve fill in the
// reflect branch).
struct CameraSource {
  const CamBatch* cams;
  int64_t hw;
  SbParams sp;
  float* state;
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

  __device__ __forceinline__ bool finish(const Seg<true>& s, D3&, D3&) {
    const double A = 1.0 - s.T;
    FwdState st;
    st.Nt = d3(0.0, 0.0, 0.0);
    st.Dt = 0.0;
    st.Nlen = 0.0;
    st.A = 0.0;
    st.branch = 0.0f;
    V3 L = v3(0.f, 0.f, 0.f);
    if (s.nhits > 0 && A > 0.0) {
      const double nl = sqrt(dot(s.N, s.N));
      st.Nt = (1.0 / nl) * s.N;
      st.Dt = s.D / A;
      st.Nlen = nl;
      st.A = A;
      if ((float)s.E > sp.tau_E) {
        st.branch = 1.0f;
        L = v3((float)s.R0, (float)s.R1, (float)s.R2);
      } else {
        st.branch = 2.0f;
      }
    }
    st.R = d3(s.R0, s.R1, s.R2);
    st.E = (float)s.E;
    st.P = d3(s.P0, s.P1, s.P2);
    store_state(state + item * EAG_FWD_PIXEL_FLOATS, st);
    rgb[item * 3 + 0] = L.x;
    rgb[item * 3 + 1] = L.y;
    rgb[item * 3 + 2] = L.z;
    return false;
  }
};

__global__ void __launch_bounds__(TRACE_BLOCK) k_sb_camera(TraceCtx tc, const CamBatch cams, int64_t hw,
                                                           int32_t n_cams, SbParams sp, float* state, float* rgb,
                                                           unsigned long long* work, uint64_t* hitlist) {
  CameraSource src;
  src.cams = &cams;
  src.hw = hw;
  src.sp = sp;
  src.state = state;
  src.rgb = rgb;
  src.item = 0;
  run_segments<Q_ALL, true>(tc, src, work, hw * n_cams, hitlist, nullptr);
}

// One (pixel, sample) secondary segment per work item; a pixel whose camera
// segment did not take the reflect branch gets R1 = 0 without tracing.
struct SecondarySource {
  const CamBatch* cams;
  int64_t hw;
  int32_t S;
  SbParams sp;
  const float* state;
  double* r1;
  int64_t item;

  __device__ __forceinline__ bool start(int64_t wid, TraceCtx&, D3& O, D3& W) {
    item = wid;
    const int64_t g = wid / S;
    const uint32_t s = (uint32_t)(wid - g * S);
    const float* ps = state + g * EAG_FWD_PIXEL_FLOATS;
    if (ps[25] != 2.0f) {
      r1[wid * 3 + 0] = 0.0;
      r1[wid * 3 + 1] = 0.0;
      r1[wid * 3 + 2] = 0.0;
      return false;
    }
    const double* d = reinterpret_cast<const double*>(ps);
    const D3 Nt = d3(d[0], d[1], d[2]);
    const double Dt = d[3];
    const CamDev& c = cams->c[g / hw];
    const uint32_t pix = (uint32_t)(g % hw);
    const D3 Wc = pixel_dir(c, pix, 0, sp.flags, sp.k0, sp.k1);
    O = d3(c.eye[0] + Dt * Wc.x, c.eye[1] + Dt * Wc.y, c.eye[2] + Dt * Wc.z);
    const uint4 w = philox(make_uint4(pix, s, 0u, c.id), sp.k0, sp.k1);
    W = cosine_dir(Nt, to_unit(w.x), to_unit(w.y));
    return true;
  }

  __device__ __forceinline__ void operator()(uint32_t, double, double, double, double, D3, D3) const {}

  __device__ __forceinline__ bool finish(const Seg<true>& sg, D3&, D3&) {
    r1[item * 3 + 0] = sg.R0;
    r1[item * 3 + 1] = sg.R1;
    r1[item * 3 + 2] = sg.R2;
    return false;
  }
};

__global__ void __launch_bounds__(TRACE_BLOCK) k_sb_secondary(
    TraceCtx tc, const CamBatch cams, int64_t hw, int32_t n_cams, SbParams sp, const float* state, double* r1,
    unsigned long long* work, uint64_t* hitlist) {
  SecondarySource src;
  src.cams = &cams;
  src.hw = hw;
  src.S = sp.spp;
  src.sp = sp;
  src.state = state;
  src.r1 = r1;
  src.item = 0;
  run_segments<Q_RADIANCE, true>(tc, src, work, hw * n_cams * sp.spp, hitlist, nullptr);
}

__global__ void k_sb_resolve(int64_t n_pix, SbParams sp, const float* state, const double* r1, float* rgb) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n_pix) return;
  const FwdState st = load_state(state + g * EAG_FWD_PIXEL_FLOATS);
  if (st.branch != 2.0f) return;
  const int S = sp.spp;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int s = 0; s < S; ++s) {
    a += r1[(g * S + s) * 3 + 0];
    b += r1[(g * S + s) * 3 + 1];
    c += r1[(g * S + s) * 3 + 2];
  }
  const double inv = 1.0 / (double)S;
  rgb[g * 3 + 0] = (float)(st.P.x * (a * inv));
  rgb[g * 3 + 1] = (float)(st.P.y * (b * inv));
  rgb[g * 3 + 2] = (float)(st.P.z * (c * inv));
}

}  // namespace

void launch_camera_pass(const TraceCtx& tc, const CamBatch& cams, int64_t hw, int32_t n_cams, const SbParams& sp,
                        float* state, float* rgb, unsigned long long* work, uint64_t* hitlist, hipStream_t st) {
  launch_zero_u64(work, 1, st);
  hipLaunchKernelGGL(k_sb_camera, dim3((unsigned)(runner_lanes() / TRACE_BLOCK)), dim3(TRACE_BLOCK), 0, st, tc, cams,
                     hw, n_cams, sp, state, rgb, work, hitlist);
  check_hip(hipGetLastError(), "camera pass launch");
}

void launch_single_bounce(const TraceCtx& tc, const CamBatch& cams, int64_t hw, int32_t n_cams,
                          const SbParams& sp, float* state, double* r1, float* rgb, unsigned long long* work,
                          uint64_t* hitlist, hipStream_t st) {
  const int64_t np = hw * n_cams;
  const unsigned grid = (unsigned)(runner_lanes() / TRACE_BLOCK);
  launch_zero_u64(work, 1, st);
  hipLaunchKernelGGL(k_sb_camera, dim3(grid), dim3(TRACE_BLOCK), 0, st, tc, cams, hw, n_cams, sp, state, rgb, work,
                     hitlist);
  launch_zero_u64(work, 1, st);
  hipLaunchKernelGGL(k_sb_secondary, dim3((unsigned)(runner_lanes() / TRACE_BLOCK)), dim3(TRACE_BLOCK), 0, st, tc,
                     cams, hw, n_cams, sp, (const float*)state, r1, work, hitlist);
  hipLaunchKernelGGL(k_sb_resolve, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, np, sp,
                     (const float*)state, (const double*)r1, rgb);
  check_hip(hipGetLastError(), "single-bounce launch");
}

}  // namespace eag
