// Single-bounce emission-aware render (Sec. 3.3, Eq. 5-7), forward pass.
//
// k_sb_camera     one thread per pixel: camera segment, branch (miss / emit /
//                 reflect), forward state.
// k_sb_secondary  one thread per (pixel, sample): cosine-sampled direction
//                 about Nt from X = O + Dt w, secondary segment blending r
//                 only (the radiance cache), R1 per sample.
// k_sb_resolve    one thread per pixel: L = P * mean_s R1 (fixed summation
//                 order, so the image does not depend on scheduling).
#include "eag_device.h"
#include "eag_internal.h"
#include "eag_render.h"

namespace eag {

namespace {

constexpr uint32_t JITTER_SEGMENT = 0xffffffffu;

__device__ __forceinline__ V3 pixel_dir(const CamDev& c, uint32_t pix, uint32_t sample, uint32_t flags,
                                        uint32_t k0, uint32_t k1) {
  const int x = (int)(pix % (uint32_t)c.width), y = (int)(pix / (uint32_t)c.width);
  float ox = 0.5f, oy = 0.5f;
  if (flags & EAG_JITTER) {
    const uint4 w = philox(make_uint4(pix, sample, JITTER_SEGMENT, c.id), k0, k1);
    ox = to_unit(w.x);
    oy = to_unit(w.y);
  }
  return camera_dir(c, x, y, ox, oy);
}

__global__ void __launch_bounds__(256) k_sb_camera(TraceCtx tc, const CamBatch cams, int64_t hw, int32_t n_cams,
                                                   SbParams sp, float* state, float* rgb) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= hw * n_cams) return;
  const CamDev c = cams.c[g / hw];
  const uint32_t pix = (uint32_t)(g % hw);
  const V3 O = v3(c.eye[0], c.eye[1], c.eye[2]);
  const V3 W = pixel_dir(c, pix, 0, sp.flags, sp.k0, sp.k1);
  const SegOut s = trace_segment<Q_ALL>(tc, O, W);
  const float A = 1.0f - s.T;
  float st[EAG_FWD_PIXEL_FLOATS];
#pragma unroll
  for (int k = 0; k < EAG_FWD_PIXEL_FLOATS; ++k) st[k] = 0.0f;
  float branch = 0.0f;
  V3 L = v3(0.f, 0.f, 0.f);
  if (s.nhits > 0 && A > 0.0f) {
    const float nl = sqrtf(dot(s.N, s.N));
    const float il = 1.0f / nl;
    st[0] = s.N.x * il; st[1] = s.N.y * il; st[2] = s.N.z * il;
    st[3] = s.D / A;
    st[12] = nl;
    if (s.E > sp.tau_E) {
      branch = 1.0f;
      L = s.R;
    } else {
      branch = 2.0f;
    }
  }
  st[4] = s.R.x; st[5] = s.R.y; st[6] = s.R.z;
  st[7] = s.E;
  st[8] = s.P.x; st[9] = s.P.y; st[10] = s.P.z;
  st[11] = A;
  st[13] = branch;
  float4* sp4 = reinterpret_cast<float4*>(state + g * EAG_FWD_PIXEL_FLOATS);
#pragma unroll
  for (int k = 0; k < EAG_FWD_PIXEL_FLOATS / 4; ++k) sp4[k] = make_float4(st[4 * k], st[4 * k + 1], st[4 * k + 2], st[4 * k + 3]);
  rgb[g * 3 + 0] = L.x;
  rgb[g * 3 + 1] = L.y;
  rgb[g * 3 + 2] = L.z;
}

__global__ void __launch_bounds__(256) k_sb_secondary(TraceCtx tc, const CamBatch cams, int64_t hw, int32_t n_cams,
                                                      SbParams sp, const float* state, float* r1) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t S = sp.spp;
  if (t >= hw * n_cams * S) return;
  const int64_t g = t / S;
  const uint32_t s = (uint32_t)(t % S);
  const float* st = state + g * EAG_FWD_PIXEL_FLOATS;
  V3 R = v3(0.f, 0.f, 0.f);
  if (st[13] == 2.0f) {
    const CamDev c = cams.c[g / hw];
    const uint32_t pix = (uint32_t)(g % hw);
    const V3 W = pixel_dir(c, pix, 0, sp.flags, sp.k0, sp.k1);
    const float Dt = st[3];
    const V3 X = v3(c.eye[0] + Dt * W.x, c.eye[1] + Dt * W.y, c.eye[2] + Dt * W.z);
    const uint4 w = philox(make_uint4(pix, s, 0u, c.id), sp.k0, sp.k1);
    const V3 Wd = cosine_dir(v3(st[0], st[1], st[2]), to_unit(w.x), to_unit(w.y));
    R = trace_segment<Q_RADIANCE>(tc, X, Wd).R;
  }
  r1[t * 3 + 0] = R.x;
  r1[t * 3 + 1] = R.y;
  r1[t * 3 + 2] = R.z;
}

__global__ void k_sb_resolve(int64_t n_pix, SbParams sp, const float* state, const float* r1, float* rgb) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n_pix) return;
  const float* st = state + g * EAG_FWD_PIXEL_FLOATS;
  if (st[13] != 2.0f) return;
  const int S = sp.spp;
  float a = 0.f, b = 0.f, c = 0.f;
  for (int s = 0; s < S; ++s) {
    a += r1[(g * S + s) * 3 + 0];
    b += r1[(g * S + s) * 3 + 1];
    c += r1[(g * S + s) * 3 + 2];
  }
  const float inv = 1.0f / (float)S;
  rgb[g * 3 + 0] = st[8] * (a * inv);
  rgb[g * 3 + 1] = st[9] * (b * inv);
  rgb[g * 3 + 2] = st[10] * (c * inv);
}

}  // namespace

void launch_single_bounce(const TraceCtx& tc, const CamBatch& cams, int64_t hw, int32_t n_cams,
                          const SbParams& sp, float* state, float* r1, float* rgb, hipStream_t st) {
  const int64_t np = hw * n_cams;
  hipLaunchKernelGGL(k_sb_camera, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, tc, cams, hw, n_cams,
                     sp, state, rgb);
  const int64_t ns = np * sp.spp;
  hipLaunchKernelGGL(k_sb_secondary, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, tc, cams, hw,
                     n_cams, sp, (const float*)state, r1);
  hipLaunchKernelGGL(k_sb_resolve, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, np, sp,
                     (const float*)state, (const float*)r1, rgb);
  check_hip(hipGetLastError(), "single-bounce launch");
}

}  // namespace eag
