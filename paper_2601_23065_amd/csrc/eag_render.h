// Launch interfaces of the single-bounce render and path-tracing kernels.
#pragma once

#include "eag_device.h"
#include "eag_internal.h"

namespace eag {

constexpr int MAX_CAMS_PER_LAUNCH = 8;
struct CamBatch {
  CamDev c[MAX_CAMS_PER_LAUNCH];
};

struct SbParams {
  int32_t spp;
  uint32_t flags;
  uint32_t k0, k1;           // Philox key
  float tau_E;
};

void launch_single_bounce(const TraceCtx& tc, const CamBatch& cams, int64_t hw, int32_t n_cams,
                          const SbParams& sp, float* state, float* r1, float* rgb, hipStream_t st);

struct PtParams {
  int32_t max_depth;
  int32_t rr_start;
  uint32_t flags;
  uint32_t k0, k1;
  float tau_E;
  uint32_t sample_begin;
  uint32_t sample_count;
  int32_t tiles_x;           // 8x8 pixel tiles across
  int64_t tile_pixels;       // tiles_x * tiles_y * 64
};

void launch_path_trace(const TraceCtx& tc, const CamDev& cam, const PtParams& pp, int64_t* accum,
                       unsigned long long* work_counter, unsigned long long* counters, hipStream_t st);
void launch_single_bounce_backward(const TraceCtx& tc, const eag_surfels& s, const CamBatch& cams, int64_t hw,
                                   int32_t n_cams, const SbParams& sp, const float* state, const float* r1,
                                   const float* dL, const eag_surfel_grads& g, float* scratch, hipStream_t st);
void launch_apply_edit(const eag_edit& e, const eag_surfel_attrs& a, hipStream_t st);
void launch_accum_resolve(const int64_t* accum, int64_t n_values, double scale, float* rgb, hipStream_t st);

}  // namespace eag
