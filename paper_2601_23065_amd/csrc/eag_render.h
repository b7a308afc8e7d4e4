// Launch interfaces of the single-bounce render and path-tracing kernels.
#pragma once

#include "eag_device.h"
#include "eag_internal.h"

namespace eag {

constexpr int MAX_CAMS_PER_LAUNCH = 8;
struct CamBatch {
  CamDev c[MAX_CAMS_PER_LAUNCH];
};

constexpr uint32_t JITTER_SEGMENT = 0xffffffffu;

// Camera ray through pixel `pix` (pixel centre, or a Philox jitter).
__device__ __forceinline__ D3 pixel_dir(const CamDev& c, uint32_t pix, uint32_t sample, uint32_t flags, uint32_t k0,
                                        uint32_t k1) {
  const int x = (int)(pix % (uint32_t)c.width), y = (int)(pix / (uint32_t)c.width);
  double ox = 0.5, oy = 0.5;
  if (flags & EAG_JITTER) {
    const uint4 w = philox(make_uint4(pix, sample, JITTER_SEGMENT, c.id), k0, k1);
    ox = to_unit(w.x);
    oy = to_unit(w.y);
  }
  return camera_dir(c, x, y, ox, oy);
}

// Per-pixel forward state of the single-bounce render (EAG_FWD_PIXEL_FLOATS
// floats), all in double except E and the branch: Nt, Dt, |N|, A place the
// bounce; R and P are the totals the adjoint subtracts running prefixes from.
struct FwdState {
  D3 Nt;
  double Dt, Nlen, A;
  D3 R, P;
  float E;
  float branch;   // 0 miss, 1 emitter, 2 reflect
};

__device__ __forceinline__ void store_state(float* p, const FwdState& s) {
  double* d = reinterpret_cast<double*>(p);
  d[0] = s.Nt.x; d[1] = s.Nt.y; d[2] = s.Nt.z;
  d[3] = s.Dt; d[4] = s.Nlen; d[5] = s.A;
  d[6] = s.R.x; d[7] = s.R.y; d[8] = s.R.z;
  d[9] = s.P.x; d[10] = s.P.y; d[11] = s.P.z;
  p[24] = s.E;
  p[25] = s.branch;
  p[26] = 0.0f;
  p[27] = 0.0f;
}

__device__ __forceinline__ FwdState load_state(const float* p) {
  const double* d = reinterpret_cast<const double*>(p);
  FwdState s;
  s.Nt = d3(d[0], d[1], d[2]);
  s.Dt = d[3]; s.Nlen = d[4]; s.A = d[5];
  s.R = d3(d[6], d[7], d[8]);
  s.P = d3(d[9], d[10], d[11]);
  s.E = p[24];
  s.branch = p[25];
  return s;
}

struct SbParams {
  int32_t spp;
  uint32_t flags;
  uint32_t k0, k1;           // Philox key
  float tau_E;
};

// work: a device counter; hitlist: runner_lanes() * HL_CAP keys.
void launch_single_bounce(const TraceCtx& tc, const CamBatch& cams, int64_t hw, int32_t n_cams,
                          const SbParams& sp, float* state, double* r1, float* rgb, unsigned long long* work,
                          uint64_t* hitlist, hipStream_t st);

// One request's share of a path-tracing launch. Work items of a request are
// numbered sample-major over 8x8 pixel tiles: item w has sample
// sample_begin + w / tile_pixels and tile slot w % tile_pixels. A launch
// covers items [work_begin, work_begin + count) of each slot; slots are laid
// end to end in the launch's own numbering (global_end = running total).
struct PtSlot {
  CamDev cam;
  int64_t* accum;            // int64 fixed point [H][W][3]
  const Attr* attrs;         // attribute records of the request's scene version
  int64_t work_begin;
  int64_t global_end;
  int64_t tile_pixels;       // tiles_x * tiles_y * 64
  uint32_t sample_begin;
  int32_t tiles_x;           // 8x8 pixel tiles across
  int32_t max_depth;
  int32_t rr_start;
  uint32_t flags;
  uint32_t k0, k1;
  float tau_E;
};

constexpr int PT_MAX_SLOTS = 8;
struct PtLaunch {
  PtSlot s[PT_MAX_SLOTS];
  int32_t n_slots;
  int64_t n_work;            // = s[n_slots - 1].global_end
};

// Lanes of the persistent runner grid on the current device (the hit list
// holds HL_CAP keys for each), and a launch that zeroes n counters.
int64_t runner_lanes();
void launch_zero_u64(unsigned long long* p, int n, hipStream_t st);
// hitlist: pt_lanes() * HL_CAP keys, or null to trace without the list.
void launch_path_trace(const TraceCtx& tc, const PtLaunch& L, unsigned long long* work_counter,
                       unsigned long long* counters, uint64_t* hitlist, hipStream_t st);

// Per-hit gradient records of the secondary adjoint (see eag_backward.hip):
// workspace buffers for the records of a camera batch.
constexpr int64_t GRAD_RECS_PER_ITEM = 20;          // records per (pixel, sample) item
constexpr int64_t GRAD_RECS_MAX = int64_t(1) << 27;   // at most 8 GiB of records
constexpr int64_t REC_CHUNK = 1024;                   // slots a wave claims at a time
struct GradRecs {
  float* rec;                   // [n_chunks * REC_CHUNK][16] accumulator rows of each hit
  uint32_t* idx;                // surfel index of each record
  uint32_t* cnt;                // [n] records per surfel
  uint32_t* cursor;             // [n] placement cursor per surfel
  uint32_t* off;                // [n] exclusive scan of cnt
  uint32_t* order;              // slots grouped by surfel
  uint32_t* chunk_used;         // [n_chunks] slots used in each chunk of REC_CHUNK slots
  unsigned long long* chunk_next;   // chunks claimed (set by the launch)
  int64_t n_chunks;             // records: n_chunks * REC_CHUNK
  void* scan_tmp;
  size_t scan_bytes;
};
int64_t grad_rec_capacity(int64_t n_items);
size_t grad_rec_scan_bytes(int64_t n);

void launch_single_bounce_backward(const TraceCtx& tc, const eag_surfels& s, const CamBatch& cams, int64_t hw,
                                   int32_t n_cams, const SbParams& sp, const float* state, const double* r1,
                                   const float* dL, double* gacc, float* scratch, const GradRecs& grecs,
                                   unsigned long long* work, uint64_t* hitlist, hipStream_t st);
// The camera segment of every pixel (forward state and emitter-branch colour).
void launch_camera_pass(const TraceCtx& tc, const CamBatch& cams, int64_t hw, int32_t n_cams, const SbParams& sp,
                        float* state, float* rgb, unsigned long long* work, uint64_t* hitlist, hipStream_t st);

// Stage 0 (eag_stage0.hip, eag_backward.hip). images: [pixels][8] = Nt, Dt, R, E.
constexpr int STAGE0_FLOATS = 8;
void launch_stage0_images(const float* state, int64_t n_pix, float* images, hipStream_t st);
// counts: 3 device counters (hit pixels, pixels valid for the distance normal, all pixels), set by the count
// launch, which also zeroes loss; contrib: [pixels][4] floats; a loss batch covers pixels [g0, g0 + nb) of one
// camera batch; the gather then completes dimg's Dt.
void launch_stage0_count(const float* images, int64_t n_pix, int64_t W, int64_t H, unsigned long long* counts,
                         double* loss, hipStream_t st);
void launch_stage0_loss_batch(const float* images, const float* rgb_gt, const float* n_mono, const float* mask,
                              const CamBatch& cams, int64_t g0, int64_t nb, int64_t W, int64_t H, const SbParams& sp,
                              const double w[4], const unsigned long long* counts, float* contrib, float* dimg,
                              double* loss, hipStream_t st);
void launch_stage0_gather(const float* contrib, int64_t n_pix, int64_t W, int64_t H, float* dimg, hipStream_t st);
void launch_stage0_backward(const TraceCtx& tc, const eag_surfels& s, const CamBatch& cams, int64_t hw,
                            int32_t n_cams, const SbParams& sp, const float* state, const float* dimg, double* gacc,
                            const GradRecs& grecs, unsigned long long* work, uint64_t* hitlist, hipStream_t st);
void launch_stage0_finalize(const double* gacc, int64_t n, const eag_surfel_grads& g, float* grad_emissive,
                            hipStream_t st);

// Geometric edits (eag_geom.hip).
size_t select_scan_bytes(int64_t n);
void launch_select_box(const float* pos, int64_t n, const float lo[3], const float hi[3], uint32_t* flags,
                       uint32_t* scan, void* tmp, size_t tmp_bytes, int32_t* idx, int64_t* count, hipStream_t st);
void launch_move(float* pos, float* rot, int64_t n, const int32_t* idx, int64_t count, const float r[4],
                 const float pivot[3], const float t[3], hipStream_t st);
void launch_delete(float* opacity, int64_t n, const int32_t* idx, int64_t count, hipStream_t st);
void launch_append(const eag_surfels& src, const int32_t* idx, int64_t count, const eag_surfels_out& dst,
                   const float r[4], const float pivot[3], const float t[3], hipStream_t st);
void launch_sah_cost(const Node4* nodes, const BvhHeader* h, int64_t max_nodes, int32_t root, double* acc,
                     double* cost, hipStream_t st);

// Light baking (eag_bake.hip).
void launch_zero_bounce(const TraceCtx& tc, const CamBatch& cams, int64_t hw, int32_t n_cams, const SbParams& sp,
                        float* rgb, unsigned long long* work, uint64_t* hitlist, hipStream_t st);
void launch_zero_bounce_adj_r(const TraceCtx& tc, const CamBatch& cams, int64_t hw, int32_t n_cams,
                              const SbParams& sp, const float* dL, double* gacc, int64_t n, unsigned long long* work,
                              uint64_t* hitlist, hipStream_t st);
void launch_zero_f64(double* p, int64_t count, hipStream_t st);
void launch_add_grad(const double* acc, int64_t count, float* g, hipStream_t st);
void launch_bake_loss(const float* rgb, const float* target, int64_t m, float* dL, double* loss, hipStream_t st);
void launch_adam(float* r, const double* g, float* m, float* v, int64_t count, const eag_adam& a, int32_t step,
                 hipStream_t st);
void launch_adam(float* r, const float* g, float* m, float* v, int64_t count, const eag_adam& a, int32_t step,
                 hipStream_t st);

// Emitter sampling with multiple importance sampling (eag_nee.hip).
// An emitter's geometry for the light pdf, in the tree's leaf order: centre,
// frame (t_u, t_v, n from its normalised quaternion) and scales in double
// precision, and rho, the area density of the point sampler on its ellipse.
struct __align__(16) EmitGeo {
  double p[3], tu[3], tv[3], n[3];
  double su, sv, rho;
  int32_t cell, pad;         // the emitter's cell (selection by cells)
};
struct EmitterDev {
  const Node4* nodes;        // 4-wide tree over the emitters
  const EmitGeo* geo;        // [n] geometry by leaf position
  const double* rho;         // [n] area density of the point sampler on each emitter's ellipse
  const double* cdf;         // [n] inclusive prefix sums of the selection weights
  const float* pos;          // [3][n] compacted centres
  const float* rot;          // [4][n] compacted quaternions
  const float* scale;        // [2][n] compacted scales
  int64_t n;                 // emitters (0: no light samples, every weight 1)
  double W;                  // total selection weight
  double k, k2;              // k_sigma and its square
  int32_t root;
  int32_t n_cells;           // selection by cells: cells (0: selection by power)
  double cell;               // cell size (0: selection by power)
  const double* cdf_in;      // [n] prefix sums of the weights within each cell
  const double4* cells;      // [n_cells] centre and total weight
  const int32_t* begin;      // [n_cells + 1] first entry of each cell, then n
};
size_t emitters_mem_bytes(int64_t n);
size_t emitters_ws_bytes(int64_t n);
// queue: pdf_queue_bytes(queue_entries) bytes of device memory for the
// contributions that wait for their light pdf; a launch of P paths at max
// depth D needs pdf_queue_entries = P (D + 1).
constexpr uint32_t MIS_CHUNK_SPP = 4;   // samples per launch of eag_path_trace_mis
size_t pdf_queue_bytes(int64_t entries);
int64_t pdf_queue_entries(int64_t pixels, int32_t max_depth, uint32_t chunk);
void launch_path_trace_mis(const TraceCtx& tc, const PtLaunch& L, const EmitterDev& E, void* queue,
                           int64_t queue_entries, unsigned long long* work_counter, unsigned long long* counters,
                           uint64_t* hitlist, hipStream_t st);

size_t grad_accum_doubles(int64_t n);
void launch_grad_zero(double* gacc, int64_t n, hipStream_t st);
void launch_grad_finalize(const double* gacc, int64_t n, const eag_surfel_grads& g, hipStream_t st);
void launch_apply_edit(const eag_edit& e, const eag_surfel_attrs& a, hipStream_t st);
void launch_accum_resolve(const int64_t* accum, int64_t n_values, double scale, float* rgb, hipStream_t st);

}  // namespace eag

// Host handle of an emitter table (device storage in caller memory).
struct eag_emitters {
  eag::EmitterDev dev;
  eag_bvh* bvh;              // tree over the emitters (null when there are none)
  int64_t n_src;             // surfels of the scene it was built from
  float tau_E, k_sigma;      // the parameters it was built for
  float cell;                // cell size of the selection (0: by power)
};

namespace eag {
void build_emitters(const eag_surfels* s, float tau_E, float k_sigma, float cell, void* mem, size_t mem_bytes,
                    void* ws, size_t ws_bytes, hipStream_t st, eag_emitters* out);
}  // namespace eag
