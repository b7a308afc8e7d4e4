// Multi-bounce diffuse path tracing (Sec. 3.4, Eq. 9) as a persistent
// wavefront kernel.
//
// Each lane of a wave64 carries one path and runs it as a small state
// machine over the steps of a segment (eag_device.h): start a k-buffer
// round, traverse, blend the round's hits, shade. Lanes advance
// independently, so a lane whose segment needs one round does not wait for
// a neighbour that needs four:
//   * idle lanes are refilled from a global work counter (the wave ballots
//     its idle lanes, one lane claims that many work items with a single
//     atomic, and each idle lane takes base + its rank among them);
//   * lanes whose round needs the BVH traverse together; the wave leaves
//     the traversal loop once PT_BLEND_BATCH lanes wait to blend (or no lane
//     traverses), blends and shades those lanes, starts their next rounds or
//     segments, and resumes: traversal state stays in registers and LDS.
// Shading a finished segment: miss -> path ends; E > tau_E -> add beta * R,
// path ends; depth == max_depth -> discarded; otherwise beta *= P, a
// cosine-weighted direction about Nt is drawn with Philox counter (pixel,
// sample, depth, camera id), the path moves to X = O + Dt w, and Russian
// roulette (q = min(0.95, max beta), survive iff u2 < q, beta /= q) applies
// once the new depth reaches rr_start.
// A wave exits when the work counter is exhausted and all its lanes are
// idle. One launch can serve several requests (slots), each with its own
// camera, parameters, accumulator and scene version; the server uses this to
// batch requests that are live at the same time.
//
// Work items are sample-major over 8x8 pixel tiles, so a wave's first
// segments are spatially coherent. Contributions are added to int64 fixed
// point accumulators, which makes every pixel sum independent of the order
// in which lanes finish.
#include "eag_device.h"
#include "eag_internal.h"
#include "eag_render.h"

namespace eag {

namespace {

constexpr int PT_BLEND_BATCH = 20;   // lanes waiting to blend that end a traversal stretch

enum { ST_IDLE = 0, ST_ROUND = 1, ST_TRAV = 2, ST_BLEND = 3 };

__device__ __forceinline__ void add_fixed(int64_t* acc, float v) {
  if (v != 0.0f) {
    const long long q = (long long)rint((double)v * EAG_ACCUM_SCALE);
    atomicAdd(reinterpret_cast<unsigned long long*>(acc), (unsigned long long)q);
  }
}

__global__ void __launch_bounds__(TRACE_BLOCK) k_path_trace(TraceCtx tc, PtLaunch L,
                                                            unsigned long long* work_counter,
                                                            unsigned long long* counters, uint64_t* hitlist) {
  __shared__ int s_stack[STACK_LDS * TRACE_BLOCK];
  __shared__ int s_pend[PEND * TRACE_BLOCK];
  int s_ovf[STACK_OVF];
  TravStack st;
  st.lds = s_stack + threadIdx.x;
  st.ovf = s_ovf;
  st.sp = 0;
  int* const pend = s_pend + threadIdx.x;
  const int lane = (int)(threadIdx.x & 63);
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  TraceCtx tcl = tc;
  tcl.hl = hitlist ? hitlist + ((int64_t)blockIdx.x * TRACE_BLOCK + threadIdx.x) * HL_CAP : nullptr;

  int stage = ST_IDLE;
  int slot = 0;
  uint32_t pix = 0, sample = 0;
  int depth = 0;
  V3 beta = v3(1.f, 1.f, 1.f);
  Seg<false> s;
  seg_begin(s, d3(0.0, 0.0, 0.0), d3(0.0, 0.0, 1.0));
  Round r;
  r.cnt = 0;
  r.trav = false;
  r.np = 0;
  unsigned long long n_segments = 0, n_rounds = 0, n_tests = 0, n_paths = 0, n_hits = 0, n_visits = 0;

  while (true) {
    // ---- refill idle lanes from the global work counter
    const bool need = stage == ST_IDLE;
    const uint64_t idle = __ballot(need);
    bool exhausted = false;
    if (idle) {
      const int leader = __ffsll((unsigned long long)idle) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(work_counter, (unsigned long long)__popcll(idle));
      base = __shfl(base, leader);
      exhausted = base + (unsigned long long)__popcll(idle) >= (unsigned long long)L.n_work;
      if (need) {
        const int64_t wid = (int64_t)base + __popcll(idle & lt_mask);
        if (wid < L.n_work) {
          int k = 0;
          while (k < L.n_slots - 1 && wid >= L.s[k].global_end) ++k;
          const PtSlot& S = L.s[k];
          const int64_t item = S.work_begin + (wid - (k ? L.s[k - 1].global_end : 0));
          const int64_t s_rel = item / S.tile_pixels;
          const int64_t tp = item - s_rel * S.tile_pixels;
          const int64_t tile = tp >> 6;
          const int within = (int)(tp & 63);
          const int x = (int)(tile % S.tiles_x) * 8 + (within & 7);
          const int y = (int)(tile / S.tiles_x) * 8 + (within >> 3);
          if (x < S.cam.width && y < S.cam.height) {
            slot = k;
            pix = (uint32_t)(y * S.cam.width + x);
            sample = S.sample_begin + (uint32_t)s_rel;
            beta = v3(1.f, 1.f, 1.f);
            depth = 0;
            tcl.attrs = S.attrs;
            seg_begin(s, d3(S.cam.eye[0], S.cam.eye[1], S.cam.eye[2]),
                      pixel_dir(S.cam, pix, sample, S.flags, S.k0, S.k1));
            stage = ST_ROUND;
            ++n_paths;
            ++n_segments;
          }
        }
      }
    }
    // Every lane idle: stop once the counter is exhausted, else claim again
    // (a claim can hold only pixels outside the image).
    if (__ballot(stage != ST_IDLE) == 0) {
      if (exhausted) break;
      continue;
    }

    // ---- start rounds
    if (stage == ST_ROUND) stage = round_begin(tcl, s, r, st, pend) ? ST_TRAV : ST_BLEND;

    // ---- traverse until enough lanes wait to blend
    while (true) {
      if (stage == ST_TRAV) {
        while (r.trav && r.np <= PEND - 4) {
          node_visit(tcl, s, r, st, pend);
          if (__all(r.np > 0 || !r.trav)) break;
        }
        leaf_phase(tcl, s, r, pend);
        if (!r.trav) {
          round_end_traversal(tcl, s, r);
          stage = ST_BLEND;
        }
      }
      if (__ballot(stage == ST_TRAV) == 0 || __popcll(__ballot(stage == ST_BLEND)) >= PT_BLEND_BATCH) break;
    }

    // ---- blend, and shade finished segments
    if (stage != ST_BLEND) continue;
    NoHit nh;
    blend_round<Q_ALL>(tcl, s, r, nh, nullptr, 0);
    if (!s.done) {
      stage = ST_ROUND;
      continue;
    }
    n_rounds += s.rounds;
    n_tests += s.tests;
    n_hits += s.nhits;
    n_visits += s.visits;
    stage = ST_IDLE;
    const PtSlot& S = L.s[slot];
    const double A = 1.0 - s.T;
    if (s.nhits == 0 || !(A > 0.0)) continue;
    const bool emit = s.E > S.tau_E;
    if ((S.flags & EAG_ADDITIVE_EMISSION) || emit) {
      int64_t* acc = S.accum + (int64_t)pix * 3;
      add_fixed(acc + 0, beta.x * s.R0);
      add_fixed(acc + 1, beta.y * s.R1);
      add_fixed(acc + 2, beta.z * s.R2);
      if (!(S.flags & EAG_ADDITIVE_EMISSION)) continue;
    }
    if (depth >= S.max_depth) continue;
    beta = v3(beta.x * s.P0, beta.y * s.P1, beta.z * s.P2);
    const uint4 w = philox(make_uint4(pix, sample, (uint32_t)depth, S.cam.id), S.k0, S.k1);
    ++depth;
    if (S.rr_start > 0 && depth >= S.rr_start) {
      const float q = fminf(0.95f, fmaxf(fmaxf(beta.x, beta.y), beta.z));
      if (!(to_unit(w.z) < q)) continue;
      const float iq = 1.0f / q;
      beta = v3(beta.x * iq, beta.y * iq, beta.z * iq);
    }
    const D3 Nt = (1.0 / sqrt(dot(s.N, s.N))) * s.N;
    const double Dt = s.D / A;
    const D3 X = d3(s.O.x + Dt * s.W.x, s.O.y + Dt * s.W.y, s.O.z + Dt * s.W.z);
    seg_begin(s, X, cosine_dir(Nt, to_unit(w.x), to_unit(w.y)));
    stage = ST_ROUND;
    ++n_segments;
  }
  if (counters) {
    atomicAdd(&counters[0], n_segments);
    atomicAdd(&counters[1], n_paths);
    atomicAdd(&counters[2], n_rounds);
    atomicAdd(&counters[3], n_tests);
    atomicAdd(&counters[4], n_hits);
    atomicAdd(&counters[5], n_visits);
  }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

__global__ void k_resolve(const int64_t* accum, int64_t n, double scale, float* rgb) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) rgb[i] = (float)((double)accum[i] * scale);
}

}  // namespace

int64_t pt_lanes() {
  int dev = 0, cus = 0, per_cu = 0;
  check_hip(hipGetDevice(&dev), "hipGetDevice");
  check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
  check_hip(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_path_trace),
                                                        TRACE_BLOCK, 0),
            "occupancy");
  if (per_cu < 1) per_cu = 1;
  return (int64_t)cus * per_cu * TRACE_BLOCK;
}

void launch_path_trace(const TraceCtx& tc, const PtLaunch& L, unsigned long long* work_counter,
                       unsigned long long* counters, uint64_t* hitlist, hipStream_t st) {
  // one resident block per TRACE_BLOCK lanes: the hit list is sized for exactly this grid
  const unsigned blocks = (unsigned)(pt_lanes() / TRACE_BLOCK);
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
