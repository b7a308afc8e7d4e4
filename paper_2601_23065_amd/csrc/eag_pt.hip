// Multi-bounce diffuse path tracing (Sec. 3.4, Eq. 9) as a persistent
// wavefront kernel.
//
// Each wave64 keeps one path per lane. Every iteration, lanes whose path has
// ended are refilled from a global work counter: the wave ballots its idle
// lanes, one lane claims that many work items with a single atomic, and each
// idle lane takes base + (its rank among the idle lanes). Every live lane
// then traces one segment and shades it: miss -> path ends; E > tau_E ->
// add beta * R, path ends; depth == max_depth -> discarded; otherwise
// beta *= P, a cosine-weighted direction about Nt is drawn with Philox
// counter (pixel, sample, depth, camera id), the path moves to
// X = O + Dt w, and Russian roulette (q = min(0.95, max beta), survive iff
// u2 < q, beta /= q) applies once the new depth reaches rr_start.
// A wave exits when the counter is exhausted and all its lanes are idle.
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

namespace eag {

namespace {

__device__ __forceinline__ void add_fixed(int64_t* acc, float v) {
  if (v != 0.0f) {
    const long long q = (long long)rint((double)v * EAG_ACCUM_SCALE);
    atomicAdd(reinterpret_cast<unsigned long long*>(acc), (unsigned long long)q);
  }
}

__global__ void __launch_bounds__(256) k_path_trace(TraceCtx tc, PtLaunch L, unsigned long long* work_counter,
                                                    unsigned long long* counters, uint64_t* hitlist) {
  const int lane = (int)(threadIdx.x & 63);
  uint64_t* const hl =
      hitlist ? hitlist + ((int64_t)blockIdx.x * (TRACE_BLOCK / 64) + (threadIdx.x >> 6)) * (HL_CAP * HL_STRIDE) + lane
              : nullptr;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  bool alive = false;
  int slot = 0;
  uint32_t pix = 0, sample = 0;
  int depth = 0;
  D3 O = d3(0.0, 0.0, 0.0), Wd = d3(0.0, 0.0, 1.0);
  V3 beta = v3(1.f, 1.f, 1.f);
  unsigned long long n_rounds = 0, n_tests = 0, n_paths = 0, n_hits = 0, n_visits = 0;

  while (true) {
    // ---- refill idle lanes from the global work counter
    const bool need = !alive;
    const uint64_t idle = __ballot(need);
    if (idle) {
      const int leader = __ffsll((unsigned long long)idle) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(work_counter, (unsigned long long)__popcll(idle));
      base = __shfl(base, leader);
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
            O = d3(S.cam.eye[0], S.cam.eye[1], S.cam.eye[2]);
            Wd = pixel_dir(S.cam, pix, sample, S.flags, S.k0, S.k1);
            beta = v3(1.f, 1.f, 1.f);
            depth = 0;
            alive = true;
            ++n_paths;
          }
        }
      }
    }
    const uint64_t live = __ballot(alive);
    // All lanes idle after a refill means this wave claimed 64 consecutive
    // work items without a valid one. Every tile holds a valid pixel at its
    // first slot, so 64 consecutive items always contain one unless they lie
    // past the end: the counter is exhausted and the wave is done.
    if (live == 0) break;
    if (lane == __ffsll((unsigned long long)live) - 1 && counters)
      atomicAdd(&counters[0], (unsigned long long)__popcll(live));
    if (!alive) continue;

    // ---- one segment, through the attributes of this path's scene version
    const PtSlot& S = L.s[slot];
    TraceCtx tcl = tc;
    tcl.attrs = S.attrs;
    tcl.hl = hl;
    const SegOut s = trace_segment<Q_ALL>(tcl, O, Wd);
    n_rounds += s.rounds;
    n_tests += s.tests;
    n_hits += s.nhits;
    n_visits += s.visits;
    const double A = 1.0 - s.T;
    if (s.nhits == 0 || !(A > 0.0)) {
      alive = false;
      continue;
    }
    const bool emit = (float)s.E > S.tau_E;
    if ((S.flags & EAG_ADDITIVE_EMISSION) || emit) {
      int64_t* acc = S.accum + (int64_t)pix * 3;
      add_fixed(acc + 0, beta.x * (float)s.R.x);
      add_fixed(acc + 1, beta.y * (float)s.R.y);
      add_fixed(acc + 2, beta.z * (float)s.R.z);
      if (!(S.flags & EAG_ADDITIVE_EMISSION)) {
        alive = false;
        continue;
      }
    }
    if (depth >= S.max_depth) {
      alive = false;
      continue;
    }
    beta = v3(beta.x * (float)s.P.x, beta.y * (float)s.P.y, beta.z * (float)s.P.z);
    const uint4 w = philox(make_uint4(pix, sample, (uint32_t)depth, S.cam.id), S.k0, S.k1);
    const D3 Nt = (1.0 / sqrt(dot(s.N, s.N))) * s.N;
    const double Dt = s.D / A;
    O = d3(O.x + Dt * Wd.x, O.y + Dt * Wd.y, O.z + Dt * Wd.z);
    Wd = cosine_dir(Nt, to_unit(w.x), to_unit(w.y));
    ++depth;
    if (S.rr_start > 0 && depth >= S.rr_start) {
      const float q = fminf(0.95f, fmaxf(fmaxf(beta.x, beta.y), beta.z));
      if (!(to_unit(w.z) < q)) {
        alive = false;
        continue;
      }
      const float iq = 1.0f / q;
      beta = v3(beta.x * iq, beta.y * iq, beta.z * iq);
    }
  }
  if (counters) {
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
