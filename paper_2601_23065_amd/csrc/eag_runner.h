// Persistent segment runner: the per-lane state machine that drives the
// segment engine (eag_device.h) over a stream of work items.
//
// Each lane of a wave64 carries one work item and runs its segments as a
// small state machine over the engine's steps: start a k-buffer round,
// traverse, blend the round's hits, finish the segment. Lanes advance
// independently, so a lane whose segment needs one round does not wait for a
// neighbour that needs four:
//   * idle lanes are refilled from a global work counter (the wave ballots
//     its idle lanes, one lane claims that many work items with a single
//     atomic, and each idle lane takes base + its rank among them);
//   * lanes whose round needs the BVH traverse together; the wave leaves the
//     traversal loop once RUN_BLEND_BATCH lanes wait to blend (or no lane
//     traverses), blends those lanes' rounds, finishes their segments, starts
//     their next rounds or segments, and resumes: traversal state stays in
//     registers and LDS.
// A wave exits when the work counter is exhausted and all its lanes are
// idle.
//
// The work comes from a source object, one per lane:
//   bool start(int64_t item, TraceCtx& tcl, D3& O, D3& W)
//       set up work item `item` (0 <= item < n_work); true with the first
//       segment's ray in (O, W) (and tcl.attrs set), false when the item
//       needs no tracing (the source then writes its own result);
//   bool finish(const Seg<DACC>& s, D3& O, D3& W)
//       the lane's segment has ended; true with the next segment's ray;
//   void operator()(uint32_t pos, double t, double alpha, double w,
//                   double T_before, D3 O, D3 W)
//       called for every blended hit, in blending order (may be empty).
#pragma once

#include "eag_device.h"

namespace eag {

constexpr int RUN_BLEND_BATCH = 20;   // lanes waiting to blend that end a traversal stretch
// Runner kernels launch this many TRACE_BLOCK-thread blocks per CU: their
// LDS (stack and postponed leaves, 56 KB per block) admits two per CU, and
// the per-lane hit list is sized for exactly this grid.
constexpr int RUN_BLOCKS_PER_CU = 2;

// Per-lane statistics, added to a device array of 6 counters at the end:
// segments, items started, k-buffer rounds, candidate tests, blended hits,
// BVH nodes visited. Kept in 32 bits (registers are the runner's limit): a
// lane would need over 10^7 segments in one launch (about 10^12 segments
// over the grid, hours of tracing) to overflow one.
struct RunStats {
  uint32_t segments = 0, items = 0, rounds = 0, tests = 0, hits = 0, visits = 0;
  __device__ __forceinline__ void flush(unsigned long long* c) {
    atomicAdd(&c[0], (unsigned long long)segments);
    atomicAdd(&c[1], (unsigned long long)items);
    atomicAdd(&c[2], (unsigned long long)rounds);
    atomicAdd(&c[3], (unsigned long long)tests);
    atomicAdd(&c[4], (unsigned long long)hits);
    atomicAdd(&c[5], (unsigned long long)visits);
    segments = items = rounds = tests = hits = visits = 0;
  }
};

// A source that walks a tree of its own inside finish() (a light pdf, say)
// may declare a member `int* lds_stack`: it receives the lane's column of the
// traversal stack in LDS (entry i at lds_stack[i * TRACE_BLOCK], STACK_LDS
// entries), which is empty whenever finish() runs.
template <class Src>
__device__ __forceinline__ auto bind_lds_stack(Src& src, int* col, int) -> decltype(src.lds_stack = col, void()) {
  src.lds_stack = col;
}
template <class Src>
__device__ __forceinline__ void bind_lds_stack(Src&, int*, long) {}

template <int QMODE, bool DACC, class Src>
__device__ __forceinline__ void run_segments(const TraceCtx& tc, Src& src, unsigned long long* work_counter,
                                             int64_t n_work, uint64_t* hitlist, unsigned long long* counters) {
  enum { ST_IDLE = 0, ST_ROUND = 1, ST_TRAV = 2, ST_BLEND = 3 };
  __shared__ int s_stack[STACK_LDS * TRACE_BLOCK];
  __shared__ int s_pend[PEND * TRACE_BLOCK];
  int s_ovf[STACK_OVF];
  TravStack st;
  st.lds = s_stack + threadIdx.x;
  st.ovf = s_ovf;
  st.sp = 0;
  bind_lds_stack(src, st.lds, 0);
  int* const pend = s_pend + threadIdx.x;
  const int lane = (int)(threadIdx.x & 63);
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  TraceCtx tcl = tc;
  tcl.hl = hitlist ? hitlist + ((int64_t)blockIdx.x * TRACE_BLOCK + threadIdx.x) * HL_CAP : nullptr;

  int stage = ST_IDLE;
  Seg<DACC> s;
  seg_begin(s, d3(0.0, 0.0, 0.0), d3(0.0, 0.0, 1.0));
  Round r;
  r.cnt = 0;
  r.trav = false;
  r.np = 0;
  RunStats rs;
  D3 O = d3(0.0, 0.0, 0.0), W = d3(0.0, 0.0, 1.0);   // the next segment's ray, from the source

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
      exhausted = base + (unsigned long long)__popcll(idle) >= (unsigned long long)n_work;
      if (need) {
        const int64_t wid = (int64_t)base + __popcll(idle & lt_mask);
        if (wid < n_work && src.start(wid, tcl, O, W)) {
          seg_begin(s, O, W);
          stage = ST_ROUND;
          ++rs.items;
          ++rs.segments;
        }
      }
    }
    // Every lane idle: stop once the counter is exhausted, else claim again
    // (a claim can hold only items that need no tracing).
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
      if (__ballot(stage == ST_TRAV) == 0 || __popcll(__ballot(stage == ST_BLEND)) >= RUN_BLEND_BATCH) break;
    }

    // ---- blend, and finish ended segments
    if (stage != ST_BLEND) continue;
    blend_round<QMODE>(tcl, s, r, src, nullptr, 0);
    if (!s.done) {
      stage = ST_ROUND;
      continue;
    }
    rs.rounds += s.rounds;
    rs.tests += s.tests;
    rs.hits += s.nhits;
    rs.visits += s.visits;
    if (src.finish(s, O, W)) {
      seg_begin(s, O, W);
      stage = ST_ROUND;
      ++rs.segments;
    } else {
      stage = ST_IDLE;
    }
  }
  if (counters) rs.flush(counters);
}

}  // namespace eag
