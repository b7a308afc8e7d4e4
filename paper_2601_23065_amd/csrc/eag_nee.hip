// Emitter importance sampling on emissive surfels, combined with the cosine
// sampling of the path tracer (Sec. 3.4, Eq. 9) by multiple importance
// sampling; the paper proposes it for small emitters (Sec. 5, limitations;
// Appendix D) and leaves the estimator open. The one built here:
//
//   emitters   surfels with e > tau_E and opacity > 0 (a segment passes the
//              emitter test only if it blends one of them: its E is a sum of
//              the hits' e with weights adding up to at most one);
//   selection  by power: emitter j with probability w_j / W, w_j = sigma
//              s_u s_v (mean(r) + e), by inversion of the inclusive prefix
//              sums; or by cells: the emitters grouped by the cube of side c
//              (a power of two) holding their centre, a cell chosen at the
//              vertex X with probability I_c / sum I, I_c = W_c /
//              max(|X - m_c|^2, c^2), then an emitter of it by power (u3);
//   point      uniform on the j's k_sigma ellipse (area density rho_j =
//              sigma (mean(r) + e) / (pi k^2 W), times I_c / sum I with W_c
//              in place of W for cells);
//   light pdf  p_l(X, w) = sum over the emitter ellipses the ray X + d w
//              crosses at d > 0 of rho_j d^2 / |w . n_j|, evaluated by a
//              traversal of a 4-wide tree over the emitters alone;
//   weights    power heuristic against the cosine pdf p_b = max(0, w . Nt)
//              / pi: a light segment that passes the emitter test adds
//              beta R p_b p_l / (p_b^2 + p_l^2) (beta after the vertex's P,
//              before Russian roulette), a cosine-sampled segment k >= 1 that
//              passes it adds beta R p_b^2 / (p_b^2 + p_l^2); the camera
//              segment is not weighted.
// The light sample at the vertex after segment k draws Philox counter
// (pixel, sample, 2^31 + k, id): u0 selects, u1 and u2 place the point.
// Light segments are ordinary segments of the persistent runner: after a
// reflecting vertex the lane traces the light segment first, then the
// cosine-sampled continuation (if Russian roulette keeps the path).
//
// Table build: per-surfel flags, an exclusive scan and a compaction give the
// emitters in ascending surfel order; with cells, a stable radix sort by cell
// key reorders them to (cell, surfel) order, flags at key changes and their
// scan number the cells, and one thread per cell sums its weights in order.
// The attributes are gathered into arrays of their own, the weights'
// inclusive scan gives the prefix sums, and the ordinary builder makes the
// tree over the compacted emitters.
#include "eag_device.h"
#include "eag_internal.h"
#include "eag_render.h"
#include "eag_runner.h"

#include <cmath>
#include <cstring>


namespace eag {

namespace {

constexpr uint32_t NEE_SEGMENT = 0x80000000u;
constexpr double INV_PI = 0.3183098861837907;

__device__ __forceinline__ void add_fixed(int64_t* acc, float v) {
  if (v != 0.0f) {
    const long long q = (long long)rint((double)v * EAG_ACCUM_SCALE);
    atomicAdd(reinterpret_cast<unsigned long long*>(acc), (unsigned long long)q);
  }
}

// ---------------------------------------------------------------------------
// Light sampling and its density
// ---------------------------------------------------------------------------
// Selection by cells: I_c(X) = W_c / max(|X - m_c|^2, c^2), evaluated as
// written (no fused multiply-add), and summed over the cells in order.
__device__ __forceinline__ double cell_importance(const EmitterDev& E, int32_t c, D3 X) {
#pragma clang fp contract(off)
  const double4 q = E.cells[c];
  const double dx = X.x - q.x, dy = X.y - q.y, dz = X.z - q.z;
  const double d2 = dx * dx + dy * dy + dz * dz;
  return q.w / fmax(d2, E.cell * E.cell);
}

__device__ double cell_total(const EmitterDev& E, D3 X) {
  double S = 0.0;
  for (int32_t c = 0; c < E.n_cells; ++c) S += cell_importance(E, c, X);
  return S;
}

// The emitter selected at X: the first cell whose running sum of I exceeds
// u0 S (S = cell_total(X)), then the first emitter of the cell whose prefix
// sum within the cell exceeds u3 W_c.
__device__ int64_t select_emitter_cells(const EmitterDev& E, D3 X, double S, double u0, double u3) {
  const double x = u0 * S;
  double cum = 0.0;
  int32_t c = 0;
  for (; c < E.n_cells - 1; ++c) {
    cum += cell_importance(E, c, X);
    if (cum > x) break;
  }
  const double y = u3 * E.cells[c].w;
  int64_t lo = E.begin[c], hi = E.begin[c + 1] - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (E.cdf_in[mid] > y) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// The term of one emitter ellipse in p_l (0 if the ray does not cross it at
// d > 0), in double precision, with the tracer's acceptance test; with
// cells, before the division by S(X).
// lc, li: the last cell whose I_c(X) was evaluated, and that value (leaves
// of one cell tend to come in a row).
__device__ __forceinline__ double pdf_term(const EmitterDev& E, uint32_t pos, D3 X, D3 W, int32_t& lc, double& li) {
  const EmitGeo* g = E.geo + pos;
  const D3 n = d3(g->n[0], g->n[1], g->n[2]);
  const double den = dot(W, n);
  if (!(fabs(den) > 1e-12)) return 0.0;
  const D3 d = d3(g->p[0], g->p[1], g->p[2]) - X;
  const double t = dot(d, n) / den;
  if (!(t > 0.0)) return 0.0;
  const D3 y = t * W - d;
  const double u = dot(y, d3(g->tu[0], g->tu[1], g->tu[2])) / g->su;
  const double v = dot(y, d3(g->tv[0], g->tv[1], g->tv[2])) / g->sv;
  if (!(u * u + v * v <= E.k2)) return 0.0;
  const double term = g->rho * t * t / fabs(den);
  if (E.n_cells == 0) return term;
  if (g->cell != lc) {
    lc = g->cell;
    li = cell_importance(E, lc, X);
  }
  return term * li;
}

// p_l(X, W): every emitter box the ray meets at t >= 0 is visited. The stack
// lives in the lane's LDS column (lds, STACK_LDS entries) and spills to
// private memory beyond; at most 3 * depth + 1 entries are ever held, within
// STACK_SIZE for the deepest tree a build can make.
__device__ double light_pdf(const EmitterDev& E, D3 X, D3 W, int* lds, double S) {
  double sum = 0.0;
  if (E.n == 0) return sum;
  const float wx = (float)W.x, wy = (float)W.y, wz = (float)W.z;
  const V3 iW = v3(1.0f / (fabsf(wx) > 1e-30f ? wx : copysignf(1e-30f, wx)),
                   1.0f / (fabsf(wy) > 1e-30f ? wy : copysignf(1e-30f, wy)),
                   1.0f / (fabsf(wz) > 1e-30f ? wz : copysignf(1e-30f, wz)));
  const V3 OiW = v3((float)X.x * iW.x, (float)X.y * iW.y, (float)X.z * iW.z);
  const float inf = __builtin_inff();
  int ovf[STACK_OVF];
  TravStack st;
  st.lds = lds;
  st.ovf = ovf;
  st.sp = 0;
  st.push(E.root);
  int32_t lc = -1;
  double li = 0.0;
  while (st.sp > 0) {
    const int ref = st.pop();
    if (ref < 0) {
      sum += pdf_term(E, (uint32_t)~ref, X, W, lc, li);
      continue;
    }
    const Node4* nd = E.nodes + ref;
    const int4 cr = nd->ref;
    const float4 b0 = nd->b[0], b1 = nd->b[1], b2 = nd->b[2], b3 = nd->b[3], b4 = nd->b[4], b5 = nd->b[5];
    const float e0 = slab(b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, OiW, iW, 0.0f, inf);
    const float e1 = slab(b1.z, b1.w, b2.x, b2.y, b2.z, b2.w, OiW, iW, 0.0f, inf);
    const float e2 = slab(b3.x, b3.y, b3.z, b3.w, b4.x, b4.y, OiW, iW, 0.0f, inf);
    const float e3 = slab(b4.z, b4.w, b5.x, b5.y, b5.z, b5.w, OiW, iW, 0.0f, inf);
    if (cr.x != NODE4_EMPTY && e0 < inf && st.sp < STACK_SIZE) st.push(cr.x);
    if (cr.y != NODE4_EMPTY && e1 < inf && st.sp < STACK_SIZE) st.push(cr.y);
    if (cr.z != NODE4_EMPTY && e2 < inf && st.sp < STACK_SIZE) st.push(cr.z);
    if (cr.w != NODE4_EMPTY && e3 < inf && st.sp < STACK_SIZE) st.push(cr.w);
  }
  return E.n_cells > 0 ? sum / S : sum;
}

// The emitter selected by u0: the first j whose inclusive prefix sum exceeds
// u0 W (u0 < 1, so j < n).
__device__ __forceinline__ int64_t select_emitter(const EmitterDev& E, double u0) {
  const double x = u0 * E.W;
  int64_t lo = 0, hi = E.n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (E.cdf[mid] > x) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// Uniform point on emitter j's k_sigma ellipse.
__device__ __forceinline__ D3 emitter_point(const EmitterDev& E, int64_t j, double u1, double u2) {
  const int64_t n = E.n;
  Record rec;
  rec.p_sigma = make_float4(E.pos[j], E.pos[n + j], E.pos[2 * n + j], 1.0f);
  rec.q = make_float4(E.rot[j], E.rot[n + j], E.rot[2 * n + j], E.rot[3 * n + j]);
  rec.s_idx = make_float4(E.scale[j], E.scale[n + j], 0.0f, 0.0f);
  const Geo g = surfel_geo(rec);
  const double r = E.k * sqrt(u1);
  double s, c;
  sincos(TWO_PI * u2, &s, &c);
  const double a = r * c * g.su, b = r * s * g.sv;
  return d3(g.p.x + a * g.tu.x + b * g.tv.x, g.p.y + a * g.tu.y + b * g.tv.y, g.p.z + a * g.tu.z + b * g.tv.z);
}

// ---------------------------------------------------------------------------
// Contributions that wait for their light pdf
// ---------------------------------------------------------------------------
// The tree walk of the light pdf would run inside finish() for the few lanes
// that end a segment together, with the rest of the wave waiting. Instead the
// path kernel queues each contribution that needs it, and a second kernel
// walks the tree once per entry with every lane busy. A path queues at most
// one entry per reflecting vertex and one at its end, so a launch of P paths
// at max depth D needs at most P (D + 1) entries; the host launches sample
// chunks that fit. Integer accumulation makes the image independent of the
// order in which contributions arrive.
struct __align__(16) PdfEntry {
  double o[3], w[3];   // the segment's ray
  double pbx;          // cosine pdf of its direction at o
  double S;            // selection by cells: S at o
  float a[3], b[3];    // light segment: beta at o and R; cosine-sampled: beta R in a
  uint32_t pix;
  uint32_t light;
};
struct PdfQueue {
  PdfEntry* e;
  unsigned long long* count;
  int64_t cap;
};

// ---------------------------------------------------------------------------
// One lane's path with light segments
// ---------------------------------------------------------------------------
struct MisPathSource {
  const PtLaunch* L;
  const EmitterDev* E;
  const PdfQueue* Q;
  int* lds_stack;   // the lane's traversal-stack column, free while finishing
  uint32_t pix, sample;
  int depth;
  V3 beta;
  V3 lf;            // beta at the vertex of the pending light segment
  D3 Wb;            // the cosine-sampled continuation (from the vertex, which is
                    // the light segment's origin while that segment is in flight)
  double pb;        // cosine pdf of the direction of the segment in flight (or the continuation)
  double pbl;       // cosine pdf of the pending light segment's direction
  double Sx;        // selection by cells: S at the vertex the segment in flight started from
  bool light;       // the segment in flight is a light segment
  bool cont;        // the continuation survived Russian roulette

  __device__ __forceinline__ bool start(int64_t wid, TraceCtx& tcl, D3& O, D3& W) {
    const PtSlot& S = L->s[0];
    const int64_t s_rel = wid / S.tile_pixels;
    const int64_t tp = wid - s_rel * S.tile_pixels;
    const int64_t tile = tp >> 6;
    const int within = (int)(tp & 63);
    const int x = (int)(tile % S.tiles_x) * 8 + (within & 7);
    const int y = (int)(tile / S.tiles_x) * 8 + (within >> 3);
    if (x >= S.cam.width || y >= S.cam.height) return false;
    pix = (uint32_t)(y * S.cam.width + x);
    sample = S.sample_begin + (uint32_t)s_rel;
    beta = v3(1.f, 1.f, 1.f);
    depth = 0;
    light = false;
    cont = false;
    pb = 0.0;
    tcl.attrs = S.attrs;
    O = d3(S.cam.eye[0], S.cam.eye[1], S.cam.eye[2]);
    W = pixel_dir(S.cam, pix, sample, S.flags, S.k0, S.k1);
    return true;
  }

  __device__ __forceinline__ void operator()(uint32_t, double, double, double, double, D3, D3) const {}

  // Queue a contribution; the lanes that call this together claim their
  // slots with one atomic.
  __device__ __forceinline__ void defer(bool is_light, D3 o, D3 w, double pbx, V3 a, V3 b) {
    const int lane = (int)(threadIdx.x & 63);
    const uint64_t m = __ballot(true);
    const int leader = __ffsll((unsigned long long)m) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(Q->count, (unsigned long long)__popcll(m));
    base = __shfl(base, leader);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const unsigned long long slot = base + (unsigned long long)__popcll(m & below);
    // the host sizes launches so that this never happens; the settle kernel counts any claim past the end
    if (slot >= (unsigned long long)Q->cap) return;
    PdfEntry& e = Q->e[slot];
    e.o[0] = o.x; e.o[1] = o.y; e.o[2] = o.z;
    e.w[0] = w.x; e.w[1] = w.y; e.w[2] = w.z;
    e.pbx = pbx;
    e.S = Sx;
    e.a[0] = a.x; e.a[1] = a.y; e.a[2] = a.z;
    e.b[0] = b.x; e.b[1] = b.y; e.b[2] = b.z;
    e.pix = pix;
    e.light = is_light ? 1u : 0u;
  }

  __device__ __forceinline__ bool finish(const Seg<false>& s, D3& O, D3& W) {
    const PtSlot& S = L->s[0];
    int64_t* acc = S.accum + (int64_t)pix * 3;
    const double A = 1.0 - s.T;
    const bool hit = s.nhits > 0 && A > 0.0;
    if (light) {
      // the light pdf is needed only when the segment passes the emitter test
      light = false;
      if (hit && s.E > S.tau_E) defer(true, s.O, s.W, pbl, lf, v3(s.R0, s.R1, s.R2));
      if (!cont) return false;
      O = s.O;
      W = Wb;
      return true;
    }
    if (!hit) return false;
    if (s.E > S.tau_E) {
      const V3 bR = v3(beta.x * s.R0, beta.y * s.R1, beta.z * s.R2);
      if (depth >= 1 && E->n > 0) {
        defer(false, s.O, s.W, pb, bR, bR);
      } else {
        add_fixed(acc + 0, bR.x);
        add_fixed(acc + 1, bR.y);
        add_fixed(acc + 2, bR.z);
      }
      return false;
    }
    if (depth >= S.max_depth) return false;
    beta = v3(beta.x * s.P0, beta.y * s.P1, beta.z * s.P2);
    const D3 Nt = (1.0 / sqrt(dot(s.N, s.N))) * s.N;
    const double Dt = s.D / A;
    const D3 X = d3(s.O.x + Dt * s.W.x, s.O.y + Dt * s.W.y, s.O.z + Dt * s.W.z);
    // light sample, before Russian roulette
    D3 Wl = d3(0.0, 0.0, 1.0);
    if (E->n > 0) {
      const uint4 wl = philox(make_uint4(pix, sample, NEE_SEGMENT + (uint32_t)depth, S.cam.id), S.k0, S.k1);
      int64_t j;
      if (E->n_cells > 0) {
        Sx = cell_total(*E, X);
        j = select_emitter_cells(*E, X, Sx, to_unit(wl.x), to_unit(wl.w));
      } else {
        j = select_emitter(*E, to_unit(wl.x));
      }
      const D3 y = emitter_point(*E, j, to_unit(wl.y), to_unit(wl.z));
      const D3 dl = y - X;
      Wl = (1.0 / sqrt(dot(dl, dl))) * dl;
      const double cl = dot(Wl, Nt);
      if (cl > 0.0) {
        pbl = cl * INV_PI;
        lf = beta;
        light = true;
      }
    }
    // cosine sample and Russian roulette, as the plain path tracer
    const uint4 w = philox(make_uint4(pix, sample, (uint32_t)depth, S.cam.id), S.k0, S.k1);
    ++depth;
    cont = true;
    if (S.rr_start > 0 && depth >= S.rr_start) {
      const float q = fminf(0.95f, fmaxf(fmaxf(beta.x, beta.y), beta.z));
      if (!(to_unit(w.z) < q)) {
        cont = false;
      } else {
        const float iq = 1.0f / q;
        beta = v3(beta.x * iq, beta.y * iq, beta.z * iq);
      }
    }
    Wb = cosine_dir(Nt, to_unit(w.x), to_unit(w.y));
    pb = fmax(dot(Wb, Nt), 0.0) * INV_PI;
    O = X;
    if (light) {
      W = Wl;
      return true;
    }
    W = Wb;
    return cont;
  }
};

// Two waves per SIMD, as the plain path tracer: without the bound the
// allocator takes enough registers for one.
__global__ void __launch_bounds__(TRACE_BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
k_path_trace_mis(TraceCtx tc, PtLaunch L, EmitterDev E, PdfQueue Q, unsigned long long* work_counter,
                 unsigned long long* counters, uint64_t* hitlist) {
  MisPathSource src;
  src.L = &L;
  src.E = &E;
  src.Q = &Q;
  src.lds_stack = nullptr;
  src.pix = src.sample = 0;
  src.depth = 0;
  src.beta = src.lf = v3(0.f, 0.f, 0.f);
  src.Wb = d3(0.0, 0.0, 0.0);
  src.pb = src.pbl = src.Sx = 0.0;
  src.light = src.cont = false;
  run_segments<Q_ALL, false>(tc, src, work_counter, L.n_work, hitlist, counters);
}

// One queued contribution per thread (grid-stride): its light pdf, its MIS
// weight, and the weighted value into the pixel's accumulator.
__global__ void __launch_bounds__(TRACE_BLOCK) k_settle_pdfs(EmitterDev E, PdfQueue Q, int64_t* accum,
                                                             unsigned long long* counters) {
  __shared__ int s_stack[STACK_LDS * TRACE_BLOCK];
  const unsigned long long claimed = *Q.count;
  const unsigned long long n = claimed < (unsigned long long)Q.cap ? claimed : (unsigned long long)Q.cap;
  // Claims past the queue's end were dropped by the path kernel: counted, so
  // that a caller can see that the image lacks them.
  if (counters && blockIdx.x == 0 && threadIdx.x == 0 && claimed > n) atomicAdd(&counters[6], claimed - n);
  for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    const PdfEntry& e = Q.e[i];
    const D3 o = d3(e.o[0], e.o[1], e.o[2]), w = d3(e.w[0], e.w[1], e.w[2]);
    const double pl = light_pdf(E, o, w, s_stack + threadIdx.x, e.S);
    const double pbx = e.pbx;
    const double den = pbx * pbx + pl * pl;
    int64_t* acc = accum + (int64_t)e.pix * 3;
    if (e.light) {
      const float f = den > 0.0 ? (float)(pbx * pl / den) : 0.0f;
      add_fixed(acc + 0, (e.a[0] * f) * e.b[0]);
      add_fixed(acc + 1, (e.a[1] * f) * e.b[1]);
      add_fixed(acc + 2, (e.a[2] * f) * e.b[2]);
    } else {
      const double wgt = den > 0.0 ? pbx * pbx / den : 1.0;
      add_fixed(acc + 0, (float)(e.a[0] * wgt));
      add_fixed(acc + 1, (float)(e.a[1] * wgt));
      add_fixed(acc + 2, (float)(e.a[2] * wgt));
    }
  }
}

// ---------------------------------------------------------------------------
// Table build
// ---------------------------------------------------------------------------
__global__ void k_emit_flags(eag_surfels s, float tau_E, uint32_t* flags) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < s.n) flags[i] = (s.emissive[i] > tau_E && s.opacity[i] > 0.0f) ? 1u : 0u;
}

__global__ void k_emit_count(const uint32_t* flags, const uint32_t* scan, int64_t n, unsigned long long* count) {
  *count = (unsigned long long)scan[n - 1] + flags[n - 1];
}

__device__ __forceinline__ void copy_surfel(const eag_surfels& s, int64_t i, const eag_surfels_out& c, int64_t j) {
  const int64_t n = s.n, ne = c.n;
  for (int k = 0; k < 3; ++k) {
    c.pos[k * ne + j] = s.pos[k * n + i];
    c.albedo[k * ne + j] = s.albedo[k * n + i];
    c.radiance[k * ne + j] = s.radiance[k * n + i];
  }
  for (int k = 0; k < 4; ++k) c.rot[k * ne + j] = s.rot[k * n + i];
  for (int k = 0; k < 2; ++k) c.scale[k * ne + j] = s.scale[k * n + i];
  c.opacity[j] = s.opacity[i];
  c.emissive[j] = s.emissive[i];
}

// Emitter off[i] takes surfel i's attributes (arrays of ne), in surfel order.
__global__ void k_emit_gather(eag_surfels s, const uint32_t* flags, const uint32_t* off, eag_surfels_out c) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= s.n || !flags[i]) return;
  copy_surfel(s, i, c, off[i]);
}

// The cell key of each gathered emitter: floor(p / c) per axis (exact: c is
// a power of two), offset by 2^20 and packed 21 bits per axis, x first.
__global__ void k_emit_keys(eag_surfels_out c, float inv_cell, uint64_t* keys, uint32_t* vals) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t ne = c.n;
  if (j >= ne) return;
  uint64_t key = 0;
  for (int a = 0; a < 3; ++a) key = (key << 21) | (uint64_t)((int64_t)floorf(c.pos[a * ne + j] * inv_cell) + (1 << 20));
  keys[j] = key;
  vals[j] = (uint32_t)j;
}

// Final order: entry j takes gathered emitter order[j] (identity when null)
// and its weight.
__global__ void k_emit_permute(eag_surfels g, const uint32_t* order, eag_surfels_out c, double* w) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t ne = c.n;
  if (j >= ne) return;
  const int64_t i = order ? (int64_t)order[j] : j;
  copy_surfel(g, i, c, j);
  const double rbar = ((double)g.radiance[i] + (double)g.radiance[ne + i] + (double)g.radiance[2 * ne + i]) / 3.0;
  w[j] = (double)g.opacity[i] * (double)g.scale[i] * (double)g.scale[ne + i] * (rbar + (double)g.emissive[i]);
}

// First entry of each cell (keys sorted).
__global__ void k_cell_flags(const uint64_t* keys, int64_t ne, uint32_t* flags) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j < ne) flags[j] = (j == 0 || keys[j] != keys[j - 1]) ? 1u : 0u;
}

// cell_of holds the inclusive scan of the flags (cell index + 1).
__global__ void k_cell_begin(const uint32_t* flags, const uint32_t* cell_of, int64_t ne, int32_t* begin,
                             unsigned long long* n_cells) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= ne) return;
  if (flags[j]) begin[cell_of[j] - 1] = (int32_t)j;
  if (j == ne - 1) {
    begin[cell_of[j]] = (int32_t)ne;
    *n_cells = cell_of[j];
  }
}

// One thread per cell: its prefix sums in order, its total, its centre.
__global__ void k_cell_sums(eag_surfels_out c, const double* w, const int32_t* begin, int32_t n_cells, double cell,
                            double* cdf_in, double4* cells) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n_cells) return;
  const int32_t b = begin[k], e = begin[k + 1];
  double sum = 0.0;
  for (int32_t j = b; j < e; ++j) {
    sum += w[j];
    cdf_in[j] = sum;
  }
  const float inv = (float)(1.0 / cell);
  const int64_t ne = c.n;
  double m[3];
  for (int a = 0; a < 3; ++a) m[a] = ((double)floorf(c.pos[a * ne + b] * inv) + 0.5) * cell;
  cells[k] = make_double4(m[0], m[1], m[2], sum);
}

// rho_j against the total weight, or (cells) against the weight of j's cell.
__global__ void k_emit_rho(eag_surfels_out c, const double* cdf, const double* cdf_in, const int32_t* begin,
                           const uint32_t* cell_of, double k, double* rho) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t ne = c.n;
  if (j >= ne) return;
  const double rbar = ((double)c.radiance[j] + (double)c.radiance[ne + j] + (double)c.radiance[2 * ne + j]) / 3.0;
  const double W = cell_of ? cdf_in[begin[cell_of[j]] - 1] : cdf[ne - 1];
  rho[j] = (double)c.opacity[j] * (rbar + (double)c.emissive[j]) / (M_PI * k * k * W);
}

// Geometry of the emitter at leaf position pos, from its record.
__global__ void k_emit_geo(const Record* recs, const double* rho, const uint32_t* cell_of, int64_t ne, EmitGeo* geo) {
  const int64_t pos = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (pos >= ne) return;
  const Record rec = load_record(recs, (uint32_t)pos);
  const Geo g = surfel_geo(rec);
  EmitGeo e;
  e.p[0] = g.p.x; e.p[1] = g.p.y; e.p[2] = g.p.z;
  e.tu[0] = g.tu.x; e.tu[1] = g.tu.y; e.tu[2] = g.tu.z;
  e.tv[0] = g.tv.x; e.tv[1] = g.tv.y; e.tv[2] = g.tv.z;
  e.n[0] = g.n.x; e.n[1] = g.n.y; e.n[2] = g.n.z;
  e.su = g.su;
  e.sv = g.sv;
  e.rho = rho[rec_index(rec)];
  e.cell = cell_of ? (int32_t)cell_of[rec_index(rec)] - 1 : 0;
  e.pad = 0;
  geo[pos] = e;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

struct EmitWs {
  uint32_t* flags;
  uint32_t* off;
  unsigned long long* count;
  float* stage;            // gathered emitter attributes, 17 floats each
  uint64_t *keys, *keys_sorted;
  uint32_t *vals, *order;
  void* scan_tmp;
  size_t scan_bytes;
  void* build;
  size_t build_bytes;
  size_t bytes;
};

size_t emit_scan_bytes(int64_t n) {
  return std::max(std::max(scan_u32_bytes(n), scan_f64_bytes(n)), sort_pairs_bytes(n));
}

EmitWs emit_ws(void* base, int64_t n) {
  Carver c(base, ~size_t(0));
  EmitWs w;
  w.flags = c.take<uint32_t>(n);
  w.off = c.take<uint32_t>(n);
  w.count = c.take<unsigned long long>(2);
  w.stage = c.take<float>(17 * n);
  w.keys = c.take<uint64_t>(n);
  w.keys_sorted = c.take<uint64_t>(n);
  w.vals = c.take<uint32_t>(n);
  w.order = c.take<uint32_t>(n);
  w.scan_bytes = emit_scan_bytes(n);
  w.scan_tmp = c.take<char>(w.scan_bytes);
  w.build_bytes = build_ws_bytes(n);
  w.build = c.take<char>(w.build_bytes);
  w.bytes = c.bytes();
  return w;
}

struct EmitMem {
  float *pos, *rot, *scale, *opacity, *albedo, *radiance, *emissive;
  double *w, *cdf, *rho;
  EmitGeo* geo;
  double* cdf_in;          // prefix sums within each cell
  double4* cells;          // centre, total weight
  int32_t* begin;          // first entry of each cell, then ne
  uint32_t* cell_of;       // cell index + 1 of each entry
  void* bvh;
  size_t bvh_bytes;
  size_t bytes;
};

// Regions sized for n emitters; a table of ne <= n emitters uses strides ne.
EmitMem emit_mem(void* base, int64_t n) {
  Carver c(base, ~size_t(0));
  EmitMem m;
  m.pos = c.take<float>(3 * n);
  m.rot = c.take<float>(4 * n);
  m.scale = c.take<float>(2 * n);
  m.opacity = c.take<float>(n);
  m.albedo = c.take<float>(3 * n);
  m.radiance = c.take<float>(3 * n);
  m.emissive = c.take<float>(n);
  m.w = c.take<double>(n);
  m.cdf = c.take<double>(n);
  m.rho = c.take<double>(n);
  m.geo = c.take<EmitGeo>(n);
  m.cdf_in = c.take<double>(n);
  m.cells = c.take<double4>(n);
  m.begin = c.take<int32_t>(n + 1);
  m.cell_of = c.take<uint32_t>(n);
  m.bvh_bytes = bvh_layout(nullptr, n).bytes;
  m.bvh = c.take<char>(m.bvh_bytes);
  m.bytes = c.bytes();
  return m;
}

}  // namespace

size_t emitters_mem_bytes(int64_t n) { return emit_mem(nullptr, n).bytes; }
size_t emitters_ws_bytes(int64_t n) { return emit_ws(nullptr, n).bytes; }

void build_emitters(const eag_surfels* s, float tau_E, float k_sigma, float cell, void* mem, size_t mem_bytes,
                    void* ws, size_t ws_bytes, hipStream_t st, eag_emitters* out) {
  const int64_t n = s->n;
  const EmitMem m = emit_mem(mem, n);
  const EmitWs w = emit_ws(ws, n);
  if (mem_bytes < m.bytes) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "emitter table memory too small");
  if (ws_bytes < w.bytes) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "emitter table workspace too small");
  hipLaunchKernelGGL(k_emit_flags, dim3(blocks_for(n)), dim3(256), 0, st, *s, tau_E, w.flags);
  scan_u32(w.flags, w.off, n, false, w.scan_tmp, w.scan_bytes, st);
  hipLaunchKernelGGL(k_emit_count, dim3(1), dim3(1), 0, st, w.flags, w.off, n, w.count);
  unsigned long long ne = 0;
  check_hip(hipMemcpyAsync(&ne, w.count, sizeof(ne), hipMemcpyDeviceToHost, st), "emitter count");
  check_hip(hipStreamSynchronize(st), "emitter count sync");

  std::memset(out, 0, sizeof(*out));
  out->n_src = n;
  out->tau_E = tau_E;
  out->k_sigma = k_sigma;
  out->cell = cell;
  EmitterDev& E = out->dev;
  E.n = (int64_t)ne;
  E.k = (double)k_sigma;
  E.k2 = E.k * E.k;
  E.cell = (double)cell;
  if (ne == 0) return;

  // gathered in surfel order, then (cells) sorted by (cell, surfel): the
  // radix sort is stable
  const unsigned bne = blocks_for((int64_t)ne);
  eag_surfels_out g;
  g.n = (int64_t)ne;
  g.pos = w.stage; g.rot = w.stage + 3 * ne; g.scale = w.stage + 7 * ne; g.opacity = w.stage + 9 * ne;
  g.albedo = w.stage + 10 * ne; g.radiance = w.stage + 13 * ne; g.emissive = w.stage + 16 * ne;
  hipLaunchKernelGGL(k_emit_gather, dim3(blocks_for(n)), dim3(256), 0, st, *s, w.flags, w.off, g);
  const uint32_t* order = nullptr;
  if (cell > 0.0f) {
    hipLaunchKernelGGL(k_emit_keys, dim3(bne), dim3(256), 0, st, g, 1.0f / cell, w.keys, w.vals);
    sort_pairs_u64(w.keys, w.keys_sorted, w.vals, w.order, (int64_t)ne, 63, w.scan_tmp, w.scan_bytes, st);
    order = w.order;
  }
  eag_surfels gs;
  gs.n = (int64_t)ne;
  gs.pos = g.pos; gs.rot = g.rot; gs.scale = g.scale; gs.opacity = g.opacity;
  gs.albedo = g.albedo; gs.radiance = g.radiance; gs.emissive = g.emissive;
  eag_surfels_out c;
  c.n = (int64_t)ne;
  c.pos = m.pos; c.rot = m.rot; c.scale = m.scale; c.opacity = m.opacity;
  c.albedo = m.albedo; c.radiance = m.radiance; c.emissive = m.emissive;
  hipLaunchKernelGGL(k_emit_permute, dim3(bne), dim3(256), 0, st, gs, order, c, m.w);
  scan_f64(m.w, m.cdf, (int64_t)ne, true, w.scan_tmp, w.scan_bytes, st);
  const uint32_t* cell_of = nullptr;
  if (cell > 0.0f) {
    hipLaunchKernelGGL(k_cell_flags, dim3(bne), dim3(256), 0, st, w.keys_sorted, (int64_t)ne, w.vals);
    scan_u32(w.vals, m.cell_of, (int64_t)ne, true, w.scan_tmp, w.scan_bytes, st);
    hipLaunchKernelGGL(k_cell_begin, dim3(bne), dim3(256), 0, st, w.vals, m.cell_of, (int64_t)ne, m.begin,
                       w.count + 1);
    unsigned long long nc = 0;
    check_hip(hipMemcpyAsync(&nc, w.count + 1, sizeof(nc), hipMemcpyDeviceToHost, st), "cell count");
    check_hip(hipStreamSynchronize(st), "cell count sync");
    E.n_cells = (int32_t)nc;
    hipLaunchKernelGGL(k_cell_sums, dim3(blocks_for((int64_t)nc)), dim3(256), 0, st, c, m.w, m.begin, E.n_cells,
                       E.cell, m.cdf_in, m.cells);
    cell_of = m.cell_of;
  }
  hipLaunchKernelGGL(k_emit_rho, dim3(bne), dim3(256), 0, st, c, m.cdf, m.cdf_in, m.begin, cell_of, E.k, m.rho);
  check_hip(hipGetLastError(), "emitter table kernels");
  check_hip(hipMemcpyAsync(&E.W, m.cdf + ne - 1, sizeof(double), hipMemcpyDeviceToHost, st), "emitter total");

  // the tree over the compacted emitters
  eag_surfels cs;
  cs.n = (int64_t)ne;
  cs.pos = m.pos; cs.rot = m.rot; cs.scale = m.scale; cs.opacity = m.opacity;
  cs.albedo = m.albedo; cs.radiance = m.radiance; cs.emissive = m.emissive;
  const BvhLayout l = bvh_layout(m.bvh, (int64_t)ne);
  eag_bvh* b = new eag_bvh();
  std::memset(b, 0, sizeof(*b));
  b->n = (int64_t)ne;
  int bits = 1;
  while ((int64_t(1) << bits) < (int64_t)ne) ++bits;
  b->idx_bits = bits;
  b->mem = m.bvh;
  b->mem_bytes = m.bvh_bytes;
  bvh_attach(b, l);
  try {
    check_hip(hipEventCreateWithFlags(&b->built, hipEventDisableTiming), "build event");
    build_bvh(&cs, b, w.build, w.build_bytes, st);
  } catch (...) {
    if (b->built) (void)hipEventDestroy(b->built);
    delete b;
    throw;
  }
  // (the light-pdf walk holds at most 3 entries per level plus one: within
  // STACK_SIZE for any tree)
  hipLaunchKernelGGL(k_emit_geo, dim3(bne), dim3(256), 0, st, b->recs, m.rho, cell_of, (int64_t)ne, m.geo);
  check_hip(hipGetLastError(), "emitter geometry");
  check_hip(hipStreamSynchronize(st), "emitter table sync");
  out->bvh = b;
  E.nodes = b->nodes4;
  E.geo = m.geo;
  E.root = b->root;
  E.rho = m.rho;
  E.cdf = m.cdf;
  E.pos = m.pos;
  E.rot = m.rot;
  E.scale = m.scale;
  E.cdf_in = m.cdf_in;
  E.cells = m.cells;
  E.begin = m.begin;
}

size_t pdf_queue_bytes(int64_t entries) { return (size_t)entries * sizeof(PdfEntry) + 256; }

int64_t pdf_queue_entries(int64_t pixels, int32_t max_depth, uint32_t chunk) {
  return pixels * (int64_t)chunk * (int64_t)(max_depth + 1);
}

void launch_path_trace_mis(const TraceCtx& tc, const PtLaunch& L, const EmitterDev& E, void* queue,
                           int64_t queue_entries, unsigned long long* work_counter, unsigned long long* counters,
                           uint64_t* hitlist, hipStream_t st) {
  const unsigned blocks = (unsigned)(runner_lanes() / TRACE_BLOCK);
  PdfQueue Q;
  Q.count = reinterpret_cast<unsigned long long*>(queue);
  Q.e = reinterpret_cast<PdfEntry*>(static_cast<char*>(queue) + 256);
  Q.cap = queue_entries;
  launch_zero_u64(work_counter, 1, st);
  launch_zero_u64(Q.count, 1, st);
  hipLaunchKernelGGL(k_path_trace_mis, dim3(blocks), dim3(TRACE_BLOCK), 0, st, tc, L, E, Q, work_counter, counters,
                     hitlist);
  check_hip(hipGetLastError(), "path_trace_mis launch");
  if (E.n > 0) {
    hipLaunchKernelGGL(k_settle_pdfs, dim3(blocks), dim3(TRACE_BLOCK), 0, st, E, Q, L.s[0].accum, counters);
    check_hip(hipGetLastError(), "settle launch");
  }
}

}  // namespace eag
