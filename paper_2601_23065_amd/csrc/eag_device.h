// Device-side building blocks shared by the build, trace, render and path
// tracing kernels: Philox4x32-10, camera rays, the hemisphere frame and
// cosine-weighted sampling, the BVH node and surfel record layouts, and the
// per-ray traversal + k-buffer + compositing core.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace eag {

constexpr int KBUF = 16;          // k-buffer depth
// Traversal stack: 3 entries per level of the deepest tree a build can make
// (64 clustering iterations plus at most 23 halving iterations, each adding
// at most one level, so at most 87 levels), so that no tree needs a check on
// the host. Entries past the LDS part live in
// private memory and are rarely touched.
constexpr int STACK_SIZE = 264;

// ---------------------------------------------------------------------------
// Layouts in HBM
// ---------------------------------------------------------------------------
// Internal node, 64 B: both children's boxes and references. A reference
// c >= 0 is an internal node, c < 0 is a leaf holding the surfel at sorted
// (Morton) position ~c.
struct __align__(16) Node {
  float4 a;   // lo0.x lo0.y lo0.z hi0.x
  float4 b;   // hi0.y hi0.z lo1.x lo1.y
  float4 c;   // lo1.z hi1.x hi1.y hi1.z
  int4 d;     // child0 child1 - -
};

// 4-wide node, 128 B, collapsed from the binary tree: child k's box is
// floats [6k, 6k+6) of b (lo.xyz, hi.xyz); ref.k >= 0 is a 4-wide node,
// ref.k < 0 a leaf holding the surfel at sorted position ~ref.k, and
// NODE4_EMPTY an unused slot. src.k is the binary-tree reference the child
// came from (used to refit boxes).
constexpr int NODE4_EMPTY = 0x7fffffff;
struct __align__(16) Node4 {
  float4 b[6];
  int4 ref;
  int4 src;
};

// Geometry record of one surfel in sorted order, 48 B (three float4 loads):
//   p.x p.y p.z sigma | q.w q.x q.y q.z | s_u s_v index -
// with q the caller's (unnormalised) quaternion and index the original surfel
// index. Frames are derived in double precision at use (surfel_geo), so the
// tracer sees exactly the float32 inputs, like the float64 definition.
struct __align__(16) Record {
  float4 p_sigma;
  float4 q;
  float4 s_idx;
};

// Attributes of one surfel in sorted order, 32 B: rho.xyz e | r.xyz -
struct __align__(16) Attr {
  float4 rho_e;
  float4 r;
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): published multipliers and key
// increments, ten rounds. Counter (pixel, sample, segment, stream id).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}
// u = (w >> 8) * 2^-24, exact in float32
__device__ __forceinline__ float to_unit(uint32_t w) { return (float)(w >> 8) * (1.0f / 16777216.0f); }

// ---------------------------------------------------------------------------
// small vector helpers
// ---------------------------------------------------------------------------
struct V3 { float x, y, z; };
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return V3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// double-precision vectors for ray geometry
struct D3 { double x, y, z; };
__device__ __forceinline__ D3 d3(double x, double y, double z) { return D3{x, y, z}; }
__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return D3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return D3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ D3 operator*(double s, D3 a) { return D3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 cross(D3 a, D3 b) {
  return D3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// Pinhole camera prepared on the host in double precision: ray direction =
// normalize(dx * right + dy * up + fwd) with dx = 2 (x + ox) / W - 1,
// dy = 1 - 2 (y + oy) / H; right and up are pre-scaled by tan(vfov/2) * W/H
// and tan(vfov/2).
struct CamDev {
  double eye[3], right[3], up[3], fwd[3];
  int32_t width, height;
  uint32_t id;
  int32_t pad;
};

__device__ __forceinline__ D3 camera_dir(const CamDev& c, int px, int py, double ox, double oy) {
  const double dx = 2.0 * ((double)px + ox) / (double)c.width - 1.0;
  const double dy = 1.0 - 2.0 * ((double)py + oy) / (double)c.height;
  D3 d = d3(dx * c.right[0] + dy * c.up[0] + c.fwd[0], dx * c.right[1] + dy * c.up[1] + c.fwd[1],
            dx * c.right[2] + dy * c.up[2] + c.fwd[2]);
  return (1.0 / sqrt(dot(d, d))) * d;
}

// Hemisphere frame: Gram-Schmidt of the fixed helper h = (1,2,3)/sqrt(14)
// against the unit normal n: b1 = normalize(h - (h.n) n), b2 = n x b1.
// Cosine-weighted direction (Malley): r = sqrt(u0), phi = 2 pi u1,
// w' = r cos(phi) b1 + r sin(phi) b2 + sqrt(1 - u0) n.
constexpr double HX = 0.2672612419124244, HY = 0.5345224838248488, HZ = 0.8017837257372732;
constexpr double TWO_PI = 6.283185307179586;

__device__ __forceinline__ D3 cosine_dir(D3 n, double u0, double u1) {
  const double hn = HX * n.x + HY * n.y + HZ * n.z;
  const D3 m = d3(HX - hn * n.x, HY - hn * n.y, HZ - hn * n.z);
  const D3 b1 = (1.0 / sqrt(dot(m, m))) * m;
  const D3 b2 = cross(n, b1);
  const double r = sqrt(u0);
  double s, c;
  sincos(TWO_PI * u1, &s, &c);
  const double z = sqrt(1.0 - u0);
  return d3(r * c * b1.x + r * s * b2.x + z * n.x, r * c * b1.y + r * s * b2.y + z * n.y,
            r * c * b1.z + r * s * b2.z + z * n.z);
}

// ---------------------------------------------------------------------------
// Order key: (bucket, original index, sorted position) packed into 64 bits,
// bucket = floor(t / dq) (dq a power of two) or the float bits of t when
// dq == 0. Ordering keys as integers orders hits by (bucket, index); the
// sorted position rides along so that the blending pass can address the
// record directly.
// ---------------------------------------------------------------------------
struct TraceCtx {
  const Node4* nodes;
  const Record* recs;
  const Attr* attrs;
  int32_t root;            // >= 0: internal node index; < 0: single leaf ~root
  int32_t idx_bits;        // bits of an index (both index fields)
  uint32_t max_bucket;     // largest representable bucket
  double inv_dq;           // 1 / dq, or 0 for exact-t keys
  double dq;               // the depth quantum (a power of two, so b * dq == b / inv_dq exactly), or 0
  double t_min;
  double k2;               // k_sigma^2
  double T_min;
  // Mapped host word receiving device status codes (a key beyond the last
  // bucket); null: not reported.
  unsigned int* status;
  // Optional per-lane hit list (null: off). Entry j of this lane is
  // hl[j * HL_STRIDE]. A lane's entries are contiguous: appends happen at
  // different times in different lanes, and a lane filling its own cache
  // lines writes each line back once.
  uint64_t* hl;
};

constexpr int HL_CAP = 256;        // entries per lane (a multiple of 8: the list is scanned 8 at a time)
constexpr int HL_STRIDE = 1;
static_assert(HL_CAP % 8 == 0 && HL_STRIDE == 1, "hit-list scan reads 8 contiguous entries");

__device__ __noinline__ void report_key_range(unsigned int* status) {
  if (status) __hip_atomic_fetch_or(status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t make_key(const TraceCtx& tc, double t, uint32_t idx, uint32_t pos) {
  uint32_t bucket;
  if (tc.inv_dq > 0.0) {
    const double b = floor(t * tc.inv_dq);
    bucket = b >= (double)tc.max_bucket ? tc.max_bucket : (uint32_t)b;
  } else {
    bucket = __float_as_uint((float)t);
  }
  return ((uint64_t)bucket << (2 * tc.idx_bits)) | ((uint64_t)idx << tc.idx_bits) | (uint64_t)pos;
}
__device__ __forceinline__ uint64_t make_key_b(const TraceCtx& tc, uint32_t bucket, uint32_t idx, uint32_t pos) {
  bucket = bucket >= tc.max_bucket ? tc.max_bucket : bucket;
  return ((uint64_t)bucket << (2 * tc.idx_bits)) | ((uint64_t)idx << tc.idx_bits) | (uint64_t)pos;
}
__device__ __forceinline__ uint32_t key_pos(const TraceCtx& tc, uint64_t k) {
  return (uint32_t)(k & ((1ull << tc.idx_bits) - 1));
}
__device__ __forceinline__ uint32_t key_idx(const TraceCtx& tc, uint64_t k) {
  return (uint32_t)((k >> tc.idx_bits) & ((1ull << tc.idx_bits) - 1));
}
__device__ __forceinline__ uint32_t key_bucket(const TraceCtx& tc, uint64_t k) {
  return (uint32_t)(k >> (2 * tc.idx_bits));
}
// first key of the bucket after k's (saturating at the last bucket, which the
// hit list then never claims to cover)
__device__ __forceinline__ uint64_t next_bucket_key(const TraceCtx& tc, uint64_t k) {
  const uint32_t b = key_bucket(tc, k);
  return make_key_b(tc, b < tc.max_bucket ? b + 1u : tc.max_bucket, 0u, 0u);
}
// smallest t that can carry the given key's bucket (for culling)
__device__ __forceinline__ float key_tlo(const TraceCtx& tc, uint64_t k) {
  const uint32_t b = (uint32_t)(k >> (2 * tc.idx_bits));
  if (tc.inv_dq > 0.0) return (float)((double)b * tc.dq);
  return __uint_as_float(b);
}
// largest t whose bucket does not exceed the key's bucket
__device__ __forceinline__ float key_thi(const TraceCtx& tc, uint64_t k) {
  const uint32_t b = (uint32_t)(k >> (2 * tc.idx_bits));
  if (tc.inv_dq > 0.0) return (float)((double)(b + 1u) * tc.dq);
  return __uint_as_float(b);
}

// ---------------------------------------------------------------------------
// Ray-surfel geometry on the tangent plane (Eq. 1). Decisions and blended
// quantities are evaluated in double precision: the local coordinates come
// from a difference of nearly equal distances, and float32 there would cost
// ~1e-5 in u at room scale, which the bounce point and direction then
// amplify. Every candidate takes the double-precision test, straight-line:
// a wave nearly always holds some candidate whose decision a float32
// evaluation could not settle, so a float screen in front of it only added
// instructions.
// ---------------------------------------------------------------------------
__device__ __forceinline__ Record load_record(const Record* recs, uint32_t pos) {
  const float4* p = reinterpret_cast<const float4*>(recs + pos);
  Record r;
  r.p_sigma = p[0];
  r.q = p[1];
  r.s_idx = p[2];
  return r;
}

__device__ __forceinline__ uint32_t rec_index(const Record& r) { return __float_as_uint(r.s_idx.z); }

// A surfel's geometry in double precision (Sec. 3.1), as the adjoint's chain
// rule needs it: centre p, tangent axes t_u, t_v = the first two columns of
// the rotation of q / |q|, normal n = t_u x t_v, scales, and the normalised
// quaternion.
struct Geo {
  D3 p, tu, tv, n;
  double su, sv, sigma;
  double qw, qx, qy, qz, iq;   // unit quaternion and 1 / |q|
};

__device__ __forceinline__ Geo surfel_geo(const Record& r) {
  Geo g;
  g.p = d3(r.p_sigma.x, r.p_sigma.y, r.p_sigma.z);
  g.sigma = r.p_sigma.w;
  double w = r.q.x, x = r.q.y, y = r.q.z, z = r.q.w;
  g.iq = 1.0 / sqrt(w * w + x * x + y * y + z * z);
  w *= g.iq; x *= g.iq; y *= g.iq; z *= g.iq;
  g.qw = w; g.qx = x; g.qy = y; g.qz = z;
  g.tu = d3(1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y + w * z), 2.0 * (x * z - w * y));
  g.tv = d3(2.0 * (x * y - w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z + w * x));
  g.n = cross(g.tu, g.tv);
  g.su = r.s_idx.x;
  g.sv = r.s_idx.y;
  return g;
}

// ---------------------------------------------------------------------------
// Segment result: the traced quantities of Eq. 3 before normalisation.
// ---------------------------------------------------------------------------
struct SegOut {
  D3 N;
  double D;
  D3 R;
  double E;
  D3 P;
  double T;
  int32_t nhits;
  int32_t rounds;
  int32_t tests;
  int32_t visits;
};

enum { Q_ALL = 0, Q_RADIANCE = 1 };

// Slab test of a box against [tlo, thi]; returns the entry distance or +inf.
// OiW = O * iW per component: each plane distance (l - O) / W is one fused
// multiply-add, l * iW - OiW. Its rounding error, in space, is a few ulp of
// |O| and |l|, far inside the pad that every leaf box carries around its
// ellipse, so no box that a ray's hit lies in is rejected.
__device__ __forceinline__ float slab(float lx, float ly, float lz, float hx, float hy, float hz, V3 OiW, V3 iW,
                                      float tlo, float thi) {
  const float ax = fmaf(lx, iW.x, -OiW.x), bx = fmaf(hx, iW.x, -OiW.x);
  const float ay = fmaf(ly, iW.y, -OiW.y), by = fmaf(hy, iW.y, -OiW.y);
  const float az = fmaf(lz, iW.z, -OiW.z), bz = fmaf(hz, iW.z, -OiW.z);
  const float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), tlo));
  // widen the exit so that rounding (and the float32 copy of the ray) never
  // rejects a box the ray touches
  const float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), thi)) * 1.000002f + 1e-6f;
  return tn <= tf ? tn : __builtin_inff();
}

// No per-hit callback (forward passes).
struct NoHit {
  __device__ __forceinline__ void operator()(uint32_t, double, double, double, double, D3, D3) const {}
};

// Traversal stack: the top STACK_LDS entries of every lane live in LDS,
// strided by the thread index so that a wave's pushes hit distinct banks;
// deeper entries (rare) spill to a private array.
constexpr int STACK_LDS = 24;
constexpr int TRACE_BLOCK = 256;   // every tracing kernel runs 256-thread blocks
constexpr int PEND = 32;           // postponed leaves per lane

// The overflow array is the caller's (a private array of the kernel): kept
// out of this struct so that the struct itself stays in registers.
constexpr int STACK_OVF = STACK_SIZE - STACK_LDS;
struct TravStack {
  int* lds;        // this lane's column: lds[i * TRACE_BLOCK]
  int* ovf;        // this lane's overflow entries, STACK_OVF of them
  int sp;
  __device__ __forceinline__ void push(int v) {
    if (sp < STACK_LDS) lds[sp * TRACE_BLOCK] = v;
    else ovf[sp - STACK_LDS] = v;
    ++sp;
  }
  __device__ __forceinline__ int pop() {
    --sp;
    if (sp < STACK_LDS) return lds[sp * TRACE_BLOCK];
    // volatile keeps the (rare) private read a load of its own, so that the
    // common LDS read is not merged with it into a generic-address load
    return static_cast<volatile int*>(ovf)[sp - STACK_LDS];
  }
};

// Accept a candidate key into the sorted k-buffer (ascending; empty = ~0):
// one compare-exchange per entry carries the larger key down the buffer.
// Returns the key that falls off the end (the old last entry, or the
// candidate itself when it is not below it).
__device__ __forceinline__ uint64_t kbuf_insert(uint64_t (&kk)[KBUF], uint64_t key) {
#pragma unroll
  for (int j = 0; j < KBUF; ++j) {
    const bool lt = key < kk[j];
    const uint64_t lo = lt ? key : kk[j];
    key = lt ? kk[j] : key;
    kk[j] = lo;
  }
  return key;
}

// Compare-exchange: afterwards a <= b.
__device__ __forceinline__ void cswap_key(uint64_t& a, uint64_t& b) {
  const bool lt = b < a;
  const uint64_t lo = lt ? b : a;
  b = lt ? a : b;
  a = lo;
}

// Sort eight keys ascending: the 19-comparator, depth-6 sorting network for
// eight inputs (checked on all 256 zero-one inputs).
__device__ __forceinline__ void sort8_keys(uint64_t (&e)[8]) {
  cswap_key(e[0], e[2]); cswap_key(e[1], e[3]); cswap_key(e[4], e[6]); cswap_key(e[5], e[7]);
  cswap_key(e[0], e[4]); cswap_key(e[1], e[5]); cswap_key(e[2], e[6]); cswap_key(e[3], e[7]);
  cswap_key(e[0], e[1]); cswap_key(e[2], e[3]); cswap_key(e[4], e[5]); cswap_key(e[6], e[7]);
  cswap_key(e[2], e[4]); cswap_key(e[3], e[5]);
  cswap_key(e[1], e[4]); cswap_key(e[3], e[6]);
  cswap_key(e[1], e[2]); cswap_key(e[3], e[4]); cswap_key(e[5], e[6]);
}

// Merge eight ascending keys into the k-buffer, keeping its KBUF smallest.
// Against the buffer's upper half, taken in reverse, the elementwise minimum
// leaves the sixteen smallest of both as a bitonic sequence, which four
// compare-exchange stages sort: 8 minima and 32 compare-exchanges in place
// of the 128 steps of eight single inserts.
static_assert(KBUF == 16, "the merge network is built for a 16-entry k-buffer");
__device__ __forceinline__ void kbuf_merge8(uint64_t (&kk)[KBUF], const uint64_t (&e)[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) kk[8 + i] = e[7 - i] < kk[8 + i] ? e[7 - i] : kk[8 + i];
#pragma unroll
  for (int st = 8; st >= 1; st >>= 1) {
#pragma unroll
    for (int i = 0; i < KBUF; ++i)
      if ((i & st) == 0) cswap_key(kk[i], kk[i + st]);
  }
}

// ---------------------------------------------------------------------------
// One ray segment: multi-round k-buffer traversal and front-to-back blending.
// Round r collects the KBUF smallest keys strictly greater than the last key
// blended in round r-1, blends them in order, and stops the segment after the
// first hit with T < T_min, or when a round returns fewer than KBUF hits.
//
// With a hit list (tc.hl), a traversal round also records every accepted key
// that the k-buffer rejects or evicts and whose depth bucket does not exceed
// that of the round's KBUF-th key. Such a round has tested every surfel of
// those buckets (boxes are culled only beyond them), so after blending the
// round the list holds every hit key in (last, lhi) with lhi the first key
// of the next bucket. A later round takes its keys from the
// list when it finds KBUF of them there, and otherwise traverses only for
// keys >= lhi; when the list holds some but fewer than KBUF such keys, they
// are blended first as a round of their own, and the traversal beyond lhi
// happens only if the segment is still open. On a surface where many
// coplanar surfels share one depth
// bucket, this turns the repeated traversals of a long segment into scans
// of a short list. If the list overflows it is dropped and rounds traverse.
//
// The steps are separate functions so that a kernel can interleave them
// across lanes (the path tracer does); trace_segment_cb runs them in order.
// ---------------------------------------------------------------------------

// Segment state carried across rounds. DACC: accumulate R, E, P in double
// (the single-bounce render, whose adjoint subtracts running prefixes from
// these totals) or in float (path tracing).
template <bool DACC>
struct Seg {
  using Acc = typename std::conditional<DACC, double, float>::type;
  D3 O, W;            // the ray, double precision
  V3 OiW;             // float origin times iW, for the slab tests
  V3 iW;              // float reciprocal direction for the box tests
  D3 N;
  double D, T;
  Acc R0, R1, R2, E, P0, P1, P2;
  uint64_t last;      // keys must exceed this once have_last
  bool have_last;
  bool done;
  int nl;             // entries in the hit list
  uint64_t lhi;       // 0: list unusable; else it holds every hit key in (last, lhi)
  int32_t nhits, rounds, tests, visits;
};

// State of one round: the k-buffer and the traversal. Internal nodes are
// visited until a lane has PEND-4 leaves postponed, its traversal ends, or
// every lane of the wave has a leaf waiting; then the postponed leaves are
// tested, so that the costly surfel test runs for many lanes at once.
struct Round {
  uint64_t kk[KBUF];  // ascending; empty = ~0
  int cnt;
  uint64_t floor_key; // keys taken must exceed this (when have_floor)
  bool have_floor;
  uint64_t cut_key;   // hit list entries must be below this
  float t_cut;        // boxes entered beyond this cannot hold a key < kk[KBUF-1]
  float tlo0;         // boxes ending before this cannot hold a key > floor_key
  bool over;          // the hit list overflowed this round
  bool partial;       // list keys below lhi only: blend them, then traverse beyond lhi if still open
  uint64_t plast;     // largest key of a partial round
  bool trav;          // internal nodes remain (ref, then the stack)
  int ref;            // next internal node
  int np;             // postponed leaves
};

template <bool DACC>
__device__ __forceinline__ void seg_begin(Seg<DACC>& s, D3 O, D3 W) {
  s.O = O;
  s.W = W;
  const float wx = (float)W.x, wy = (float)W.y, wz = (float)W.z;
  s.iW = v3(1.0f / (fabsf(wx) > 1e-30f ? wx : copysignf(1e-30f, wx)),
            1.0f / (fabsf(wy) > 1e-30f ? wy : copysignf(1e-30f, wy)),
            1.0f / (fabsf(wz) > 1e-30f ? wz : copysignf(1e-30f, wz)));
  s.OiW = v3((float)O.x * s.iW.x, (float)O.y * s.iW.y, (float)O.z * s.iW.z);
  s.N = d3(0.0, 0.0, 0.0);
  s.D = 0.0;
  s.T = 1.0;
  s.R0 = s.R1 = s.R2 = s.E = s.P0 = s.P1 = s.P2 = 0;
  s.last = 0;
  s.have_last = false;
  s.done = false;
  s.nl = 0;
  s.lhi = 0;
  s.nhits = s.rounds = s.tests = s.visits = 0;
}

// Start a round. Returns true when it must traverse (r.trav / r.np are set
// up and the stack is empty), false when the hit list alone decides it.
template <bool DACC>
__device__ __forceinline__ bool round_begin(const TraceCtx& tc, Seg<DACC>& s, Round& r, TravStack& st, int* pend) {
  ++s.rounds;
#pragma unroll
  for (int j = 0; j < KBUF; ++j) r.kk[j] = ~0ull;
  r.cnt = 0;
  r.floor_key = s.last;
  r.have_floor = s.have_last;
  r.over = false;
  r.partial = false;
  bool traverse = true;
  if (s.lhi != 0) {
    // keys in (last, lhi) from the list (entries at or below last were
    // blended by earlier rounds and are skipped, not removed)
    // (loaded 8 at a time: entries up to HL_CAP are this lane's, those past
    // nl are ignored)
    const uint64_t* const hl = tc.hl;
    int w = 0;
    for (int j = 0; j < s.nl; j += 8) {
      uint64_t e[8];
#pragma unroll
      for (int u = 0; u < 8; u += 2) {
        const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(hl + j + u);
        e[u] = v.x;
        e[u + 1] = v.y;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        // branch-free: a key outside (last, lhi) enters the merge as ~0
        const bool in = j + u < s.nl && e[u] > s.last && e[u] < s.lhi;
        e[u] = in ? e[u] : ~0ull;
        w += in ? 1 : 0;
      }
      sort8_keys(e);
      kbuf_merge8(r.kk, e);
    }
    if (w == 0) s.nl = 0;
    // every key in range is below the buffer's last entry until it is full
    r.cnt = w > KBUF ? KBUF : w;
    r.plast = 0;
#pragma unroll
    for (int j = 0; j < KBUF; ++j) r.plast = j < r.cnt ? r.kk[j] : r.plast;
    if (r.cnt == KBUF || s.lhi == ~0ull) {
      traverse = false;
    } else if (r.cnt > 0) {
      // Every key >= lhi follows these, so they can be blended first; the
      // segment often ends among them, and then nothing beyond lhi is needed.
      traverse = false;
      r.partial = true;
    } else if (s.lhi - 1 > r.floor_key) {
      r.floor_key = s.lhi - 1;
      r.have_floor = true;
    }
  } else {
    s.nl = 0;
  }
  r.cut_key = r.cnt == KBUF ? next_bucket_key(tc, r.kk[KBUF - 1]) : ~0ull;
  r.t_cut = r.cnt == KBUF ? key_thi(tc, r.kk[KBUF - 1]) * 1.000002f + 1e-6f : __builtin_inff();
  const float t_floor = r.have_floor ? key_tlo(tc, r.floor_key) : 0.0f;
  r.tlo0 = fmaxf((float)tc.t_min, t_floor) * 0.99999f - 1e-6f;
  st.sp = 0;
  r.ref = tc.root;
  r.np = 0;
  r.trav = traverse && tc.root >= 0;
  if (traverse && tc.root < 0) {   // the whole scene is one surfel
    pend[0] = ~tc.root;
    r.np = 1;
  }
  return traverse;
}

// Visit internal node r.ref: leaves the ray reaches are postponed, internal
// children are visited nearest first (the others pushed farthest first).
template <bool DACC>
__device__ __forceinline__ void node_visit(const TraceCtx& tc, Seg<DACC>& s, Round& r, TravStack& st, int* pend) {
  ++s.visits;
  const Node4* nd = tc.nodes + r.ref;
  const int4 cr = nd->ref;
  const float4* bb = nd->b;
  const float4 b0 = bb[0], b1 = bb[1], b2 = bb[2], b3 = bb[3], b4 = bb[4], b5 = bb[5];
  float e[4];
  e[0] = slab(b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, s.OiW, s.iW, r.tlo0, r.t_cut);
  e[1] = slab(b1.z, b1.w, b2.x, b2.y, b2.z, b2.w, s.OiW, s.iW, r.tlo0, r.t_cut);
  e[2] = slab(b3.x, b3.y, b3.z, b3.w, b4.x, b4.y, s.OiW, s.iW, r.tlo0, r.t_cut);
  e[3] = slab(b4.z, b4.w, b5.x, b5.y, b5.z, b5.w, s.OiW, s.iW, r.tlo0, r.t_cut);
  const int c[4] = {cr.x, cr.y, cr.z, cr.w};
  float ie[4];
  int ic[4];
  int ni = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    // a missed box reports +inf (the slab test already holds the entry to the
    // widened cut), which must not pass while the cut is infinite
    const bool m = c[k] != NODE4_EMPTY && e[k] < __builtin_inff();
    // leaves are queued without a branch: the slot past the queue is always
    // written (nodes are visited only while np <= PEND - 4, so it exists)
    pend[r.np * TRACE_BLOCK] = ~c[k];
    r.np += (m && c[k] < 0) ? 1 : 0;
    ie[k] = (m && c[k] >= 0) ? e[k] : __builtin_inff();
    ic[k] = c[k];
    ni += (m && c[k] >= 0) ? 1 : 0;
  }
  if (ni > 0) {
    // sort the four (entry, child) pairs by entry, misses (+inf) last
#define EAG_CSWAP(i, j)                                  \
    if (ie[j] < ie[i]) {                                 \
      const float tf = ie[i]; ie[i] = ie[j]; ie[j] = tf; \
      const int tc_ = ic[i]; ic[i] = ic[j]; ic[j] = tc_; \
    }
    EAG_CSWAP(0, 1) EAG_CSWAP(2, 3) EAG_CSWAP(0, 2) EAG_CSWAP(1, 3) EAG_CSWAP(1, 2)
#undef EAG_CSWAP
    // push the others farthest first: bottom to top ic[ni-1] .. ic[1]
    if (st.sp + 3 <= STACK_LDS) {
      // branch-free: three slots written, the stack grows by ni - 1
      const int v0 = ni > 3 ? ic[3] : (ni > 2 ? ic[2] : ic[1]);
      const int v1 = ni > 3 ? ic[2] : ic[1];
      st.lds[(st.sp + 0) * TRACE_BLOCK] = v0;
      st.lds[(st.sp + 1) * TRACE_BLOCK] = v1;
      st.lds[(st.sp + 2) * TRACE_BLOCK] = ic[1];
      st.sp += ni - 1;
    } else {
      if (ni > 3) st.push(ic[3]);
      if (ni > 2) st.push(ic[2]);
      if (ni > 1) st.push(ic[1]);
    }
    r.ref = ic[0];
  } else if (st.sp > 0) {
    r.ref = st.pop();
  } else {
    r.trav = false;
  }
}

// The order key of a postponed leaf (its record already loaded) for the ray
// (O, W) in a round whose keys must exceed floor_key (when have_floor); ~0
// when the surfel is missed or its key cannot enter the round. cutlim: keys
// at or above it are dropped (the k-buffer's last key, or the hit list's
// cut, a bucket's first key; any larger value is also correct).
__device__ __forceinline__ uint64_t leaf_key(const TraceCtx& tc, const Record& rec, uint32_t pos, D3 O, D3 W,
                                             bool have_floor, uint64_t floor_key, uint64_t cutlim) {
  // The surfel test in double precision, straight-line. The columns of the
  // rotation of the unnormalised quaternion are |q|^2 (t_u, t_v, n): the
  // distance t = ((p - O).n) / (W.n) needs no normalisation, and the ellipse
  // test becomes u'^2 / s_u^2 + v'^2 / s_v^2 <= k^2 |q|^4 with
  // u' = y.(|q|^2 t_u). Its rounding differs from the normalised evaluation
  // by a few ulp, well inside the margins within which rim, t_min and bucket
  // decisions are flagged.
  const double w = rec.q.x, x = rec.q.y, y = rec.q.z, z = rec.q.w;
  const double q2n = w * w + x * x + y * y + z * z;
  const D3 cu = d3(w * w + x * x - y * y - z * z, 2.0 * (x * y + w * z), 2.0 * (x * z - w * y));
  const D3 cv = d3(2.0 * (x * y - w * z), w * w - x * x + y * y - z * z, 2.0 * (y * z + w * x));
  const D3 cn = d3(2.0 * (x * z + w * y), 2.0 * (y * z - w * x), w * w - x * x - y * y + z * z);
  const D3 d = d3((double)rec.p_sigma.x - O.x, (double)rec.p_sigma.y - O.y, (double)rec.p_sigma.z - O.z);
  const double den = dot(W, cn);
  const double t = dot(d, cn) / den;
  const D3 yv = d3(t * W.x - d.x, t * W.y - d.y, t * W.z - d.z);
  const double su2 = (double)rec.s_idx.x * rec.s_idx.x, sv2 = (double)rec.s_idx.y * rec.s_idx.y;
  const double up = dot(yv, cu), vp = dot(yv, cv);
  // (multiplied through by s_u^2 s_v^2, all positive: no division)
  const bool hit = fabs(den) > 1e-12 * q2n && rec.p_sigma.w > 0.0f && t > tc.t_min &&
                   up * up * sv2 + vp * vp * su2 <= tc.k2 * q2n * q2n * su2 * sv2;
  const uint64_t key = make_key(tc, t, rec_index(rec), pos);
  const bool qual = hit && !(have_floor && key <= floor_key);
  // A hit in the last bucket may stand for a farther one that the key
  // saturated into it, whose order among the others is then unknown: the
  // launch reports it (a rare branch; never taken within the range).
  if (qual && tc.inv_dq > 0.0 && key_bucket(tc, key) >= tc.max_bucket) report_key_range(tc.status);
  return qual && key < cutlim ? key : ~0ull;
}

// Take a qualifying key into the round. The list needs only keys beyond the
// round's final KBUF-th key: a key goes there when the k-buffer rejects it
// or later evicts it.
template <bool DACC>
__device__ __forceinline__ void take_key(const TraceCtx& tc, Seg<DACC>& s, Round& r, uint64_t key) {
  // The insert runs without a branch: a key not below the last entry passes
  // through the chain unchanged and comes back as the spill.
  const bool ins = key < r.kk[KBUF - 1];
  const uint64_t spill = kbuf_insert(r.kk, key);   // ~0 while the buffer is not full
  r.cnt += ins ? 1 : 0;
  if (ins && r.cnt >= KBUF) {
    r.cnt = KBUF;
    r.t_cut = key_thi(tc, r.kk[KBUF - 1]) * 1.000002f + 1e-6f;
    r.cut_key = next_bucket_key(tc, r.kk[KBUF - 1]);
  }
  if (tc.hl && spill < r.cut_key) {
    if (s.nl < HL_CAP) tc.hl[(s.nl++) * HL_STRIDE] = spill;
    else r.over = true;
  }
}

template <bool DACC>
__device__ __forceinline__ uint64_t round_cutlim(const TraceCtx& tc, const Round& r) {
  return tc.hl ? r.cut_key : r.kk[KBUF - 1];
}

// Test one postponed leaf of this lane's own ray and take its key.
template <bool DACC>
__device__ __forceinline__ void leaf_eval(const TraceCtx& tc, Seg<DACC>& s, Round& r, const Record& rec,
                                          uint32_t pos) {
  ++s.tests;
  const uint64_t key = leaf_key(tc, rec, pos, s.O, s.W, r.have_floor, r.floor_key, round_cutlim<DACC>(tc, r));
  if (key != ~0ull) take_key(tc, s, r, key);
}

// Test postponed leaves, most recent first. The next leaf's record is loaded
// before the current one is tested, so that its latency overlaps the test's
// arithmetic. A lane whose traversal continues stops once fewer than
// LEAF_MIN_LANES lanes of the wave still hold leaves, and keeps the rest for
// its next leaf phase; a lane whose traversal has ended tests all of them.
constexpr int LEAF_MIN_LANES = 16;
template <bool DACC>
__device__ __forceinline__ void leaf_phase(const TraceCtx& tc, Seg<DACC>& s, Round& r, int* pend) {
  if (r.np <= 0) return;
  uint32_t pos = (uint32_t)pend[(--r.np) * TRACE_BLOCK];
  Record rec = load_record(tc.recs, pos);
  while (true) {
    const bool more = r.np > 0 && !(r.trav && __popcll(__ballot(r.np > 0)) < LEAF_MIN_LANES);
    uint32_t npos = 0;
    Record nrec;
    if (more) {
      npos = (uint32_t)pend[(--r.np) * TRACE_BLOCK];
      nrec = load_record(tc.recs, npos);
    }
    leaf_eval(tc, s, r, rec, pos);
    if (!more) break;
    pos = npos;
    rec = nrec;
  }
}

// After a traversal round: what the hit list now covers.
template <bool DACC>
__device__ __forceinline__ void round_end_traversal(const TraceCtx& tc, Seg<DACC>& s, const Round& r) {
  if (tc.hl) s.lhi = r.over ? 0ull : (r.cnt == KBUF ? r.cut_key : ~0ull);
}

// Traverse one round to completion for this lane.
template <bool DACC>
__device__ __forceinline__ void traverse_round(const TraceCtx& tc, Seg<DACC>& s, Round& r, TravStack& st,
                                               int* pend) {
  while (true) {
    while (r.trav && r.np <= PEND - 4) {
      node_visit(tc, s, r, st, pend);
      if (__all(r.np > 0 || !r.trav)) break;
    }
    leaf_phase(tc, s, r, pend);
    if (!r.trav) break;
  }
  round_end_traversal(tc, s, r);
}

// Blend the round's hits in key order (the buffer is shifted down one entry
// per hit, which keeps its indexing static); t and alpha are recomputed from
// the record with the same double-precision test. Sets s.done after the
// first hit with T < T_min or when the round returned fewer than KBUF hits.
// on_hit(pos, t, alpha, w, T_before, O, W) is called for every blended hit; if
// hit_out is non-null, up to max_hits blended surfel indices are written.
template <int QMODE, bool DACC, class HitFn>
__device__ __forceinline__ void blend_round(const TraceCtx& tc, Seg<DACC>& s, Round& r, HitFn& on_hit,
                                           int32_t* hit_out, int max_hits) {
  using Acc = typename Seg<DACC>::Acc;
  const uint64_t round_last = r.partial ? r.plast : r.kk[KBUF - 1];
  // the next hit's record and attributes are loaded while the current one
  // is blended
  Record rec;
  Attr at;
  if (r.cnt > 0) {
    const uint32_t p0 = key_pos(tc, r.kk[0]);
    rec = load_record(tc.recs, p0);
    at = tc.attrs[p0];
  }
  for (int j = 0; j < r.cnt && !s.done; ++j) {
    const uint64_t key = r.kk[0];
#pragma unroll
    for (int m = 0; m < KBUF - 1; ++m) r.kk[m] = r.kk[m + 1];
    const uint32_t pos = key_pos(tc, key);
    Record nrec;
    Attr nat;
    if (j + 1 < r.cnt) {
      const uint32_t np = key_pos(tc, r.kk[0]);
      nrec = load_record(tc.recs, np);
      nat = tc.attrs[np];
    }
    // t, u, v and the unit normal from the columns of the unnormalised
    // quaternion's rotation, |q|^2 (t_u, t_v, n): no square root, and one
    // reciprocal c = 1 / (|q|^2 s_u s_v) for u^2 + v^2 and the normal's scale
    const double qw = rec.q.x, qx = rec.q.y, qy = rec.q.z, qz = rec.q.w;
    const double su = rec.s_idx.x, sv = rec.s_idx.y;
    const double c = 1.0 / ((qw * qw + qx * qx + qy * qy + qz * qz) * (su * sv));
    const double iq2 = c * (su * sv);
    const D3 cu = d3(qw * qw + qx * qx - qy * qy - qz * qz, 2.0 * (qx * qy + qw * qz), 2.0 * (qx * qz - qw * qy));
    const D3 cv = d3(2.0 * (qx * qy - qw * qz), qw * qw - qx * qx + qy * qy - qz * qz, 2.0 * (qy * qz + qw * qx));
    const D3 cn = d3(2.0 * (qx * qz + qw * qy), 2.0 * (qy * qz - qw * qx), qw * qw - qx * qx - qy * qy + qz * qz);
    const D3 dp = d3((double)rec.p_sigma.x - s.O.x, (double)rec.p_sigma.y - s.O.y, (double)rec.p_sigma.z - s.O.z);
    const double dn = dot(s.W, cn);
    const double t = dot(dp, cn) / dn;
    const D3 yv = d3(t * s.W.x - dp.x, t * s.W.y - dp.y, t * s.W.z - dp.z);
    const double uc = dot(yv, cu) * sv, vc = dot(yv, cv) * su;   // u, v times |q|^2 s_u s_v
    const double a = (double)rec.p_sigma.w * exp(-0.5 * ((uc * uc + vc * vc) * (c * c)));
    const double w = s.T * a;
    const Acc wf = (Acc)w;
    if (QMODE == Q_ALL) {
      const double sw = (dn > 0.0 ? -w : w) * iq2;  // n' faces the origin
      s.N.x += sw * cn.x;
      s.N.y += sw * cn.y;
      s.N.z += sw * cn.z;
      s.D += w * t;
      s.P0 += wf * at.rho_e.x;
      s.P1 += wf * at.rho_e.y;
      s.P2 += wf * at.rho_e.z;
      s.E += wf * at.rho_e.w;
    }
    s.R0 += wf * at.r.x;
    s.R1 += wf * at.r.y;
    s.R2 += wf * at.r.z;
    if (hit_out && s.nhits < max_hits) hit_out[s.nhits] = (int32_t)key_idx(tc, key);
    on_hit(pos, t, a, w, s.T, s.O, s.W);
    ++s.nhits;
    s.T *= (1.0 - a);
    if (s.T < tc.T_min) s.done = true;
    rec = nrec;
    at = nat;
  }
  if (r.cnt < KBUF && !r.partial) s.done = true;
  if (!s.done) {
    s.last = round_last;
    s.have_last = true;
  }
}

// A whole segment for this lane. Must be called from a TRACE_BLOCK-thread
// block (the traversal stack and the postponed leaves live in LDS).
template <int QMODE, bool DACC, class HitFn>
__device__ SegOut trace_segment_cb(const TraceCtx& tc, D3 O, D3 W, HitFn& on_hit, int32_t* hit_out = nullptr,
                                   int max_hits = 0) {
  __shared__ int s_stack[STACK_LDS * TRACE_BLOCK];
  __shared__ int s_pend[PEND * TRACE_BLOCK];
  int s_ovf[STACK_OVF];
  TravStack st;
  st.lds = s_stack + threadIdx.x;
  st.ovf = s_ovf;
  st.sp = 0;
  int* pend = s_pend + threadIdx.x;   // this lane's queue of postponed leaves
  Seg<DACC> s;
  seg_begin(s, O, W);
  while (!s.done) {
    Round r;
    if (round_begin(tc, s, r, st, pend)) traverse_round(tc, s, r, st, pend);
    blend_round<QMODE>(tc, s, r, on_hit, hit_out, max_hits);
  }
  SegOut o;
  o.N = s.N;
  o.D = s.D;
  o.R = d3(s.R0, s.R1, s.R2);
  o.E = s.E;
  o.P = d3(s.P0, s.P1, s.P2);
  o.T = s.T;
  o.nhits = s.nhits;
  o.rounds = s.rounds;
  o.tests = s.tests;
  o.visits = s.visits;
  return o;
}

template <int QMODE, bool DACC = false>
__device__ __forceinline__ SegOut trace_segment(const TraceCtx& tc, D3 O, D3 W, int32_t* hit_out = nullptr,
                                                int max_hits = 0) {
  NoHit nh;
  return trace_segment_cb<QMODE, DACC>(tc, O, W, nh, hit_out, max_hits);
}

}  // namespace eag

#include "eag_internal.h"
namespace eag {
TraceCtx make_ctx(const eag_bvh* b, const Attr* attrs, const eag_trace_params* p, const TraceSetup& ts);
}  // namespace eag
