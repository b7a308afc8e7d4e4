// Device-side building blocks shared by the build, trace, render and path
// tracing kernels: Philox4x32-10, camera rays, the hemisphere frame and
// cosine-weighted sampling, the BVH node and surfel record layouts, and the
// per-ray traversal + k-buffer + compositing core.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eag {

constexpr int KBUF = 16;          // k-buffer depth
constexpr int STACK_SIZE = 64;    // traversal stack; builds deeper than this are rejected on the host

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

// Geometry record of one surfel in sorted order, 64 B (one float4 load each):
//   p.x p.y p.z sigma | n.x n.y n.z index | a_u.x a_u.y a_u.z s_u | a_v.x a_v.y a_v.z s_v
// with n = t_u x t_v, a_u = t_u / s_u, a_v = t_v / s_v, index = original surfel index.
struct __align__(16) Record {
  float4 p_sigma;
  float4 n_idx;
  float4 au;
  float4 av;
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

// Pinhole camera prepared on the host (double precision, rounded once):
// ray direction = normalize(dx * right + dy * up + fwd) with
// dx = 2 (x + ox) / W - 1, dy = 1 - 2 (y + oy) / H; right and up are
// pre-scaled by tan(vfov/2) * W/H and tan(vfov/2).
struct CamDev {
  float eye[3], right[3], up[3], fwd[3];
  int32_t width, height;
  uint32_t id;
  int32_t pad;
};

__device__ __forceinline__ V3 camera_dir(const CamDev& c, int px, int py, float ox, float oy) {
  const float dx = 2.0f * ((float)px + ox) / (float)c.width - 1.0f;
  const float dy = 1.0f - 2.0f * ((float)py + oy) / (float)c.height;
  V3 d = v3(dx * c.right[0] + dy * c.up[0] + c.fwd[0], dx * c.right[1] + dy * c.up[1] + c.fwd[1],
            dx * c.right[2] + dy * c.up[2] + c.fwd[2]);
  const float inv = 1.0f / sqrtf(dot(d, d));
  return inv * d;
}

// Hemisphere frame: Gram-Schmidt of the fixed helper h = (1,2,3)/sqrt(14)
// against the unit normal n: b1 = normalize(h - (h.n) n), b2 = n x b1.
// Cosine-weighted direction (Malley): r = sqrt(u0), phi = 2 pi u1,
// w' = r cos(phi) b1 + r sin(phi) b2 + sqrt(1 - u0) n.
constexpr float HX = 0.2672612419124244f, HY = 0.5345224838248488f, HZ = 0.8017837257372732f;

__device__ __forceinline__ V3 cosine_dir(V3 n, float u0, float u1) {
  const float hn = HX * n.x + HY * n.y + HZ * n.z;
  V3 m = v3(HX - hn * n.x, HY - hn * n.y, HZ - hn * n.z);
  const float il = 1.0f / sqrtf(dot(m, m));
  const V3 b1 = il * m;
  const V3 b2 = cross(n, b1);
  const float r = sqrtf(u0);
  float s, c;
  sincosf(6.283185307179586f * u1, &s, &c);
  const float z = sqrtf(1.0f - u0);
  return v3(r * c * b1.x + r * s * b2.x + z * n.x, r * c * b1.y + r * s * b2.y + z * n.y,
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
  const Node* nodes;
  const Record* recs;
  const Attr* attrs;
  int32_t root;            // >= 0: internal node index; < 0: single leaf ~root
  int32_t idx_bits;        // bits of an index (both index fields)
  uint32_t max_bucket;     // largest representable bucket
  float inv_dq;            // 1 / dq, or 0 for exact-t keys
  float t_min;
  float k2;                // k_sigma^2
  float T_min;
};

__device__ __forceinline__ uint64_t make_key(const TraceCtx& tc, float t, uint32_t idx, uint32_t pos) {
  uint32_t bucket;
  if (tc.inv_dq > 0.0f) {
    const float b = floorf(t * tc.inv_dq);
    bucket = b >= (float)tc.max_bucket ? tc.max_bucket : (uint32_t)b;
  } else {
    bucket = __float_as_uint(t);
  }
  return ((uint64_t)bucket << (2 * tc.idx_bits)) | ((uint64_t)idx << tc.idx_bits) | (uint64_t)pos;
}
__device__ __forceinline__ uint32_t key_pos(const TraceCtx& tc, uint64_t k) {
  return (uint32_t)(k & ((1ull << tc.idx_bits) - 1));
}
__device__ __forceinline__ uint32_t key_idx(const TraceCtx& tc, uint64_t k) {
  return (uint32_t)((k >> tc.idx_bits) & ((1ull << tc.idx_bits) - 1));
}
// smallest t that can carry the given key's bucket (for culling), conservative
__device__ __forceinline__ float key_tlo(const TraceCtx& tc, uint64_t k) {
  const uint32_t b = (uint32_t)(k >> (2 * tc.idx_bits));
  if (tc.inv_dq > 0.0f) return (float)b / tc.inv_dq;
  return __uint_as_float(b);
}
// largest t whose bucket does not exceed the key's bucket
__device__ __forceinline__ float key_thi(const TraceCtx& tc, uint64_t k) {
  const uint32_t b = (uint32_t)(k >> (2 * tc.idx_bits));
  if (tc.inv_dq > 0.0f) return (float)(b + 1u) / tc.inv_dq;
  return __uint_as_float(b);
}

// ---------------------------------------------------------------------------
// Ray-surfel test on the tangent plane (Eq. 1): returns true and (t, alpha)
// when accepted.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool surfel_test(const Record& r, V3 O, V3 W, float t_min, float k2, float& t,
                                            float& alpha) {
  const V3 d = v3(r.p_sigma.x - O.x, r.p_sigma.y - O.y, r.p_sigma.z - O.z);
  const V3 n = v3(r.n_idx.x, r.n_idx.y, r.n_idx.z);
  const float den = dot(W, n);
  const float num = dot(d, n);
  if (!(fabsf(den) > 1e-12f) || !(r.p_sigma.w > 0.0f)) return false;
  t = num / den;
  if (!(t > t_min)) return false;
  const V3 y = v3(t * W.x - d.x, t * W.y - d.y, t * W.z - d.z);
  const float u = y.x * r.au.x + y.y * r.au.y + y.z * r.au.z;
  const float v = y.x * r.av.x + y.y * r.av.y + y.z * r.av.z;
  const float q2 = u * u + v * v;
  if (!(q2 <= k2)) return false;
  alpha = r.p_sigma.w * expf(-0.5f * q2);
  return true;
}

__device__ __forceinline__ Record load_record(const Record* recs, uint32_t pos) {
  const float4* p = reinterpret_cast<const float4*>(recs + pos);
  Record r;
  r.p_sigma = p[0];
  r.n_idx = p[1];
  r.au = p[2];
  r.av = p[3];
  return r;
}

// ---------------------------------------------------------------------------
// Segment result: the traced quantities of Eq. 3 before normalisation.
// ---------------------------------------------------------------------------
struct SegOut {
  V3 N;
  float D;
  V3 R;
  float E;
  V3 P;
  float T;
  int32_t nhits;
  int32_t rounds;
  int32_t tests;
};

enum { Q_ALL = 0, Q_RADIANCE = 1 };

// Slab test of a box against [tlo, thi]; returns the entry distance or +inf.
__device__ __forceinline__ float slab(float lx, float ly, float lz, float hx, float hy, float hz, V3 O, V3 iW,
                                      float tlo, float thi) {
  const float ax = (lx - O.x) * iW.x, bx = (hx - O.x) * iW.x;
  const float ay = (ly - O.y) * iW.y, by = (hy - O.y) * iW.y;
  const float az = (lz - O.z) * iW.z, bz = (hz - O.z) * iW.z;
  const float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), tlo));
  // widen the exit by 2*gamma(3) so that rounding never rejects a box the ray touches
  const float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), thi)) * 1.0000004f;
  return tn <= tf ? tn : __builtin_inff();
}

// One ray segment: multi-round k-buffer traversal and front-to-back blending.
// Round r collects the KBUF smallest keys strictly greater than the last key
// blended in round r-1, blends them in order, and stops the segment after the
// first hit with T < T_min, or when a round returns fewer than KBUF hits.
// If hit_out is non-null, up to max_hits blended surfel indices are written.
template <int QMODE>
__device__ SegOut trace_segment(const TraceCtx& tc, V3 O, V3 W, int32_t* hit_out = nullptr, int max_hits = 0) {
  SegOut o;
  o.N = v3(0.f, 0.f, 0.f);
  o.D = 0.f;
  o.R = v3(0.f, 0.f, 0.f);
  o.E = 0.f;
  o.P = v3(0.f, 0.f, 0.f);
  o.T = 1.0f;
  o.nhits = 0;
  o.rounds = 0;
  o.tests = 0;
  const V3 iW = v3(1.0f / (fabsf(W.x) > 1e-30f ? W.x : copysignf(1e-30f, W.x)),
                   1.0f / (fabsf(W.y) > 1e-30f ? W.y : copysignf(1e-30f, W.y)),
                   1.0f / (fabsf(W.z) > 1e-30f ? W.z : copysignf(1e-30f, W.z)));
  uint64_t last = 0;            // keys must exceed this (0 is below every valid key: t > 0)
  bool have_last = false;
  float t_floor = 0.0f;         // boxes ending before this cannot hold a key > last
  bool done = false;
  while (!done) {
    uint64_t kk[KBUF];
    float kt[KBUF], ka[KBUF];
#pragma unroll
    for (int j = 0; j < KBUF; ++j) { kk[j] = ~0ull; kt[j] = 0.f; ka[j] = 0.f; }
    int cnt = 0;
    float t_cut = __builtin_inff();   // boxes entered after this cannot hold a key < kk[KBUF-1]

    int stack[STACK_SIZE];
    float stack_t[STACK_SIZE];
    int sp = 0;
    int ref = tc.root;
    const float tlo0 = fmaxf(tc.t_min, t_floor) * 0.99999f - 1e-7f;
    while (true) {
      if (ref >= 0) {
        const Node nd = tc.nodes[ref];
        const float thi = t_cut;
        const float tlo = tlo0;
        float e0 = slab(nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, O, iW, tlo, thi);
        float e1 = slab(nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, O, iW, tlo, thi);
        const int c0 = nd.d.x, c1 = nd.d.y;
        // leaf children are tested right away
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          const int c = side ? c1 : c0;
          const float e = side ? e1 : e0;
          if (c < 0 && e < __builtin_inff()) {
            const uint32_t pos = (uint32_t)(~c);
            const Record r = load_record(tc.recs, pos);
            float t, a;
            ++o.tests;
            if (surfel_test(r, O, W, tc.t_min, tc.k2, t, a)) {
              const uint64_t key = make_key(tc, t, __float_as_uint(r.n_idx.w), pos);
              if ((!have_last || key > last) && key < kk[KBUF - 1]) {
                uint64_t ck = key;
                float ct = t, ca = a;
#pragma unroll
                for (int j = 0; j < KBUF; ++j) {
                  const bool sw = ck < kk[j];
                  const uint64_t tk = kk[j];
                  const float tt = kt[j], ta = ka[j];
                  kk[j] = sw ? ck : tk;
                  kt[j] = sw ? ct : tt;
                  ka[j] = sw ? ca : ta;
                  ck = sw ? tk : ck;
                  ct = sw ? tt : ct;
                  ca = sw ? ta : ca;
                }
                if (++cnt >= KBUF) {
                  cnt = KBUF;
                  t_cut = key_thi(tc, kk[KBUF - 1]) * 1.000001f + 1e-6f;
                }
              }
            }
          }
        }
        const bool h0 = c0 >= 0 && e0 <= t_cut;
        const bool h1 = c1 >= 0 && e1 <= t_cut;
        if (h0 && h1) {
          const bool first0 = e0 <= e1;
          if (sp < STACK_SIZE) {
            stack[sp] = first0 ? c1 : c0;
            stack_t[sp] = first0 ? e1 : e0;
            ++sp;
          }
          ref = first0 ? c0 : c1;
          continue;
        }
        if (h0) { ref = c0; continue; }
        if (h1) { ref = c1; continue; }
      } else {
        // the whole scene is one surfel
        const uint32_t pos = (uint32_t)(~ref);
        const Record r = load_record(tc.recs, pos);
        float t, a;
        ++o.tests;
        if (surfel_test(r, O, W, tc.t_min, tc.k2, t, a)) {
          const uint64_t key = make_key(tc, t, __float_as_uint(r.n_idx.w), pos);
          if (!have_last || key > last) { kk[0] = key; kt[0] = t; ka[0] = a; cnt = 1; }
        }
      }
      // pop, skipping entries that the tightened cut now excludes
      bool got = false;
      while (sp > 0) {
        --sp;
        if (stack_t[sp] <= t_cut) { ref = stack[sp]; got = true; break; }
      }
      if (!got) break;
    }
    ++o.rounds;

    // blend this round's hits in key order
#pragma unroll
    for (int j = 0; j < KBUF; ++j) {
      if (j < cnt && !done) {
        const uint32_t pos = key_pos(tc, kk[j]);
        const float a = ka[j];
        const float w = o.T * a;
        if (QMODE == Q_ALL) {
          const float4 nr = reinterpret_cast<const float4*>(tc.recs + pos)[1];
          const float s = (W.x * nr.x + W.y * nr.y + W.z * nr.z) > 0.0f ? -w : w;  // n' faces the origin
          o.N.x += s * nr.x;
          o.N.y += s * nr.y;
          o.N.z += s * nr.z;
          o.D += w * kt[j];
          const Attr at = tc.attrs[pos];
          o.P.x += w * at.rho_e.x;
          o.P.y += w * at.rho_e.y;
          o.P.z += w * at.rho_e.z;
          o.E += w * at.rho_e.w;
          o.R.x += w * at.r.x;
          o.R.y += w * at.r.y;
          o.R.z += w * at.r.z;
        } else {
          const float4 r = tc.attrs[pos].r;
          o.R.x += w * r.x;
          o.R.y += w * r.y;
          o.R.z += w * r.z;
        }
        if (hit_out && o.nhits < max_hits) hit_out[o.nhits] = (int32_t)key_idx(tc, kk[j]);
        ++o.nhits;
        o.T *= (1.0f - a);
        if (o.T < tc.T_min) done = true;
      }
    }
    if (cnt < KBUF) done = true;
    if (!done) {
      last = kk[KBUF - 1];
      have_last = true;
      t_floor = key_tlo(tc, last);
    }
  }
  return o;
}

}  // namespace eag

#include "eag_internal.h"
namespace eag {
TraceCtx make_ctx(const eag_bvh* b, const Attr* attrs, const eag_trace_params* p, const TraceSetup& ts);
}  // namespace eag
