// Single-bounce adjoint (reverse of Sec. 3.3, Eq. 7; the gradient the Stage-1
// objective of Eq. 8 needs, extended to every surfel parameter but e).
//
// Hit lists are recomputed, not stored: each kernel re-traces its segment
// with the forward's exact code, so the k-buffer visits the same hits
// in the same order, and reverses the blending on the fly. For a blended
// quantity V = sum_i T_{i-1} alpha_i v_i,
//   dV/dalpha_j = T_{j-1} v_j - (V - V_{<=j}) / (1 - alpha_j),
// where the suffix V - V_{<=j} comes from the forward's stored total minus
// the running prefix; A = 1 - T_m adds T_m / (1 - alpha_j).
//
// k_sb_bwd_secondary  one work item per (pixel, sample) of reflecting pixels,
//   on the persistent segment runner:
//   upstream dR1 = P * dL / spp; per hit: radiance gradient, alpha -> opacity,
//   tangent-plane coordinates -> centre, quaternion, scales, and the ray's
//   origin X and direction w'. Writes dL/dX and dL/dNt (through the
//   hemisphere frame) per sample.
// k_sb_bwd_camera     one work item per pixel, on the runner: gathers its samples' dX, dNt in
//   order, maps them to dN, dD, dA through Nt = N/|N| and Dt = D/A, adds dP =
//   dL * mean R1 (or dR = dL for emitter pixels) and reverses the camera
//   segment.
// Gradients are summed in double precision in a workspace accumulator,
// through per-hit records (float terms) grouped by surfel, and added to the
// caller's float arrays at the end.
#include "eag_device.h"
#include "eag_internal.h"
#include "eag_render.h"
#include "eag_runner.h"


namespace eag {

namespace {

// Gradient accumulators: double precision in the workspace (component-major,
// pos[3] rot[4] scale[2] opacity albedo[3] radiance[3] = 16 rows of n), so
// that sums of many opposing contributions keep their small results; they
// are added to the caller's float arrays once at the end.
constexpr int GRAD_ROWS = 16;
struct GradPtrs {
  double* pos;
  double* rot;
  double* scale;
  double* opacity;
  double* albedo;
  double* radiance;
  int64_t n;
};

__device__ __forceinline__ void atomic_add3(double* base, int64_t n, int64_t i, D3 v) {
  atomicAdd(base + i, v.x);
  atomicAdd(base + n + i, v.y);
  atomicAdd(base + 2 * n + i, v.z);
}

// Chain of one hit's opacity-term gradient g_alpha, distance gradient g_t and
// normal gradient g_n into the surfel's centre, quaternion, scales and opacity
// (out, in accumulator-row order: pos 0-2, rot 3-6, scale 7-8, opacity 9), and
// into the ray origin and direction (accumulated in gO, gW). Double
// precision, like the forward geometry.
__device__ __forceinline__ void chain_values(const Geo& ge, D3 O, D3 W, double t, double g_alpha, double g_t, D3 g_n,
                                             bool ray_grad, D3& gO, D3& gW, double (&out)[10]) {
  const D3 d = ge.p - O;
  const double den = dot(W, ge.n);
  const D3 y = d3(t * W.x - d.x, t * W.y - d.y, t * W.z - d.z);
  const double u = dot(y, ge.tu) / ge.su, v = dot(y, ge.tv) / ge.sv;
  const double g = exp(-0.5 * (u * u + v * v));
  // alpha = sigma g, g = exp(-(u^2+v^2)/2)
  const double g_sigma = g_alpha * g;
  const double g_q2 = -0.5 * g * (g_alpha * ge.sigma);
  const double gu = 2.0 * u * g_q2, gv = 2.0 * v * g_q2;
  // u = y.t_u / s_u, v = y.t_v / s_v
  const D3 gy = (gu / ge.su) * ge.tu + (gv / ge.sv) * ge.tv;
  // y = t W - d, t = (d.n) / (W.n)
  const double gt = g_t + dot(gy, W);
  const double gnum = gt / den, gden = -gt * t / den;
  const D3 gd = gnum * ge.n - gy;
  const D3 gn = g_n + gnum * d + gden * W;
  if (ray_grad) {
    gW = gW + t * gy + gden * ge.n;
    gO = gO - gd;
  }
  // t_u, t_v: through u, v and n = t_u x t_v
  const D3 gtu = (gu / ge.su) * y + cross(ge.tv, gn);
  const D3 gtv = (gv / ge.sv) * y + cross(gn, ge.tu);
  const double gsu = -gu * u / ge.su;
  const double gsv = -gv * v / ge.sv;
  const double qw = ge.qw, qx = ge.qx, qy = ge.qy, qz = ge.qz;
  const double gqw = 2.0 * (gtu.y * qz - gtu.z * qy - gtv.x * qz + gtv.z * qx);
  const double gqx = 2.0 * (gtu.y * qy + gtu.z * qz + gtv.x * qy - 2.0 * gtv.y * qx + gtv.z * qw);
  const double gqy = 2.0 * (-2.0 * gtu.x * qy + gtu.y * qx - gtu.z * qw + gtv.x * qx + gtv.z * qz);
  const double gqz = 2.0 * (-2.0 * gtu.x * qz + gtu.y * qw + gtu.z * qx - gtv.x * qw - 2.0 * gtv.y * qz + gtv.z * qy);
  // q_hat = q / |q|
  const double proj = qw * gqw + qx * gqx + qy * gqy + qz * gqz;
  out[0] = gd.x;
  out[1] = gd.y;
  out[2] = gd.z;
  out[3] = (gqw - qw * proj) * ge.iq;
  out[4] = (gqx - qx * proj) * ge.iq;
  out[5] = (gqy - qy * proj) * ge.iq;
  out[6] = (gqz - qz * proj) * ge.iq;
  out[7] = gsu;
  out[8] = gsv;
  out[9] = g_sigma;
}

// Per-hit gradient records of both adjoint passes. Added with atomics, a
// pass is limited by their rate (13 to 16 per hit). Instead, each hit writes
// one record of the 16 accumulator rows (64 B: each term rounded to float,
// their sums taken in double, so a surfel's sum carries an error of about
// 2^-24 of the sum of its terms' magnitudes at most) to the next slot of its
// wave's current chunk of REC_CHUNK slots, and counts itself in a per-surfel
// counter with an atomic whose result it does not wait for. A wave claims a
// chunk from a global counter when the lanes of a call do not fit in its
// current one (one atomic per many hits) and records how much of the chunk it
// used; its cursor lives in LDS. After the pass, an exclusive scan of the
// counters and a placement pass group the slots by surfel, and one wave per
// surfel sums its records. Hits that find the chunks exhausted fall back to
// atomics, so any capacity is correct.
constexpr unsigned REC_NO_CHUNK = 0xffffffffu;   // none claimed yet
constexpr unsigned REC_SPENT = 0xfffffffeu;      // the chunks are exhausted: atomics from here on
__device__ __forceinline__ void emit_record(const GradRecs& gr, const GradPtrs& gp, unsigned* wcur, uint32_t idx,
                                            const double (&v)[GRAD_ROWS]) {
  // wcur[0]: slots used in the wave's chunk, wcur[1]: the chunk (or none)
  const uint64_t act = __ballot(1);
  const int lane = (int)(threadIdx.x & 63);
  const int leader = __ffsll((unsigned long long)act) - 1;
  const unsigned k = (unsigned)__popcll(act);
  unsigned base = 0, chunk = REC_NO_CHUNK;
  if (lane == leader) {
    unsigned cur = wcur[0], ch = wcur[1];
    if (ch == REC_NO_CHUNK || (ch != REC_SPENT && cur + k > (unsigned)REC_CHUNK)) {
      if (ch < (unsigned)gr.n_chunks) gr.chunk_used[ch] = cur;
      const unsigned long long c = atomicAdd(gr.chunk_next, 1ull);
      ch = c < (unsigned long long)gr.n_chunks ? (unsigned)c : REC_SPENT;
      cur = 0;
    }
    base = cur;
    chunk = ch;
    wcur[0] = cur + k;
    wcur[1] = ch;
  }
  base = __shfl(base, leader);
  chunk = __shfl(chunk, leader);
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  if (chunk < (unsigned)gr.n_chunks) {
    const int64_t slot = (int64_t)chunk * REC_CHUNK + base + __popcll(act & below);
    float4* dst = reinterpret_cast<float4*>(gr.rec + slot * GRAD_ROWS);
#pragma unroll
    for (int q = 0; q < GRAD_ROWS / 4; ++q)
      dst[q] = make_float4((float)v[4 * q], (float)v[4 * q + 1], (float)v[4 * q + 2], (float)v[4 * q + 3]);
    gr.idx[slot] = idx;
    atomicAdd(gr.cnt + idx, 1u);   // no return value: the lane does not wait for it
  } else {
    const int64_t n = gp.n;
    atomic_add3(gp.pos, n, idx, d3(v[0], v[1], v[2]));
#pragma unroll
    for (int k = 0; k < 4; ++k) atomicAdd(gp.rot + k * n + idx, v[3 + k]);
    atomicAdd(gp.scale + idx, v[7]);
    atomicAdd(gp.scale + n + idx, v[8]);
    atomicAdd(gp.opacity + idx, v[9]);
    atomic_add3(gp.albedo, n, idx, d3(v[10], v[11], v[12]));
    atomic_add3(gp.radiance, n, idx, d3(v[13], v[14], v[15]));
  }
}

// Secondary segments on the persistent segment runner (eag_runner.h): one
// work item per (pixel, sample); only R1 = sum w r is used. Items of pixels
// that did not take the reflect branch write zero adjoints without tracing.
struct SecondaryAdjSource {
  const Record* recs;
  const Attr* attrs;
  const CamBatch* cams;
  int64_t hw;
  int32_t S;
  SbParams sp;
  const float* state;
  const double* r1;
  const float* dL;
  GradPtrs gp;
  GradRecs gr;
  unsigned* wcur;     // this wave's record cursor and chunk (LDS)
  double* adj;
  bool ray_grad;
  // per item
  int64_t item;
  D3 gR1;
  double G;          // gR1 . R1 (the forward total)
  double prefix;
  D3 gO, gW;

  // the item's pixel state, camera and bounce samples
  __device__ __forceinline__ void frame(int64_t g, uint32_t s, D3& X, D3& Nt, double& u0, double& u1) const {
    const double* d = reinterpret_cast<const double*>(state + g * EAG_FWD_PIXEL_FLOATS);
    Nt = d3(d[0], d[1], d[2]);
    const double Dt = d[3];
    const CamDev& c = cams->c[g / hw];
    const uint32_t pix = (uint32_t)(g % hw);
    const D3 Wc = pixel_dir(c, pix, 0, sp.flags, sp.k0, sp.k1);
    X = d3(c.eye[0] + Dt * Wc.x, c.eye[1] + Dt * Wc.y, c.eye[2] + Dt * Wc.z);
    const uint4 w4 = philox(make_uint4(pix, s, 0u, c.id), sp.k0, sp.k1);
    u0 = to_unit(w4.x);
    u1 = to_unit(w4.y);
  }

  __device__ __forceinline__ bool start(int64_t wid, TraceCtx&, D3& O, D3& W) {
    item = wid;
    const int64_t g = wid / S;
    const uint32_t s = (uint32_t)(wid - g * S);
    if (state[g * EAG_FWD_PIXEL_FLOATS + 25] != 2.0f) {
#pragma unroll
      for (int k = 0; k < 6; ++k) adj[wid * 6 + k] = 0.0;
      return false;
    }
    D3 Nt;
    double u0, u1;
    frame(g, s, O, Nt, u0, u1);
    W = cosine_dir(Nt, u0, u1);
    const double* d = reinterpret_cast<const double*>(state + g * EAG_FWD_PIXEL_FLOATS);
    const double inv = 1.0 / (double)S;
    gR1 = d3(d[9] * dL[g * 3 + 0] * inv, d[10] * dL[g * 3 + 1] * inv, d[11] * dL[g * 3 + 2] * inv);
    const double* R1 = r1 + wid * 3;
    G = gR1.x * R1[0] + gR1.y * R1[1] + gR1.z * R1[2];
    prefix = 0.0;
    gO = d3(0.0, 0.0, 0.0);
    gW = d3(0.0, 0.0, 0.0);
    return true;
  }

  __device__ __forceinline__ void operator()(uint32_t pos, double t, double alpha, double w, double Tb, D3 O, D3 W) {
    const Record r = load_record(recs, pos);
    const uint32_t idx = rec_index(r);
    const Geo ge = surfel_geo(r);
    const float4 rr = attrs[pos].r;
    const double c = gR1.x * rr.x + gR1.y * rr.y + gR1.z * rr.z;
    prefix += w * c;
    const double g_alpha = Tb * c - (G - prefix) / (1.0 - alpha);
    double v[GRAD_ROWS];
    double cv[10];
    chain_values(ge, O, W, t, g_alpha, 0.0, d3(0.0, 0.0, 0.0), ray_grad, gO, gW, cv);
#pragma unroll
    for (int k = 0; k < 10; ++k) v[k] = cv[k];
    v[10] = v[11] = v[12] = 0.0;   // albedo: the secondary pass has none
    v[13] = w * gR1.x;
    v[14] = w * gR1.y;
    v[15] = w * gR1.z;
    emit_record(gr, gp, wcur, idx, v);
  }

  __device__ __forceinline__ bool finish(const Seg<true>&, D3&, D3&) {
    double out[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (ray_grad) {
      const int64_t g = item / S;
      const uint32_t s = (uint32_t)(item - g * S);
      D3 X, Nt;
      double u0, u1;
      frame(g, s, X, Nt, u0, u1);
      // w' = c1 b1 + c2 b2 + c3 Nt, b1 = m / |m|, m = h - (h.Nt) Nt, b2 = Nt x b1
      const D3 h = d3(HX, HY, HZ);
      const double hn = dot(h, Nt);
      const D3 m = h - hn * Nt;
      const double ml = sqrt(dot(m, m));
      const D3 b1 = (1.0 / ml) * m;
      const double rr = sqrt(u0);
      double sn, cs;
      sincos(TWO_PI * u1, &sn, &cs);
      const double c1 = rr * cs, c2 = rr * sn, c3 = sqrt(1.0 - u0);
      const D3 gb2 = c2 * gW;
      const D3 gb1 = c1 * gW + cross(gb2, Nt);
      D3 gNt = c3 * gW + cross(b1, gb2);
      const D3 gm = (1.0 / ml) * (gb1 - dot(b1, gb1) * b1);
      gNt = gNt - hn * gm - dot(gm, Nt) * h;
      out[0] = gO.x; out[1] = gO.y; out[2] = gO.z;
      out[3] = gNt.x; out[4] = gNt.y; out[5] = gNt.z;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) adj[item * 6 + k] = out[k];
    return false;
  }
};

__global__ void __launch_bounds__(TRACE_BLOCK) __attribute__((amdgpu_waves_per_eu(2))) k_sb_bwd_secondary(TraceCtx tc, const CamBatch cams, int64_t hw,
                                                                  int32_t n_cams, SbParams sp, const float* state,
                                                                  const double* r1, const float* dL, GradPtrs gp,
                                                                  GradRecs gr, double* adj, unsigned long long* work,
                                                                  uint64_t* hitlist) {
  SecondaryAdjSource src;
  src.recs = tc.recs;
  src.attrs = tc.attrs;
  src.cams = &cams;
  src.hw = hw;
  src.S = sp.spp;
  src.sp = sp;
  src.state = state;
  src.r1 = r1;
  src.dL = dL;
  __shared__ unsigned s_wcur[2 * (TRACE_BLOCK / 64)];
  const int wv = (int)(threadIdx.x >> 6);
  if ((threadIdx.x & 63) == 0) {
    s_wcur[2 * wv] = 0u;
    s_wcur[2 * wv + 1] = REC_NO_CHUNK;
  }
  src.gp = gp;
  src.gr = gr;
  src.wcur = s_wcur + 2 * wv;
  src.adj = adj;
  src.ray_grad = !(sp.flags & EAG_DETACH_BOUNCE);
  src.item = 0;
  src.gR1 = src.gO = src.gW = d3(0.0, 0.0, 0.0);
  src.G = src.prefix = 0.0;
  run_segments<Q_RADIANCE, true>(tc, src, work, hw * n_cams * sp.spp, hitlist, nullptr);
  // (the runner's loop ends for the whole wave at once)
  if ((threadIdx.x & 63) == 0 && s_wcur[2 * wv + 1] < (unsigned)gr.n_chunks)
    gr.chunk_used[s_wcur[2 * wv + 1]] = s_wcur[2 * wv];
}

// Camera segments on the persistent segment runner: one work item per pixel;
// N, D, R (emitter pixels), P (reflecting pixels) and A are reversed. The
// pixel's samples' dX, dNt are gathered in order and mapped to dN, dD, dA
// through Nt = N/|N| and Dt = D/A; dP = dL * mean R1 (or dR = dL for emitter
// pixels). Missed pixels have nothing to reverse.
struct CameraAdjSource {
  const Record* recs;
  const Attr* attrs;
  const CamBatch* cams;
  int64_t hw;
  SbParams sp;
  const float* state;
  const double* r1;
  const double* adj;
  const float* dL;
  GradPtrs gp;
  GradRecs gr;
  unsigned* wcur;     // this wave's record cursor and chunk (LDS)
  // per item
  D3 gN, gR, gP;
  double gD, gA, Tm, G, prefix;
  bool has_R, has_P;

  __device__ __forceinline__ bool start(int64_t g, TraceCtx&, D3& O, D3& W) {
    const FwdState st = load_state(state + g * EAG_FWD_PIXEL_FLOATS);
    if (st.branch == 0.0f) return false;
    const CamDev& c = cams->c[g / hw];
    W = pixel_dir(c, (uint32_t)(g % hw), 0, sp.flags, sp.k0, sp.k1);
    O = d3(c.eye[0], c.eye[1], c.eye[2]);
    const D3 dl = d3(dL[g * 3 + 0], dL[g * 3 + 1], dL[g * 3 + 2]);
    gN = gR = gP = d3(0.0, 0.0, 0.0);
    gD = gA = 0.0;
    Tm = 1.0 - st.A;
    has_R = st.branch == 1.0f;
    has_P = st.branch == 2.0f;
    if (has_R) {
      gR = dl;
      G = dot(dl, st.R);
    } else {
      const int S = sp.spp;
      double m0 = 0.0, m1 = 0.0, m2 = 0.0;
      D3 gX = d3(0.0, 0.0, 0.0), gNt = d3(0.0, 0.0, 0.0);
      for (int s = 0; s < S; ++s) {
        const double* q = r1 + (g * S + s) * 3;
        m0 += q[0];
        m1 += q[1];
        m2 += q[2];
        const double* ad = adj + (g * S + s) * 6;
        gX = gX + d3(ad[0], ad[1], ad[2]);
        gNt = gNt + d3(ad[3], ad[4], ad[5]);
      }
      const double inv = 1.0 / (double)S;
      gP = d3(dl.x * (m0 * inv), dl.y * (m1 * inv), dl.z * (m2 * inv));
      // X = O + Dt W; Nt = N / |N|; Dt = D / A
      const double gDt = dot(gX, W);
      gN = (1.0 / st.Nlen) * (gNt - dot(st.Nt, gNt) * st.Nt);
      gD = gDt / st.A;
      gA = -gDt * st.Dt / st.A;
      G = dot(gN, st.Nlen * st.Nt) + gD * (st.Dt * st.A) + dot(gP, st.P);
    }
    prefix = 0.0;
    return true;
  }

  __device__ __forceinline__ void operator()(uint32_t pos, double t, double alpha, double w, double Tb, D3 O, D3 W) {
    const Record r = load_record(recs, pos);
    const uint32_t idx = rec_index(r);
    const Geo ge = surfel_geo(r);
    const Attr at = attrs[pos];
    const D3 nn = ge.n;
    const double sgn = dot(W, nn) > 0.0 ? -1.0 : 1.0;   // n' = sgn n faces the origin
    const D3 rho = d3(at.rho_e.x, at.rho_e.y, at.rho_e.z), rad = d3(at.r.x, at.r.y, at.r.z);
    const double c = sgn * dot(gN, nn) + gD * t + dot(gR, rad) + dot(gP, rho);
    prefix += w * c;
    const double g_alpha = Tb * c - (G - prefix - gA * Tm) / (1.0 - alpha);
    D3 dummyO = d3(0.0, 0.0, 0.0), dummyW = d3(0.0, 0.0, 0.0);
    double v[GRAD_ROWS];
    double cv[10];
    chain_values(ge, O, W, t, g_alpha, w * gD, (sgn * w) * gN, false, dummyO, dummyW, cv);
#pragma unroll
    for (int k = 0; k < 10; ++k) v[k] = cv[k];
    v[10] = has_P ? w * gP.x : 0.0;
    v[11] = has_P ? w * gP.y : 0.0;
    v[12] = has_P ? w * gP.z : 0.0;
    v[13] = has_R ? w * gR.x : 0.0;
    v[14] = has_R ? w * gR.y : 0.0;
    v[15] = has_R ? w * gR.z : 0.0;
    emit_record(gr, gp, wcur, idx, v);
  }

  __device__ __forceinline__ bool finish(const Seg<true>&, D3&, D3&) { return false; }
};

__global__ void __launch_bounds__(TRACE_BLOCK) __attribute__((amdgpu_waves_per_eu(2))) k_sb_bwd_camera(TraceCtx tc, const CamBatch cams, int64_t hw,
                                                               int32_t n_cams, SbParams sp, const float* state,
                                                               const double* r1, const double* adj, const float* dL,
                                                               GradPtrs gp, GradRecs gr, unsigned long long* work,
                                                               uint64_t* hitlist) {
  CameraAdjSource src;
  src.recs = tc.recs;
  src.attrs = tc.attrs;
  src.cams = &cams;
  src.hw = hw;
  src.sp = sp;
  src.state = state;
  src.r1 = r1;
  src.adj = adj;
  src.dL = dL;
  src.gp = gp;
  __shared__ unsigned s_wcur[2 * (TRACE_BLOCK / 64)];
  const int wv = (int)(threadIdx.x >> 6);
  if ((threadIdx.x & 63) == 0) {
    s_wcur[2 * wv] = 0u;
    s_wcur[2 * wv + 1] = REC_NO_CHUNK;
  }
  src.gr = gr;
  src.wcur = s_wcur + 2 * wv;
  src.gN = src.gR = src.gP = d3(0.0, 0.0, 0.0);
  src.gD = src.gA = src.Tm = src.G = src.prefix = 0.0;
  src.has_R = src.has_P = false;
  run_segments<Q_ALL, true>(tc, src, work, hw * n_cams, hitlist, nullptr);
  if ((threadIdx.x & 63) == 0 && s_wcur[2 * wv + 1] < (unsigned)gr.n_chunks)
    gr.chunk_used[s_wcur[2 * wv + 1]] = s_wcur[2 * wv];
}

// Stage-0 adjoint (Sec. 3.2, Eq. 4): one work item per pixel on the
// runner; the upstream gradient of the pixel's images (Nt, Dt, R, E; 8
// floats) is reversed through Nt = N/|N| and Dt = D/A into dN, dD, dA, dR,
// dE and then through the blended hits. Records carry the emissive gradient
// w dE in row 10 (the albedo rows are otherwise unused here).
struct Stage0AdjSource {
  const Record* recs;
  const Attr* attrs;
  const CamBatch* cams;
  int64_t hw;
  SbParams sp;
  const float* state;
  const float* dimg;
  GradPtrs gp;
  GradRecs gr;
  unsigned* wcur;
  // per item
  D3 gN, gR;
  double gD, gA, gE, Tm, G, prefix;

  __device__ __forceinline__ bool start(int64_t g, TraceCtx&, D3& O, D3& W) {
    const FwdState st = load_state(state + g * EAG_FWD_PIXEL_FLOATS);
    if (!(st.A > 0.0)) return false;   // a miss: every image is 0
    const float* d = dimg + g * 8;
    const D3 gNt = d3(d[0], d[1], d[2]);
    const double gDt = d[3];
    gR = d3(d[4], d[5], d[6]);
    gE = d[7];
    gN = (1.0 / st.Nlen) * (gNt - dot(st.Nt, gNt) * st.Nt);
    gD = gDt / st.A;
    gA = -gDt * st.Dt / st.A;
    Tm = 1.0 - st.A;
    G = dot(gN, st.Nlen * st.Nt) + gD * (st.Dt * st.A) + dot(gR, st.R) + gE * (double)st.E;
    prefix = 0.0;
    const CamDev& c = cams->c[g / hw];
    W = pixel_dir(c, (uint32_t)(g % hw), 0, sp.flags, sp.k0, sp.k1);
    O = d3(c.eye[0], c.eye[1], c.eye[2]);
    return true;
  }

  __device__ __forceinline__ void operator()(uint32_t pos, double t, double alpha, double w, double Tb, D3 O, D3 W) {
    const Record r = load_record(recs, pos);
    const uint32_t idx = rec_index(r);
    const Geo ge = surfel_geo(r);
    const Attr at = attrs[pos];
    const double sgn = dot(W, ge.n) > 0.0 ? -1.0 : 1.0;   // n' = sgn n faces the origin
    const double c = sgn * dot(gN, ge.n) + gD * t + gR.x * at.r.x + gR.y * at.r.y + gR.z * at.r.z +
                     gE * at.rho_e.w;
    prefix += w * c;
    const double g_alpha = Tb * c - (G - prefix - gA * Tm) / (1.0 - alpha);
    D3 dummyO = d3(0.0, 0.0, 0.0), dummyW = d3(0.0, 0.0, 0.0);
    double v[GRAD_ROWS];
    double cv[10];
    chain_values(ge, O, W, t, g_alpha, w * gD, (sgn * w) * gN, false, dummyO, dummyW, cv);
#pragma unroll
    for (int k = 0; k < 10; ++k) v[k] = cv[k];
    v[10] = w * gE;
    v[11] = v[12] = 0.0;
    v[13] = w * gR.x;
    v[14] = w * gR.y;
    v[15] = w * gR.z;
    emit_record(gr, gp, wcur, idx, v);
  }

  __device__ __forceinline__ bool finish(const Seg<true>&, D3&, D3&) { return false; }
};

__global__ void __launch_bounds__(TRACE_BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
k_stage0_bwd(TraceCtx tc, const CamBatch cams, int64_t hw, int32_t n_cams, SbParams sp, const float* state,
             const float* dimg, GradPtrs gp, GradRecs gr, unsigned long long* work, uint64_t* hitlist) {
  Stage0AdjSource src;
  src.recs = tc.recs;
  src.attrs = tc.attrs;
  src.cams = &cams;
  src.hw = hw;
  src.sp = sp;
  src.state = state;
  src.dimg = dimg;
  src.gp = gp;
  __shared__ unsigned s_wcur[2 * (TRACE_BLOCK / 64)];
  const int wv = (int)(threadIdx.x >> 6);
  if ((threadIdx.x & 63) == 0) {
    s_wcur[2 * wv] = 0u;
    s_wcur[2 * wv + 1] = REC_NO_CHUNK;
  }
  src.gr = gr;
  src.wcur = s_wcur + 2 * wv;
  src.gN = src.gR = d3(0.0, 0.0, 0.0);
  src.gD = src.gA = src.gE = src.Tm = src.G = src.prefix = 0.0;
  run_segments<Q_ALL, true>(tc, src, work, hw * n_cams, hitlist, nullptr);
  if ((threadIdx.x & 63) == 0 && s_wcur[2 * wv + 1] < (unsigned)gr.n_chunks)
    gr.chunk_used[s_wcur[2 * wv + 1]] = s_wcur[2 * wv];
}

// Stage-0 gradients to the caller's arrays: rows 0-9 (pos, rot, scale,
// opacity), row 10 (emissive), rows 13-15 (radiance).
__global__ void k_stage0_finalize(const double* acc, int64_t n, eag_surfel_grads g, float* ge) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n * GRAD_ROWS) return;
  const int64_t row = i / n, j = i - row * n;
  float* dst = nullptr;
  if (row < 3) dst = g.pos + row * n;
  else if (row < 7) dst = g.rot + (row - 3) * n;
  else if (row < 9) dst = g.scale + (row - 7) * n;
  else if (row < 10) dst = g.opacity;
  else if (row == 10) dst = ge;
  else if (row >= 13) dst = g.radiance + (row - 13) * n;
  if (dst) dst[j] += (float)acc[i];
}

__global__ void k_zero_u32(uint32_t* p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Every used slot of the claimed chunks goes to the next free position of its
// surfel's range [off[i], off[i] + cnt[i]) of order (cursor: zeroed per-surfel
// counts). Blocks stride over the claimed chunks only.
__global__ void __launch_bounds__(256) k_rec_place(GradRecs gr) {
  const unsigned long long claimed = *gr.chunk_next;
  const int64_t nc = claimed < (unsigned long long)gr.n_chunks ? (int64_t)claimed : gr.n_chunks;
  for (int64_t ch = blockIdx.x; ch < nc; ch += gridDim.x) {
    const uint32_t used = gr.chunk_used[ch];
    for (uint32_t j = threadIdx.x; j < used; j += blockDim.x) {
      const int64_t s = ch * REC_CHUNK + j;
      const uint32_t i = gr.idx[s];
      gr.order[gr.off[i] + atomicAdd(gr.cursor + i, 1u)] = (uint32_t)s;
    }
  }
}

// One wave per surfel: its records, summed lane-strided and then across the
// wave in a fixed order, are added to the accumulator rows.
__global__ void __launch_bounds__(256) k_rec_reduce(GradRecs gr, double* gacc, int64_t n) {
  const int64_t i = blockIdx.x * 4 + (int64_t)(threadIdx.x >> 6);
  const int lane = (int)(threadIdx.x & 63);
  if (i >= n) return;
  const uint32_t c = gr.cnt[i], o = gr.off[i];
  if (c == 0) return;
  double acc[GRAD_ROWS];
#pragma unroll
  for (int k = 0; k < GRAD_ROWS; ++k) acc[k] = 0.0;
  for (uint32_t j = (uint32_t)lane; j < c; j += 64) {
    const float4* r = reinterpret_cast<const float4*>(gr.rec + (size_t)gr.order[o + j] * GRAD_ROWS);
#pragma unroll
    for (int k = 0; k < GRAD_ROWS / 4; ++k) {
      const float4 v = r[k];
      acc[4 * k] += v.x;
      acc[4 * k + 1] += v.y;
      acc[4 * k + 2] += v.z;
      acc[4 * k + 3] += v.w;
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
#pragma unroll
    for (int k = 0; k < GRAD_ROWS; ++k) acc[k] += __shfl_xor(acc[k], m);
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < GRAD_ROWS; ++k) gacc[k * n + i] += acc[k];
  }
}

__global__ void k_zero_f64(double* p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ void k_grad_finalize(const double* acc, int64_t n, eag_surfel_grads g) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n * GRAD_ROWS) return;
  const int64_t row = i / n, j = i - row * n;
  float* dst;
  if (row < 3) dst = g.pos + row * n;
  else if (row < 7) dst = g.rot + (row - 3) * n;
  else if (row < 9) dst = g.scale + (row - 7) * n;
  else if (row < 10) dst = g.opacity;
  else if (row < 13) dst = g.albedo + (row - 10) * n;
  else dst = g.radiance + (row - 13) * n;
  dst[j] += (float)acc[i];
}

}  // namespace

size_t grad_accum_doubles(int64_t n) { return (size_t)n * GRAD_ROWS; }

int64_t grad_rec_capacity(int64_t n_items) {
  const int64_t c = n_items * GRAD_RECS_PER_ITEM;
  return c < GRAD_RECS_MAX ? c : GRAD_RECS_MAX;
}

size_t grad_rec_scan_bytes(int64_t n) { return scan_u32_bytes(n); }

void zero_record_counts(const GradRecs& gr, int64_t n, hipStream_t st) {
  if (gr.n_chunks <= 0) return;
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, gr.cnt, n);
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, gr.cursor, n);
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((gr.n_chunks + 255) / 256)), dim3(256), 0, st, gr.chunk_used,
                     gr.n_chunks);
  launch_zero_u64(gr.chunk_next, 1, st);
}

// Group the records of the pass just run by surfel and add their sums.
void reduce_records(const GradRecs& gr, double* gacc, int64_t n, hipStream_t st) {
  if (gr.n_chunks <= 0) return;
  scan_u32(gr.cnt, gr.off, n, false, gr.scan_tmp, gr.scan_bytes, st);
  hipLaunchKernelGGL(k_rec_place, dim3(4096), dim3(256), 0, st, gr);
  hipLaunchKernelGGL(k_rec_reduce, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, gr, gacc, n);
}

void launch_single_bounce_backward(const TraceCtx& tc, const eag_surfels& s, const CamBatch& cams, int64_t hw,
                                   int32_t n_cams, const SbParams& sp, const float* state, const double* r1,
                                   const float* dL, double* gacc, float* scratch, const GradRecs& grecs,
                                   unsigned long long* work, uint64_t* hitlist, hipStream_t st) {
  const int64_t n = s.n;
  GradPtrs gp{gacc, gacc + 3 * n, gacc + 7 * n, gacc + 9 * n, gacc + 10 * n, gacc + 13 * n, n};
  GradRecs gr = grecs;
  gr.chunk_next = work + 1;
  const unsigned grid = (unsigned)(runner_lanes() / TRACE_BLOCK);
  launch_zero_u64(work, 1, st);
  zero_record_counts(gr, n, st);
  hipLaunchKernelGGL(k_sb_bwd_secondary, dim3(grid), dim3(TRACE_BLOCK), 0, st, tc, cams, hw, n_cams, sp, state, r1,
                     dL, gp, gr, reinterpret_cast<double*>(scratch), work, hitlist);
  reduce_records(gr, gacc, n, st);
  launch_zero_u64(work, 1, st);
  zero_record_counts(gr, n, st);
  hipLaunchKernelGGL(k_sb_bwd_camera, dim3(grid), dim3(TRACE_BLOCK), 0, st, tc, cams, hw, n_cams, sp, state, r1,
                     reinterpret_cast<const double*>(scratch), dL, gp, gr, work, hitlist);
  reduce_records(gr, gacc, n, st);
  check_hip(hipGetLastError(), "single-bounce backward launch");
}

void launch_stage0_backward(const TraceCtx& tc, const eag_surfels& s, const CamBatch& cams, int64_t hw,
                            int32_t n_cams, const SbParams& sp, const float* state, const float* dimg, double* gacc,
                            const GradRecs& grecs, unsigned long long* work, uint64_t* hitlist, hipStream_t st) {
  const int64_t n = s.n;
  GradPtrs gp{gacc, gacc + 3 * n, gacc + 7 * n, gacc + 9 * n, gacc + 10 * n, gacc + 13 * n, n};
  GradRecs gr = grecs;
  gr.chunk_next = work + 1;
  launch_zero_u64(work, 1, st);
  zero_record_counts(gr, n, st);
  hipLaunchKernelGGL(k_stage0_bwd, dim3((unsigned)(runner_lanes() / TRACE_BLOCK)), dim3(TRACE_BLOCK), 0, st, tc, cams,
                     hw, n_cams, sp, state, dimg, gp, gr, work, hitlist);
  reduce_records(gr, gacc, n, st);
  check_hip(hipGetLastError(), "stage-0 backward launch");
}

void launch_stage0_finalize(const double* gacc, int64_t n, const eag_surfel_grads& g, float* grad_emissive,
                            hipStream_t st) {
  const int64_t m = n * GRAD_ROWS;
  hipLaunchKernelGGL(k_stage0_finalize, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, gacc, n, g,
                     grad_emissive);
  check_hip(hipGetLastError(), "stage-0 finalize launch");
}

void launch_grad_zero(double* gacc, int64_t n, hipStream_t st) {
  const int64_t m = n * GRAD_ROWS;
  hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, gacc, m);
}

void launch_grad_finalize(const double* gacc, int64_t n, const eag_surfel_grads& g, hipStream_t st) {
  const int64_t m = n * GRAD_ROWS;
  hipLaunchKernelGGL(k_grad_finalize, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, gacc, n, g);
  check_hip(hipGetLastError(), "gradient finalize launch");
}

}  // namespace eag
