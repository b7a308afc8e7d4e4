// Linear BVH build and refit over 2D Gaussian surfels.
//
// 1. frames and k_sigma-ellipse boxes of every surfel (the surfel of
//    Sec. 3.1: centre p, tangent axes t_u, t_v from the normalised
//    quaternion, scales s_u, s_v), and the scene bounds;
// 2. 63-bit Morton codes of the centres, radix-sorted (eag_prim.hip);
// 3. a binary hierarchy by locally-ordered agglomerative clustering of the
//    sorted boxes (below), which writes each node's child boxes as it makes
//    the node;
// 4. geometry records in sorted order (one 48-B record per surfel);
// 5. the depth of the binary tree, and its collapse into a 4-wide tree.
// A refit keeps the topology and recomputes the node boxes in the order of
// the clustering iterations that made the nodes.
// Everything is enqueued on the caller's stream: the depths, node count and
// bounds stay in the device header, and the host waits for them only when
// asked (eag_bvh_get_info).
#include <hip/hip_runtime.h>

#include "eag_device.h"
#include "eag_internal.h"

#include <algorithm>

namespace eag {

namespace {

__device__ __forceinline__ uint32_t fenc(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ __forceinline__ float fdec(uint32_t e) {
  const uint32_t b = (e & 0x80000000u) ? (e & 0x7fffffffu) : ~e;
  float f;
  __builtin_memcpy(&f, &b, 4);
  return f;
}

struct Frame {
  D3 tu, tv, n;
};
__device__ __forceinline__ Frame frame_of(const float* rot, int64_t n, int64_t i) {
  double w = rot[i], x = rot[n + i], y = rot[2 * n + i], z = rot[3 * n + i];
  const double inv = 1.0 / sqrt(w * w + x * x + y * y + z * z);
  w *= inv; x *= inv; y *= inv; z *= inv;
  Frame f;
  f.tu = d3(1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y + w * z), 2.0 * (x * z - w * y));
  f.tv = d3(2.0 * (x * y - w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z + w * x));
  f.n = cross(f.tu, f.tv);
  return f;
}

// Bounds only (a refit keeps the depths and the node count).
__global__ void k_reset_bounds(BvhHeader* h) {
  if (threadIdx.x < 3) {
    h->plo[threadIdx.x] = 0xffffffffu;
    h->phi[threadIdx.x] = 0u;
    h->blo[threadIdx.x] = 0xffffffffu;
    h->bhi[threadIdx.x] = 0u;
  }
}

__global__ void k_init_header(BvhHeader* h) {
  if (threadIdx.x < 3) {
    h->plo[threadIdx.x] = 0xffffffffu;
    h->phi[threadIdx.x] = 0u;
    h->blo[threadIdx.x] = 0xffffffffu;
    h->bhi[threadIdx.x] = 0u;
  }
  if (threadIdx.x == 0) {
    h->max_depth = 0;
    h->n_nodes4 = 0;
    h->depth4 = 0;
  }
}

// Box of the k_sigma ellipse: half extent along axis a is
// k * sqrt((s_u t_u,a)^2 + (s_v t_v,a)^2), padded so that float32 rounding in
// the surfel test can never place an accepted hit outside its box.
__global__ void k_boxes(eag_surfels s, float k, float* box, BvhHeader* h) {
  const int64_t n = s.n;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  float plo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
  float phi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
  float blo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
  float bhi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
  if (i < n) {
    const Frame f = frame_of(s.rot, n, i);
    const double su = s.scale[i], sv = s.scale[n + i];
    const float p[3] = {s.pos[i], s.pos[n + i], s.pos[2 * n + i]};
    const float pad = 2e-5f * (1.0f + fmaxf(fmaxf(fabsf(p[0]), fabsf(p[1])), fabsf(p[2])));
    const double tu[3] = {f.tu.x, f.tu.y, f.tu.z}, tv[3] = {f.tv.x, f.tv.y, f.tv.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float e = (float)(k * sqrt((su * tu[a]) * (su * tu[a]) + (sv * tv[a]) * (sv * tv[a]))) + pad;
      box[a * n + i] = p[a] - e;
      box[(3 + a) * n + i] = p[a] + e;
      plo[a] = phi[a] = p[a];
      blo[a] = p[a] - e;
      bhi[a] = p[a] + e;
    }
  }
  // block reduction of the bounds, then one atomic per block and component
  __shared__ float red[12][256];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    red[a][threadIdx.x] = plo[a];
    red[3 + a][threadIdx.x] = phi[a];
    red[6 + a][threadIdx.x] = blo[a];
    red[9 + a][threadIdx.x] = bhi[a];
  }
  __syncthreads();
  for (int s2 = blockDim.x / 2; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + s2]);
        red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + s2]);
        red[6 + a][threadIdx.x] = fminf(red[6 + a][threadIdx.x], red[6 + a][threadIdx.x + s2]);
        red[9 + a][threadIdx.x] = fmaxf(red[9 + a][threadIdx.x], red[9 + a][threadIdx.x + s2]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) {
    const int a = threadIdx.x;
    atomicMin(&h->plo[a], fenc(red[a][0]));
    atomicMax(&h->phi[a], fenc(red[3 + a][0]));
    atomicMin(&h->blo[a], fenc(red[6 + a][0]));
    atomicMax(&h->bhi[a], fenc(red[9 + a][0]));
  }
}

__device__ __forceinline__ uint64_t spread3(uint32_t a) {
  uint64_t x = a & 0x1fffffu;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}

__global__ void k_morton(eag_surfels s, const BvhHeader* h, uint64_t* codes, uint32_t* ids) {
  const int64_t n = s.n;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t q[3];
  float ext = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) ext = fmaxf(ext, fdec(h->phi[a]) - fdec(h->plo[a]));
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float lo = fdec(h->plo[a]);
    float x = ext > 0.0f ? (s.pos[a * n + i] - lo) / ext : 0.0f;
    x = fminf(fmaxf(x, 0.0f), 1.0f);
    q[a] = min((uint32_t)(x * 2097152.0f), 2097151u);
  }
  codes[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
  ids[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// Binary hierarchy by locally-ordered agglomerative clustering (PLOC, Meister
// and Bittner, TVCG 2018). The clusters start as the leaves in Morton order.
// Each iteration finds every cluster's nearest neighbour among the PLOC_R
// clusters on either side in the current order, by the surface area of the
// union of their boxes (ties to the lower position), merges every mutual pair
// into a new internal node at the lower position, and compacts the order.
// A cluster made in iteration t is at most t levels high, so iterations are
// launched a fixed number of times: PLOC_ITERS of them, then at most
// ceil(log2 n) halving iterations that pair positions 2k and 2k + 1, which
// bound the tree's height by PLOC_ITERS + ceil(log2 n) whatever the input.
// Every launch reads the cluster count from the device and returns at once
// when one cluster is left. Internal nodes are numbered from the top: the
// k-th node made is n - 2 - k, so the last (the root) is node 0.
// ---------------------------------------------------------------------------
constexpr int PLOC_R = 2;          // search radius (measured best of 1 to 16 for the path tracer)
constexpr int PLOC_ITERS = 64;     // iterations before the halving fallback
constexpr int PLOC_GRID = 1024;    // blocks of every clustering launch
constexpr int PLOC_TILE = 256;
constexpr int PLOC_LEVELS = PLOC_ITERS + 24;   // iterations launched for up to 2^23 surfels, and more

struct PlocState {
  int32_t n;          // clusters now
  int32_t n_prev;     // clusters before the last merge step
  int32_t cur;        // buffer holding the current clusters
  int32_t active;     // the last scan found work to merge
  int32_t made;       // internal nodes made so far
  int32_t made_base;  // nodes made before the last merge step
  int32_t pad[2];
};

struct Ploc {
  int32_t* cl[2];     // cluster references (node >= 0, leaf ~position)
  float4* cb[2];      // cluster boxes: [2i] lo.xyz, [2i + 1] hi.xyz
  int32_t* nn;        // nearest neighbour of each cluster
  int32_t* bsum;      // per block: clusters kept, nodes made
  int32_t* boff;      // exclusive offsets of bsum
  PlocState* st;
};

__device__ __forceinline__ float union_area(float4 al, float4 ah, float4 bl, float4 bh) {
  const float dx = fmaxf(ah.x, bh.x) - fminf(al.x, bl.x);
  const float dy = fmaxf(ah.y, bh.y) - fminf(al.y, bl.y);
  const float dz = fmaxf(ah.z, bh.z) - fminf(al.z, bl.z);
  return dx * dy + dy * dz + dz * dx;
}

__global__ void k_ploc_init(int64_t n, const float* box, const int32_t* perm, Ploc P, int32_t* node_parent) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j == 0) {
    PlocState s = {};
    s.n = (int32_t)n;
    *P.st = s;
    node_parent[0] = -1;
  }
  if (j >= n) return;
  const int64_t i = perm[j];
  P.cl[0][j] = ~(int32_t)j;
  P.cb[0][2 * j] = make_float4(box[i], box[n + i], box[2 * n + i], 0.0f);
  P.cb[0][2 * j + 1] = make_float4(box[3 * n + i], box[4 * n + i], box[5 * n + i], 0.0f);
}

// Nearest neighbour of every cluster (halving: the other of its pair).
__global__ void __launch_bounds__(PLOC_TILE) k_ploc_nn(Ploc P, int halving) {
  __shared__ float4 slo[PLOC_TILE + 2 * PLOC_R], shi[PLOC_TILE + 2 * PLOC_R];
  const int n = P.st->n;
  if (n <= 1) return;
  const int p = P.st->cur;
  const float4* cb = P.cb[p];
  for (int base = blockIdx.x * PLOC_TILE; base < n; base += gridDim.x * PLOC_TILE) {
    const int i = base + (int)threadIdx.x;
    if (halving) {
      if (i < n) P.nn[i] = (i ^ 1) < n ? (i ^ 1) : i;
      continue;
    }
    for (int k = threadIdx.x; k < PLOC_TILE + 2 * PLOC_R; k += PLOC_TILE) {
      const int g = base - PLOC_R + k;
      if (g >= 0 && g < n) {
        slo[k] = cb[2 * g];
        shi[k] = cb[2 * g + 1];
      }
    }
    __syncthreads();
    if (i < n) {
      const int li = (int)threadIdx.x + PLOC_R;
      const float4 al = slo[li], ah = shi[li];
      float best = INFINITY;
      int bj = i;
      for (int d = -PLOC_R; d <= PLOC_R; ++d) {
        const int g = i + d;
        if (d == 0 || g < 0 || g >= n) continue;
        const float a = union_area(al, ah, slo[li + d], shi[li + d]);
        if (a < best) {   // ascending g: ties keep the lower position
          best = a;
          bj = g;
        }
      }
      P.nn[i] = bj;
    }
    __syncthreads();
  }
}

// Per position: kept (a cluster survives there) and made (a node is made
// there, at the lower position of a mutual pair).
__device__ __forceinline__ void ploc_decide(const int32_t* nn, int i, int& j, bool& keep, bool& made) {
  j = nn[i];
  const bool mutual = j != i && nn[j] == i;
  keep = !mutual || i < j;
  made = mutual && i < j;
}

// Exclusive block scan of two counts (each at most PLOC_TILE per tile),
// packed in one int; returns the block's totals in *tot.
__device__ __forceinline__ int scan_pair(int v, int* lds, int* tot) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(x, o);
    if (lane >= o) x += t;
  }
  if (lane == 63) lds[w] = x;
  __syncthreads();
  int before = 0;
  for (int k = 0; k < w; ++k) before += lds[k];
  *tot = lds[0] + lds[1] + lds[2] + lds[3];
  __syncthreads();
  return before + x - v;
}

__device__ __forceinline__ void ploc_chunk(int n, int& lo, int& hi) {
  const int chunk = (n + gridDim.x - 1) / gridDim.x;
  lo = min(n, (int)blockIdx.x * chunk);
  hi = min(n, lo + chunk);
}

__global__ void __launch_bounds__(PLOC_TILE) k_ploc_count(Ploc P) {
  __shared__ int lds[4];
  const int n = P.st->n;
  if (n <= 1) return;
  int lo, hi;
  ploc_chunk(n, lo, hi);
  int keep_sum = 0, made_sum = 0;
  for (int base = lo; base < hi; base += PLOC_TILE) {
    const int i = base + (int)threadIdx.x;
    int v = 0;
    if (i < hi) {
      int j;
      bool keep, made;
      ploc_decide(P.nn, i, j, keep, made);
      v = (keep ? 1 : 0) | (made ? 1 << 16 : 0);
    }
    int tot;
    scan_pair(v, lds, &tot);
    keep_sum += tot & 0xffff;
    made_sum += tot >> 16;
  }
  if (threadIdx.x == 0) {
    P.bsum[2 * blockIdx.x] = keep_sum;
    P.bsum[2 * blockIdx.x + 1] = made_sum;
  }
}

// One block: offsets of the blocks' kept clusters and made nodes, and the
// state for the write step.
// levels[t]: the nodes made before iteration t (iteration t makes the ids
// n - 2 - k for k in [levels[t], levels[t + 1])), kept with the tree for
// refits.
__global__ void __launch_bounds__(PLOC_GRID) k_ploc_scan(Ploc P, int blocks, int t_iter, int32_t* levels) {
  __shared__ int lk[PLOC_GRID / 64], lm[PLOC_GRID / 64];
  PlocState* st = P.st;
  const int n = st->n;
  if (threadIdx.x == 0) levels[t_iter] = st->made;
  if (n <= 1) {
    if (threadIdx.x == 0) st->active = 0;
    return;
  }
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int k0 = t < blocks ? P.bsum[2 * t] : 0, m0 = t < blocks ? P.bsum[2 * t + 1] : 0;
  int k = k0, m = m0;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int a = __shfl_up(k, o), b = __shfl_up(m, o);
    if (lane >= o) {
      k += a;
      m += b;
    }
  }
  if (lane == 63) {
    lk[w] = k;
    lm[w] = m;
  }
  __syncthreads();
  int kb = 0, mb = 0, kt = 0, mt = 0;
  for (int q = 0; q < PLOC_GRID / 64; ++q) {
    if (q < w) {
      kb += lk[q];
      mb += lm[q];
    }
    kt += lk[q];
    mt += lm[q];
  }
  if (t < blocks) {
    P.boff[2 * t] = kb + k - k0;
    P.boff[2 * t + 1] = mb + m - m0;
  }
  if (t == 0) {
    st->n_prev = n;
    st->n = kt;
    st->cur ^= 1;
    st->active = 1;
    st->made_base = st->made;
    st->made += mt;
  }
}

__global__ void __launch_bounds__(PLOC_TILE) k_ploc_write(Ploc P, int64_t n_leaves, Node* nodes,
                                                         int32_t* leaf_parent, int32_t* node_parent) {
  __shared__ int lds[4];
  const PlocState* st = P.st;
  if (!st->active) return;
  const int n = st->n_prev;
  const int out = st->cur, in = out ^ 1;
  const int32_t* cl = P.cl[in];
  const float4* cb = P.cb[in];
  int lo, hi;
  ploc_chunk(n, lo, hi);
  int keep_at = P.boff[2 * blockIdx.x];
  int made_at = st->made_base + P.boff[2 * blockIdx.x + 1];
  for (int base = lo; base < hi; base += PLOC_TILE) {
    const int i = base + (int)threadIdx.x;
    int j = i;
    bool keep = false, made = false;
    if (i < hi) ploc_decide(P.nn, i, j, keep, made);
    int tot;
    const int off = scan_pair((keep ? 1 : 0) | (made ? 1 << 16 : 0), lds, &tot);
    if (keep) {
      const int o = keep_at + (off & 0xffff);
      if (made) {
        const int id = (int)(n_leaves - 2) - (made_at + (off >> 16));
        const int c0 = cl[i], c1 = cl[j];
        const float4 l0 = cb[2 * i], h0 = cb[2 * i + 1], l1 = cb[2 * j], h1 = cb[2 * j + 1];
        Node nd;
        nd.a = make_float4(l0.x, l0.y, l0.z, h0.x);
        nd.b = make_float4(h0.y, h0.z, l1.x, l1.y);
        nd.c = make_float4(l1.z, h1.x, h1.y, h1.z);
        nd.d = make_int4(c0, c1, 0, 0);
        nodes[id] = nd;
        if (c0 < 0) leaf_parent[~c0] = id; else node_parent[c0] = id;
        if (c1 < 0) leaf_parent[~c1] = id; else node_parent[c1] = id;
        P.cl[out][o] = id;
        P.cb[out][2 * o] = make_float4(fminf(l0.x, l1.x), fminf(l0.y, l1.y), fminf(l0.z, l1.z), 0.0f);
        P.cb[out][2 * o + 1] = make_float4(fmaxf(h0.x, h1.x), fmaxf(h0.y, h1.y), fmaxf(h0.z, h1.z), 0.0f);
      } else {
        P.cl[out][o] = cl[i];
        P.cb[out][2 * o] = cb[2 * i];
        P.cb[out][2 * o + 1] = cb[2 * i + 1];
      }
    }
    keep_at += tot & 0xffff;
    made_at += tot >> 16;
  }
}

__global__ void k_ploc_done(const PlocState* st, int32_t* levels, int iters) {
  if (threadIdx.x == 0) levels[iters] = st->made;
}

// Refit of the nodes made in clustering iteration t: their children were
// made in earlier iterations (refitted by earlier launches) or are leaves.
__global__ void __launch_bounds__(256) k_refit_level(int64_t n, const float* box, const int32_t* perm, Node* nodes,
                                                    const int32_t* levels, int t) {
  const int k0 = levels[t], k1 = levels[t + 1];
  for (int k = k0 + (int)(blockIdx.x * blockDim.x + threadIdx.x); k < k1; k += (int)(gridDim.x * blockDim.x)) {
    const int id = (int)(n - 2) - k;
    Node& nd = nodes[id];
    float lo[2][3], hi[2][3];
    const int ch[2] = {nd.d.x, nd.d.y};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (ch[c] < 0) {
        const int64_t i = perm[~ch[c]];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          lo[c][a] = box[a * n + i];
          hi[c][a] = box[(3 + a) * n + i];
        }
      } else {
        const Node& cn = nodes[ch[c]];
        const float4 A = cn.a, Bv = cn.b, C = cn.c;
        lo[c][0] = fminf(A.x, Bv.z);
        lo[c][1] = fminf(A.y, Bv.w);
        lo[c][2] = fminf(A.z, C.x);
        hi[c][0] = fmaxf(A.w, C.y);
        hi[c][1] = fmaxf(Bv.x, C.z);
        hi[c][2] = fmaxf(Bv.y, C.w);
      }
    }
    nd.a = make_float4(lo[0][0], lo[0][1], lo[0][2], hi[0][0]);
    nd.b = make_float4(hi[0][1], hi[0][2], lo[1][0], lo[1][1]);
    nd.c = make_float4(lo[1][2], hi[1][0], hi[1][1], hi[1][2]);
  }
}

__global__ void k_records(eag_surfels s, const int32_t* perm, Record* recs) {
  const int64_t n = s.n;
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t i = perm[j];
  float4* r = reinterpret_cast<float4*>(recs + j);
  r[0] = make_float4(s.pos[i], s.pos[n + i], s.pos[2 * n + i], s.opacity[i]);
  r[1] = make_float4(s.rot[i], s.rot[n + i], s.rot[2 * n + i], s.rot[3 * n + i]);
  r[2] = make_float4(s.scale[i], s.scale[n + i], __uint_as_float((uint32_t)i), 0.0f);
}

__global__ void k_zero_i32(int32_t* p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_depth(int64_t n, const int32_t* leaf_parent, const int32_t* node_parent, BvhHeader* h) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  int d = 0;
  int p = leaf_parent[j];
  while (p >= 0) {
    ++d;
    p = node_parent[p];
  }
  atomicMax(&h->max_depth, d);
}

__global__ void k_attrs(eag_surfels s, const int32_t* perm, Attr* attrs) {
  const int64_t n = s.n;
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t i = perm[j];
  float4* a = reinterpret_cast<float4*>(attrs + j);
  a[0] = make_float4(s.albedo[i], s.albedo[n + i], s.albedo[2 * n + i], s.emissive[i]);
  a[1] = make_float4(s.radiance[i], s.radiance[n + i], s.radiance[2 * n + i], 0.0f);
}

// ---------------------------------------------------------------------------
// Collapse of the binary tree into a 4-wide tree, level by level. A queue
// entry (binary internal node b, 4-wide node m) expands b's two children;
// while fewer than four children are held and one of them is an internal
// binary node, the internal child with the largest box surface area is
// replaced by its two children. Internal children left over become 4-wide
// nodes of the next level.
// ---------------------------------------------------------------------------
struct Collapse {
  int2* q[2];         // ping-pong queues of (binary node, 4-wide node)
  int32_t* counts;    // counts[l] = entries of level l; counts[MAXL] = nodes allocated
};
constexpr int COLLAPSE_MAXL = 128;

__device__ __forceinline__ void child_box(const Node& nd, int slot, float* lo, float* hi) {
  const float* f = reinterpret_cast<const float*>(&nd);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = f[slot * 6 + a];
    hi[a] = f[slot * 6 + 3 + a];
  }
}

__device__ __forceinline__ float half_area(const float* lo, const float* hi) {
  const float dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
  return dx * dy + dy * dz + dz * dx;
}

__global__ void k_collapse_init(int32_t* counts, int2* q0) {
  const int i = threadIdx.x;
  for (int k = i; k <= COLLAPSE_MAXL; k += blockDim.x) counts[k] = 0;
  if (i == 0) {
    q0[0] = make_int2(0, 0);
  }
  __syncthreads();
  if (i == 0) {
    counts[0] = 1;
    counts[COLLAPSE_MAXL] = 1;   // node 0 is the root
  }
}

__global__ void k_collapse_level(const Node* bin, Node4* out, Collapse cq, int level) {
  const int count = cq.counts[level];
  const int2* qin = cq.q[level & 1];
  int2* qout = cq.q[(level + 1) & 1];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < count; e += gridDim.x * blockDim.x) {
    const int2 job = qin[e];
    int ref[4];
    float lo[4][3], hi[4][3];
    int cnt = 2;
    ref[0] = bin[job.x].d.x;
    ref[1] = bin[job.x].d.y;
    child_box(bin[job.x], 0, lo[0], hi[0]);
    child_box(bin[job.x], 1, lo[1], hi[1]);
    while (cnt < 4) {
      int best = -1;
      float area = -1.0f;
      for (int k = 0; k < cnt; ++k) {
        if (ref[k] >= 0) {
          const float a = half_area(lo[k], hi[k]);
          if (a > area) { area = a; best = k; }
        }
      }
      if (best < 0) break;
      const Node& nb = bin[ref[best]];
      ref[cnt] = nb.d.y;
      child_box(nb, 1, lo[cnt], hi[cnt]);
      ref[best] = nb.d.x;
      child_box(nb, 0, lo[best], hi[best]);
      ++cnt;
    }
    Node4& m = out[job.y];
    float* bf = reinterpret_cast<float*>(m.b);
    int dst[4], src[4];
    for (int k = 0; k < 4; ++k) {
      if (k < cnt) {
        for (int a = 0; a < 3; ++a) {
          bf[k * 6 + a] = lo[k][a];
          bf[k * 6 + 3 + a] = hi[k][a];
        }
        src[k] = ref[k];
        if (ref[k] >= 0) {
          const int id = atomicAdd(&cq.counts[COLLAPSE_MAXL], 1);
          const int slot = atomicAdd(&cq.counts[level + 1], 1);
          qout[slot] = make_int2(ref[k], id);
          dst[k] = id;
        } else {
          dst[k] = ref[k];
        }
      } else {
        for (int a = 0; a < 6; ++a) bf[k * 6 + a] = 0.0f;
        src[k] = NODE4_EMPTY;
        dst[k] = NODE4_EMPTY;
      }
    }
    m.ref = make_int4(dst[0], dst[1], dst[2], dst[3]);
    m.src = make_int4(src[0], src[1], src[2], src[3]);
  }
}

// Refit of 4-wide boxes from the binary tree (internal children) and the
// surfel boxes (leaves).
__global__ void k_node4_boxes(const Node* bin, Node4* out, const BvhHeader* h, const float* box,
                              const int32_t* perm, int64_t n) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= h->n_nodes4) return;
  Node4& nd = out[m];
  const int s[4] = {nd.src.x, nd.src.y, nd.src.z, nd.src.w};
  float* bf = reinterpret_cast<float*>(nd.b);
  for (int k = 0; k < 4; ++k) {
    if (s[k] == NODE4_EMPTY) continue;
    float lo[3], hi[3];
    if (s[k] >= 0) {
      float l2[3], h2[3];
      child_box(bin[s[k]], 0, lo, hi);
      child_box(bin[s[k]], 1, l2, h2);
      for (int a = 0; a < 3; ++a) {
        lo[a] = fminf(lo[a], l2[a]);
        hi[a] = fmaxf(hi[a], h2[a]);
      }
    } else {
      const int64_t i = perm[~s[k]];
      for (int a = 0; a < 3; ++a) {
        lo[a] = box[a * n + i];
        hi[a] = box[(3 + a) * n + i];
      }
    }
    for (int a = 0; a < 3; ++a) {
      bf[k * 6 + a] = lo[a];
      bf[k * 6 + 3 + a] = hi[a];
    }
  }
}

__global__ void k_collapse_finish(const int32_t* counts, BvhHeader* h) {
  if (threadIdx.x == 0) {
    h->n_nodes4 = counts[COLLAPSE_MAXL];
    int l = 0;
    while (l < COLLAPSE_MAXL && counts[l] > 0) ++l;
    h->depth4 = l;
  }
}

inline unsigned blocks(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

struct BuildWs {
  int2* q0;
  int2* q1;
  int32_t* counts;
  float* box;
  uint64_t* codes_in;
  uint64_t* codes_out;
  uint32_t* ids_in;
  int32_t* nn;
  float4* cbox[2];
  int32_t* bsum;
  int32_t* boff;
  PlocState* ploc;
  void* sort_tmp;
  size_t sort_bytes;
  size_t bytes;
};

BuildWs build_ws(void* base, int64_t n) {
  Carver c(base, ~size_t(0));
  BuildWs w;
  w.q0 = c.take<int2>(n);
  w.q1 = c.take<int2>(n);
  w.counts = c.take<int32_t>(COLLAPSE_MAXL + 1);
  w.box = c.take<float>(6 * n);
  w.codes_in = c.take<uint64_t>(n);
  w.codes_out = c.take<uint64_t>(n);
  w.ids_in = c.take<uint32_t>(n);
  w.nn = c.take<int32_t>(n);
  w.cbox[0] = c.take<float4>(2 * n);
  w.cbox[1] = c.take<float4>(2 * n);
  w.bsum = c.take<int32_t>(2 * PLOC_GRID);
  w.boff = c.take<int32_t>(2 * PLOC_GRID);
  w.ploc = c.take<PlocState>(1);
  w.sort_bytes = sort_pairs_bytes(n);
  w.sort_tmp = c.take<char>(w.sort_bytes);
  w.bytes = c.bytes();
  return w;
}

// The clustering's state in the build workspace. The collapse queues are
// free while it runs and hold the two cluster orders.
Ploc ploc_ws(const BuildWs& w) {
  Ploc P;
  P.cl[0] = reinterpret_cast<int32_t*>(w.q0);
  P.cl[1] = reinterpret_cast<int32_t*>(w.q1);
  P.cb[0] = w.cbox[0];
  P.cb[1] = w.cbox[1];
  P.nn = w.nn;
  P.bsum = w.bsum;
  P.boff = w.boff;
  P.st = w.ploc;
  return P;
}

// Levels the collapse is launched for: the clustering's tree is at most
// PLOC_ITERS + ceil(log2 n) <= PLOC_ITERS + idx_bits levels high, and a
// 4-wide level spans at least one binary level. Levels past the tree's depth
// find an empty queue and return at once.
int collapse_levels(int32_t idx_bits) { return std::min(COLLAPSE_MAXL, PLOC_ITERS + idx_bits); }
static_assert(PLOC_ITERS + 23 <= COLLAPSE_MAXL, "the collapse covers the deepest tree of 2^23 surfels");
static_assert(PLOC_ITERS + 23 <= PLOC_LEVELS, "levels has an entry per clustering iteration of 2^23 surfels");

}  // namespace

BvhLayout bvh_layout(void* base, int64_t n) {
  Carver c(base, ~size_t(0));
  BvhLayout l;
  l.hdr = c.take<BvhHeader>(1);
  l.nodes = c.take<Node>(n > 1 ? n - 1 : 1);
  l.nodes4 = c.take<Node4>(n > 1 ? n - 1 : 1);
  l.recs = c.take<Record>(n);
  l.perm = c.take<int32_t>(n);
  l.leaf_parent = c.take<int32_t>(n);
  l.node_parent = c.take<int32_t>(n > 1 ? n - 1 : 1);
  l.levels = c.take<int32_t>(PLOC_LEVELS + 1);
  l.bytes = c.bytes();
  return l;
}

void bvh_attach(eag_bvh* b, const BvhLayout& l) {
  b->hdr = l.hdr;
  b->nodes = l.nodes;
  b->nodes4 = l.nodes4;
  b->recs = l.recs;
  b->perm = l.perm;
  b->leaf_parent = l.leaf_parent;
  b->node_parent = l.node_parent;
  b->levels = l.levels;
}

size_t build_ws_bytes(int64_t n) { return build_ws(nullptr, n).bytes; }

void validate_surfels(const eag_surfels* s) {
  if (!s) fail(EAG_ERR_INVALID_ARGUMENT, "surfels is null");
  if (s->n < 1 || s->n > (int64_t(1) << 23)) fail(EAG_ERR_INVALID_ARGUMENT, "surfel count must be in [1, 2^23]");
  if (!s->pos || !s->rot || !s->scale || !s->opacity || !s->albedo || !s->radiance || !s->emissive)
    fail(EAG_ERR_INVALID_ARGUMENT, "a surfel array pointer is null");
}

static void geometry_pass(const eag_surfels* s, eag_bvh* b, const BuildWs& w, hipStream_t st) {
  const int64_t n = s->n;
  hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, st, b->hdr);
  hipLaunchKernelGGL(k_boxes, dim3(blocks(n)), dim3(256), 0, st, *s, 3.0f, w.box, b->hdr);
}

void build_bvh(const eag_surfels* s, eag_bvh* b, void* ws, size_t ws_bytes, hipStream_t st) {
  const int64_t n = s->n;
  if (!b->hdr || !b->nodes || !b->nodes4 || !b->recs || !b->perm || !b->leaf_parent || !b->node_parent || !b->levels)
    fail(EAG_ERR_INTERNAL, "bvh handle without its device arrays");
  BuildWs w = build_ws(ws, n);
  if (ws_bytes < w.bytes) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "build workspace too small");
  geometry_pass(s, b, w, st);
  hipLaunchKernelGGL(k_morton, dim3(blocks(n)), dim3(256), 0, st, *s, b->hdr, w.codes_in, w.ids_in);
  sort_pairs_u64(w.codes_in, w.codes_out, w.ids_in, reinterpret_cast<uint32_t*>(b->perm), n, 63, w.sort_tmp,
                 w.sort_bytes, st);
  if (n > 1) {
    const Ploc P = ploc_ws(w);
    hipLaunchKernelGGL(k_ploc_init, dim3(blocks(n)), dim3(256), 0, st, n, w.box, b->perm, P, b->node_parent);
    const unsigned g = std::min<unsigned>(blocks(n, PLOC_TILE), (unsigned)PLOC_GRID);
    const int iters = PLOC_ITERS + b->idx_bits;
    for (int t = 0; t < iters; ++t) {
      hipLaunchKernelGGL(k_ploc_nn, dim3(g), dim3(PLOC_TILE), 0, st, P, t >= PLOC_ITERS ? 1 : 0);
      hipLaunchKernelGGL(k_ploc_count, dim3(g), dim3(PLOC_TILE), 0, st, P);
      hipLaunchKernelGGL(k_ploc_scan, dim3(1), dim3(PLOC_GRID), 0, st, P, (int)g, t, b->levels);
      hipLaunchKernelGGL(k_ploc_write, dim3(g), dim3(PLOC_TILE), 0, st, P, n, b->nodes, b->leaf_parent,
                         b->node_parent);
    }
    hipLaunchKernelGGL(k_ploc_done, dim3(1), dim3(64), 0, st, (const PlocState*)P.st, b->levels, iters);
  } else {
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, b->leaf_parent, (int64_t)1);
  }
  hipLaunchKernelGGL(k_records, dim3(blocks(n)), dim3(256), 0, st, *s, b->perm, b->recs);
  if (n > 1)
    hipLaunchKernelGGL(k_depth, dim3(blocks(n)), dim3(256), 0, st, n, b->leaf_parent, b->node_parent, b->hdr);
  check_hip(hipGetLastError(), "build launch");
  b->root = n > 1 ? 0 : ~0;
  if (n > 1) {
    Collapse cq{{w.q0, w.q1}, w.counts};
    hipLaunchKernelGGL(k_collapse_init, dim3(1), dim3(256), 0, st, w.counts, w.q0);
    const unsigned g = std::min<unsigned>(blocks(n), 1024u);
    const int levels = collapse_levels(b->idx_bits);
    for (int level = 0; level < levels; ++level)
      hipLaunchKernelGGL(k_collapse_level, dim3(g), dim3(256), 0, st, b->nodes, b->nodes4, cq, level);
    hipLaunchKernelGGL(k_collapse_finish, dim3(1), dim3(64), 0, st, w.counts, b->hdr);
    check_hip(hipGetLastError(), "collapse launch");
  }
  check_hip(hipEventRecord(b->built, st), "build event");
}

void refit_bvh(const eag_surfels* s, eag_bvh* b, void* ws, size_t ws_bytes, hipStream_t st) {
  const int64_t n = s->n;
  if (!b->hdr || !b->nodes || !b->nodes4 || !b->recs || !b->perm || !b->levels)
    fail(EAG_ERR_INTERNAL, "bvh handle without its device arrays");
  BuildWs w = build_ws(ws, n);
  if (ws_bytes < w.bytes) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "refit workspace too small");
  BvhHeader* h = b->hdr;
  // bounds are recomputed; the depths and node count stay, since the
  // topology is unchanged
  hipLaunchKernelGGL(k_reset_bounds, dim3(1), dim3(64), 0, st, h);
  hipLaunchKernelGGL(k_boxes, dim3(blocks(n)), dim3(256), 0, st, *s, 3.0f, w.box, h);
  hipLaunchKernelGGL(k_records, dim3(blocks(n)), dim3(256), 0, st, *s, b->perm, b->recs);
  if (n > 1) {
    // iteration by iteration of the clustering that made the tree
    const unsigned g = std::min<unsigned>(blocks(n), 1024u);
    const int iters = PLOC_ITERS + b->idx_bits;
    for (int t = 0; t < iters; ++t)
      hipLaunchKernelGGL(k_refit_level, dim3(g), dim3(256), 0, st, n, (const float*)w.box, (const int32_t*)b->perm,
                         b->nodes, (const int32_t*)b->levels, t);
    // (the 4-wide node count is on the device: the grid covers the n - 1 it
    // can reach)
    hipLaunchKernelGGL(k_node4_boxes, dim3(blocks(n - 1)), dim3(256), 0, st, b->nodes, b->nodes4, h, w.box,
                       b->perm, n);
  }
  check_hip(hipGetLastError(), "refit launch");
  check_hip(hipEventRecord(b->built, st), "refit event");
}

void pack_attrs(const eag_surfels* s, const eag_bvh* b, Attr* attrs, hipStream_t st) {
  hipLaunchKernelGGL(k_attrs, dim3(blocks(s->n)), dim3(256), 0, st, *s, b->perm, attrs);
}

}  // namespace eag
