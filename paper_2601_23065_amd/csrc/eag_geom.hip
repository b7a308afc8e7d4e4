// Geometric scene edits (Sec. 1 and Sec. 5: moving, importing and deleting
// objects) and the tree cost that decides between refitting and rebuilding.
//
// k_box_flags / k_box_compact  surfels whose centre lies in [lo, hi]
//                              (compared in float32), ascending, via an
//                              exclusive scan of per-surfel flags.
// k_move                       p' = R(r)(p - pivot) + pivot + t, q' = r (x) q,
//                              in double precision, stored as float32.
// k_delete                     opacity 0 (the tracer skips such surfels).
// k_append                     the scene, then the moved copies of the
//                              selected surfels, into arrays of n + count.
// k_sah_sum / k_sah_final      1 + sum over all nodes of their children's box
//                              areas / the root's box area.
#include "eag_device.h"
#include "eag_internal.h"
#include "eag_render.h"

#include <cmath>


namespace eag {

namespace {

struct Rigid {
  double r[4];      // unit quaternion (w, x, y, z)
  double R[9];      // its rotation, row-major
  double pivot[3], t[3];
};

__global__ void k_box_flags(const float* pos, int64_t n, float3 lo, float3 hi, uint32_t* flags) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = pos[i], y = pos[n + i], z = pos[2 * n + i];
  flags[i] = (x >= lo.x && x <= hi.x && y >= lo.y && y <= hi.y && z >= lo.z && z <= hi.z) ? 1u : 0u;
}

__global__ void k_box_compact(const uint32_t* flags, const uint32_t* scan, int64_t n, int32_t* idx, int64_t* count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (flags[i]) idx[scan[i]] = (int32_t)i;
  if (i == n - 1) *count = (int64_t)scan[i] + (int64_t)flags[i];
}

__device__ __forceinline__ void move_one(const Rigid& m, const float* pin, const float* qin, int64_t ns, int64_t i,
                                         float* pout, float* qout, int64_t nd, int64_t j) {
  const double d0 = (double)pin[i] - m.pivot[0], d1 = (double)pin[ns + i] - m.pivot[1],
               d2 = (double)pin[2 * ns + i] - m.pivot[2];
  pout[j] = (float)(m.R[0] * d0 + m.R[1] * d1 + m.R[2] * d2 + m.pivot[0] + m.t[0]);
  pout[nd + j] = (float)(m.R[3] * d0 + m.R[4] * d1 + m.R[5] * d2 + m.pivot[1] + m.t[1]);
  pout[2 * nd + j] = (float)(m.R[6] * d0 + m.R[7] * d1 + m.R[8] * d2 + m.pivot[2] + m.t[2]);
  const double bw = qin[i], bx = qin[ns + i], by = qin[2 * ns + i], bz = qin[3 * ns + i];
  const double aw = m.r[0], ax = m.r[1], ay = m.r[2], az = m.r[3];
  qout[j] = (float)(aw * bw - ax * bx - ay * by - az * bz);
  qout[nd + j] = (float)(aw * bx + ax * bw + ay * bz - az * by);
  qout[2 * nd + j] = (float)(aw * by - ax * bz + ay * bw + az * bx);
  qout[3 * nd + j] = (float)(aw * bz + ax * by - ay * bx + az * bw);
}

__global__ void k_move(float* pos, float* rot, int64_t n, const int32_t* idx, int64_t count, Rigid m) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= count) return;
  const int64_t i = idx[k];
  if (i < 0 || i >= n) return;   // out-of-range indices are ignored
  move_one(m, pos, rot, n, i, pos, rot, n, i);
}

__global__ void k_delete(float* opacity, int64_t n, const int32_t* idx, int64_t count) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= count) return;
  const int64_t i = idx[k];
  if (i >= 0 && i < n) opacity[i] = 0.0f;
}

// Thread j < n copies surfel j; thread n + k writes the moved copy of idx[k].
__global__ void k_append(eag_surfels src, const int32_t* idx, int64_t count, eag_surfels_out dst, Rigid m) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t n = src.n, nd = dst.n;
  if (j >= n + count) return;
  const int64_t i = j < n ? j : (int64_t)idx[j - n];
  if (i < 0 || i >= n) return;   // an out-of-range index leaves its slot unwritten
  if (j < n) {
    for (int a = 0; a < 3; ++a) dst.pos[a * nd + j] = src.pos[a * n + i];
    for (int a = 0; a < 4; ++a) dst.rot[a * nd + j] = src.rot[a * n + i];
  } else {
    move_one(m, src.pos, src.rot, n, i, dst.pos, dst.rot, nd, j);
  }
  for (int a = 0; a < 2; ++a) dst.scale[a * nd + j] = src.scale[a * n + i];
  dst.opacity[j] = src.opacity[i];
  for (int a = 0; a < 3; ++a) dst.albedo[a * nd + j] = src.albedo[a * n + i];
  for (int a = 0; a < 3; ++a) dst.radiance[a * nd + j] = src.radiance[a * n + i];
  dst.emissive[j] = src.emissive[i];
}

__device__ __forceinline__ double box_area(double lx, double ly, double lz, double hx, double hy, double hz) {
  const double ex = fmax(hx - lx, 0.0), ey = fmax(hy - ly, 0.0), ez = fmax(hz - lz, 0.0);
  return 2.0 * (ex * ey + ey * ez + ez * ex);
}

// Child k of a 4-wide node: its box from the node's six float4.
__device__ __forceinline__ double child_area(const Node4& nd, int k) {
  const float4* b = nd.b;
  switch (k) {
    case 0: return box_area(b[0].x, b[0].y, b[0].z, b[0].w, b[1].x, b[1].y);
    case 1: return box_area(b[1].z, b[1].w, b[2].x, b[2].y, b[2].z, b[2].w);
    case 2: return box_area(b[3].x, b[3].y, b[3].z, b[3].w, b[4].x, b[4].y);
    default: return box_area(b[4].z, b[4].w, b[5].x, b[5].y, b[5].z, b[5].w);
  }
}

__global__ void __launch_bounds__(256) k_sah_sum(const Node4* nodes, const BvhHeader* h, int32_t root, double* acc) {
  __shared__ double part[4];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double a = 0.0;
  if (i < h->n_nodes4) {
    const Node4& nd = nodes[i];
    const int c[4] = {nd.ref.x, nd.ref.y, nd.ref.z, nd.ref.w};
    for (int k = 0; k < 4; ++k)
      if (c[k] != NODE4_EMPTY) a += child_area(nd, k);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&acc[0], part[0] + part[1] + part[2] + part[3]);
  if (i == root) {
    // the root's box: the union of its children's
    const Node4& nd = nodes[i];
    const int c[4] = {nd.ref.x, nd.ref.y, nd.ref.z, nd.ref.w};
    const float4* b = nd.b;
    const float lo[4][3] = {{b[0].x, b[0].y, b[0].z}, {b[1].z, b[1].w, b[2].x}, {b[3].x, b[3].y, b[3].z},
                            {b[4].z, b[4].w, b[5].x}};
    const float hi[4][3] = {{b[0].w, b[1].x, b[1].y}, {b[2].y, b[2].z, b[2].w}, {b[3].w, b[4].x, b[4].y},
                            {b[5].y, b[5].z, b[5].w}};
    double L[3] = {1e300, 1e300, 1e300}, H[3] = {-1e300, -1e300, -1e300};
    for (int k = 0; k < 4; ++k) {
      if (c[k] == NODE4_EMPTY) continue;
      for (int d = 0; d < 3; ++d) {
        L[d] = fmin(L[d], (double)lo[k][d]);
        H[d] = fmax(H[d], (double)hi[k][d]);
      }
    }
    acc[1] = box_area(L[0], L[1], L[2], H[0], H[1], H[2]);
  }
}

__global__ void k_sah_final(const double* acc, double* cost) {
  if (threadIdx.x == 0) cost[0] = acc[1] > 0.0 ? 1.0 + acc[0] / acc[1] : 1.0;
}

__global__ void k_sah_zero(double* acc) {
  if (threadIdx.x < 2) acc[threadIdx.x] = 0.0;
}

__global__ void k_sah_single(double* cost) {
  if (threadIdx.x == 0) cost[0] = 1.0;
}

unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

Rigid make_rigid(const float r[4], const float pivot[3], const float t[3]) {
  Rigid m;
  double q[4] = {r[0], r[1], r[2], r[3]};
  const double l = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (double& v : q) v /= l;
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                       2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                       2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
  for (int k = 0; k < 4; ++k) m.r[k] = q[k];
  for (int k = 0; k < 9; ++k) m.R[k] = R[k];
  for (int k = 0; k < 3; ++k) {
    m.pivot[k] = pivot[k];
    m.t[k] = t[k];
  }
  return m;
}

}  // namespace

size_t select_scan_bytes(int64_t n) { return scan_u32_bytes(n); }

void launch_select_box(const float* pos, int64_t n, const float lo[3], const float hi[3], uint32_t* flags,
                       uint32_t* scan, void* tmp, size_t tmp_bytes, int32_t* idx, int64_t* count, hipStream_t st) {
  hipLaunchKernelGGL(k_box_flags, dim3(nb(n)), dim3(256), 0, st, pos, n, make_float3(lo[0], lo[1], lo[2]),
                     make_float3(hi[0], hi[1], hi[2]), flags);
  scan_u32(flags, scan, n, false, tmp, tmp_bytes, st);
  hipLaunchKernelGGL(k_box_compact, dim3(nb(n)), dim3(256), 0, st, flags, scan, n, idx, count);
  check_hip(hipGetLastError(), "selection launch");
}

void launch_move(float* pos, float* rot, int64_t n, const int32_t* idx, int64_t count, const float r[4],
                 const float pivot[3], const float t[3], hipStream_t st) {
  if (count > 0)
    hipLaunchKernelGGL(k_move, dim3(nb(count)), dim3(256), 0, st, pos, rot, n, idx, count, make_rigid(r, pivot, t));
  check_hip(hipGetLastError(), "move launch");
}

void launch_delete(float* opacity, int64_t n, const int32_t* idx, int64_t count, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_delete, dim3(nb(count)), dim3(256), 0, st, opacity, n, idx, count);
  check_hip(hipGetLastError(), "delete launch");
}

void launch_append(const eag_surfels& src, const int32_t* idx, int64_t count, const eag_surfels_out& dst,
                   const float r[4], const float pivot[3], const float t[3], hipStream_t st) {
  hipLaunchKernelGGL(k_append, dim3(nb(src.n + count)), dim3(256), 0, st, src, idx, count, dst,
                     make_rigid(r, pivot, t));
  check_hip(hipGetLastError(), "append launch");
}

void launch_sah_cost(const Node4* nodes, const BvhHeader* h, int64_t max_nodes, int32_t root, double* acc,
                     double* cost, hipStream_t st) {
  if (root < 0 || max_nodes <= 0) {
    hipLaunchKernelGGL(k_sah_single, dim3(1), dim3(64), 0, st, cost);
  } else {
    // the node count is in the device header: the grid covers the most there can be
    hipLaunchKernelGGL(k_sah_zero, dim3(1), dim3(64), 0, st, acc);
    hipLaunchKernelGGL(k_sah_sum, dim3(nb(max_nodes)), dim3(256), 0, st, nodes, h, root, acc);
    hipLaunchKernelGGL(k_sah_final, dim3(1), dim3(64), 0, st, acc, cost);
  }
  check_hip(hipGetLastError(), "tree cost launch");
}

}  // namespace eag
