// Stage-0 radiant-scene objective (Sec. 3.2, Eq. 4) on the images of the
// camera segment, per pixel: Nt = N/|N|, Dt = D/A, R, E (Sec. 3.1, Eq. 3).
//
// k_stage0_images  forward state of the camera pass -> images [pixel][8].
// k_stage0_count   pixels that carry the normal term (hit) and the
//                  distance-normal term (hit, inside, four hit neighbours);
//                  counts = {hit, valid, all pixels}.
// k_stage0_loss    per pixel: lc |PQ(R) - PQ(R_gt)| over 3 M values,
//                  ln (1 - Nt.N_mono) over hit pixels, le |E - M| over M
//                  pixels, ld (1 - N_d.N_mono) over valid pixels; writes the
//                  image gradient of the pixel's own terms and, for the
//                  distance normal, the four contributions to its
//                  neighbours' Dt (contrib), and adds the loss.
// k_stage0_gather  adds each pixel's Dt contributions from its neighbours.
//
// The distance normal: X = O + Dt W for each pixel's ray, N_d =
// normalize((X(x+1,y) - X(x-1,y)) x (X(x,y+1) - X(x,y-1))), turned to face the
// camera (N_d.W <= 0). PQ as in light baking (ST 2084, Y = L / 10000, slope
// at max(Y, 2^-24)). Double precision throughout.
#include "eag_device.h"
#include "eag_internal.h"
#include "eag_render.h"

namespace eag {

namespace {

constexpr double S0_M1 = 2610.0 / 16384.0;
constexpr double S0_M2 = 2523.0 / 4096.0 * 128.0;
constexpr double S0_C1 = 3424.0 / 4096.0;
constexpr double S0_C2 = 2413.0 / 4096.0 * 32.0;
constexpr double S0_C3 = 2392.0 / 4096.0 * 32.0;
constexpr double S0_PEAK = 10000.0;
constexpr double S0_YMIN = 5.9604644775390625e-08;   // 2^-24

__device__ __forceinline__ double pq_value(double L) {
  const double ym = pow(fmax(L, 0.0) / S0_PEAK, S0_M1);
  return pow((S0_C1 + S0_C2 * ym) / (1.0 + S0_C3 * ym), S0_M2);
}

__device__ __forceinline__ double pq_deriv(double L) {
  if (L < 0.0) return 0.0;
  const double y = fmax(L / S0_PEAK, S0_YMIN);
  const double ym = pow(y, S0_M1);
  const double num = S0_C1 + S0_C2 * ym, den = 1.0 + S0_C3 * ym;
  const double dbase = (S0_C2 * den - S0_C3 * num) / (den * den);
  return S0_M2 * pow(num / den, S0_M2 - 1.0) * dbase * (S0_M1 * ym / y) / S0_PEAK;
}

__device__ __forceinline__ bool is_hit(const float* img) {
  return img[0] != 0.0f || img[1] != 0.0f || img[2] != 0.0f;   // Nt is a unit vector on hit pixels
}

// pixel g = (c, y, x) of a stack of n_cams images of W x H
__device__ __forceinline__ bool dn_valid(const float* images, int64_t g, int64_t W, int64_t H) {
  const int64_t hw = W * H, p = g % hw, x = p % W, y = p / W;
  if (x <= 0 || x >= W - 1 || y <= 0 || y >= H - 1) return false;
  return is_hit(images + g * STAGE0_FLOATS) && is_hit(images + (g - 1) * STAGE0_FLOATS) &&
         is_hit(images + (g + 1) * STAGE0_FLOATS) && is_hit(images + (g - W) * STAGE0_FLOATS) &&
         is_hit(images + (g + W) * STAGE0_FLOATS);
}

__global__ void k_stage0_images(const float* state, int64_t n_pix, float* images) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n_pix) return;
  const FwdState st = load_state(state + g * EAG_FWD_PIXEL_FLOATS);
  float* o = images + g * STAGE0_FLOATS;
  const bool hit = st.A > 0.0;
  o[0] = hit ? (float)st.Nt.x : 0.0f;
  o[1] = hit ? (float)st.Nt.y : 0.0f;
  o[2] = hit ? (float)st.Nt.z : 0.0f;
  o[3] = hit ? (float)st.Dt : 0.0f;
  o[4] = hit ? (float)st.R.x : 0.0f;
  o[5] = hit ? (float)st.R.y : 0.0f;
  o[6] = hit ? (float)st.R.z : 0.0f;
  o[7] = hit ? st.E : 0.0f;
}

__global__ void k_stage0_count(const float* images, int64_t n_pix, int64_t W, int64_t H, unsigned long long* counts) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool in = g < n_pix;
  const bool hit = in && is_hit(images + g * STAGE0_FLOATS);
  const bool valid = in && dn_valid(images, g, W, H);
  const uint64_t bh = __ballot(hit), bv = __ballot(valid);
  if ((threadIdx.x & 63) == 0) {
    if (bh) atomicAdd(&counts[0], (unsigned long long)__popcll(bh));
    if (bv) atomicAdd(&counts[1], (unsigned long long)__popcll(bv));
  }
}

__device__ __forceinline__ D3 pixel_point(const CamDev& c, int64_t p, double Dt, const SbParams& sp, D3& Wd) {
  Wd = pixel_dir(c, (uint32_t)p, 0, sp.flags, sp.k0, sp.k1);
  return d3(c.eye[0] + Dt * Wd.x, c.eye[1] + Dt * Wd.y, c.eye[2] + Dt * Wd.z);
}

// One camera batch: pixels g0 + [0, nb) of the whole stack.
__global__ void __launch_bounds__(256) k_stage0_loss(const float* images, const float* rgb_gt, const float* n_mono,
                                                    const float* mask, const CamBatch cams, int64_t g0, int64_t nb,
                                                    int64_t W, int64_t H, SbParams sp, double lc, double ln, double ld,
                                                    double le, const unsigned long long* counts, float* contrib,
                                                    float* dimg, double* loss) {
  __shared__ double part[4];
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (j < nb) {
    const int64_t g = g0 + j, hw = W * H;
    const double M = (double)counts[2];
    const double nh = (double)counts[0], nv = (double)counts[1];
    const float* im = images + g * STAGE0_FLOATS;
    float* d = dimg + g * STAGE0_FLOATS;
    // colour: mean over 3 M values
    for (int k = 0; k < 3; ++k) {
      const double diff = pq_value(im[4 + k]) - pq_value(rgb_gt[g * 3 + k]);
      acc += lc * fabs(diff) / (3.0 * M);
      d[4 + k] = (float)(lc / (3.0 * M) * (diff > 0.0 ? 1.0 : (diff < 0.0 ? -1.0 : 0.0)) * pq_deriv(im[4 + k]));
    }
    // emission: mean over M pixels
    const double de = (double)im[7] - (double)mask[g];
    acc += le * fabs(de) / M;
    d[7] = (float)(le / M * (de > 0.0 ? 1.0 : (de < 0.0 ? -1.0 : 0.0)));
    // shading normal: mean over hit pixels
    const D3 nm = d3(n_mono[g * 3 + 0], n_mono[g * 3 + 1], n_mono[g * 3 + 2]);
    if (is_hit(im)) {
      acc += ln * (1.0 - ((double)im[0] * nm.x + (double)im[1] * nm.y + (double)im[2] * nm.z)) / nh;
      d[0] = (float)(-ln / nh * nm.x);
      d[1] = (float)(-ln / nh * nm.y);
      d[2] = (float)(-ln / nh * nm.z);
    } else {
      d[0] = d[1] = d[2] = 0.0f;
    }
    d[3] = 0.0f;   // Dt: the distance-normal terms are gathered afterwards
    float* cb = contrib + g * 4;
    cb[0] = cb[1] = cb[2] = cb[3] = 0.0f;
    if (dn_valid(images, g, W, H)) {
      const CamDev& c = cams.c[j / hw];
      const int64_t p = g % hw;
      D3 Wl, Wr, Wu, Wdn, Wp;
      const D3 Xl = pixel_point(c, p - 1, images[(g - 1) * STAGE0_FLOATS + 3], sp, Wl);
      const D3 Xr = pixel_point(c, p + 1, images[(g + 1) * STAGE0_FLOATS + 3], sp, Wr);
      const D3 Xu = pixel_point(c, p - W, images[(g - W) * STAGE0_FLOATS + 3], sp, Wu);
      const D3 Xd = pixel_point(c, p + W, images[(g + W) * STAGE0_FLOATS + 3], sp, Wdn);
      Wp = pixel_dir(c, (uint32_t)p, 0, sp.flags, sp.k0, sp.k1);
      const D3 ex = Xr - Xl, ey = Xd - Xu;
      const D3 cr = cross(ex, ey);
      const double cl = sqrt(dot(cr, cr));
      D3 nd = (1.0 / cl) * cr;
      const double s = dot(nd, Wp) > 0.0 ? -1.0 : 1.0;
      nd = s * nd;
      acc += ld * (1.0 - dot(nd, nm)) / nv;
      // d/d nd of -ld/nv nd.nm, back through the flip and the normalisation
      const D3 gnd = (-ld / nv * s) * nm;
      const D3 nu = (1.0 / cl) * cr;
      const D3 gc = (1.0 / cl) * (gnd - dot(nu, gnd) * nu);
      const D3 gex = cross(ey, gc), gey = cross(gc, ex);
      // X = O + Dt W: dDt = dX . W
      cb[0] = (float)dot(gex, Wr);          // to the right neighbour
      cb[1] = (float)(-dot(gex, Wl));       // to the left neighbour
      cb[2] = (float)dot(gey, Wdn);         // to the neighbour below
      cb[3] = (float)(-dot(gey, Wu));       // to the neighbour above
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, part[0] + part[1] + part[2] + part[3]);
}

// dDt of pixel g: the contributions its neighbours' distance normals sent it.
__global__ void k_stage0_gather(const float* contrib, int64_t n_pix, int64_t W, int64_t H, float* dimg) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n_pix) return;
  const int64_t hw = W * H, p = g % hw, x = p % W, y = p / W;
  double s = 0.0;
  if (x >= 1) s += contrib[(g - 1) * 4 + 0];       // g is the right neighbour of g - 1
  if (x + 1 < W) s += contrib[(g + 1) * 4 + 1];    // the left neighbour of g + 1
  if (y >= 1) s += contrib[(g - W) * 4 + 2];       // below g - W
  if (y + 1 < H) s += contrib[(g + W) * 4 + 3];    // above g + W
  dimg[g * STAGE0_FLOATS + 3] = (float)s;
}

__global__ void k_set_u64(unsigned long long* p, unsigned long long v0, unsigned long long v1, unsigned long long v2) {
  if (threadIdx.x == 0) {
    p[0] = v0;
    p[1] = v1;
    p[2] = v2;
  }
}

__global__ void k_zero_f64_s0(double* p) {
  if (threadIdx.x == 0) p[0] = 0.0;
}

unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void launch_stage0_images(const float* state, int64_t n_pix, float* images, hipStream_t st) {
  if (n_pix > 0) hipLaunchKernelGGL(k_stage0_images, dim3(nblocks(n_pix)), dim3(256), 0, st, state, n_pix, images);
  check_hip(hipGetLastError(), "stage-0 images launch");
}

void launch_stage0_count(const float* images, int64_t n_pix, int64_t W, int64_t H, unsigned long long* counts,
                         double* loss, hipStream_t st) {
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, st, counts, 0ull, 0ull, (unsigned long long)n_pix);
  hipLaunchKernelGGL(k_zero_f64_s0, dim3(1), dim3(64), 0, st, loss);
  if (n_pix > 0)
    hipLaunchKernelGGL(k_stage0_count, dim3(nblocks(n_pix)), dim3(256), 0, st, images, n_pix, W, H, counts);
  check_hip(hipGetLastError(), "stage-0 count launch");
}

void launch_stage0_loss_batch(const float* images, const float* rgb_gt, const float* n_mono, const float* mask,
                              const CamBatch& cams, int64_t g0, int64_t nb, int64_t W, int64_t H, const SbParams& sp,
                              const double w[4], const unsigned long long* counts, float* contrib, float* dimg,
                              double* loss, hipStream_t st) {
  if (nb > 0)
    hipLaunchKernelGGL(k_stage0_loss, dim3(nblocks(nb)), dim3(256), 0, st, images, rgb_gt, n_mono, mask, cams, g0, nb,
                       W, H, sp, w[0], w[1], w[2], w[3], counts, contrib, dimg, loss);
  check_hip(hipGetLastError(), "stage-0 loss launch");
}

void launch_stage0_gather(const float* contrib, int64_t n_pix, int64_t W, int64_t H, float* dimg, hipStream_t st) {
  if (n_pix > 0) hipLaunchKernelGGL(k_stage0_gather, dim3(nblocks(n_pix)), dim3(256), 0, st, contrib, n_pix, W, H, dimg);
  check_hip(hipGetLastError(), "stage-0 gather launch");
}

}  // namespace eag
