// Device-wide scans and a radix sort, written for 64-wide waves. All of them
// are deterministic: a scan adds in a fixed tree order whatever the device
// load, and the sort is stable. They run on the caller's stream and take
// their scratch memory from a caller's workspace.
//
// scan (inclusive or exclusive, uint32 or double):
//   1. k_scan_reduce: each block sums a tile of SCAN_TILE elements;
//   2. the block sums are scanned (exclusive) by the same scan, recursively,
//      until one tile holds them;
//   3. k_scan_tile: each block scans its tile and adds its block's offset.
//
// radix sort of (uint64 key, uint32 value) pairs by the key's low end_bit
// bits, least significant digit first, 8 bits per pass:
//   1. k_rs_hist: per block and digit, the count of the block's tile of
//      RS_TILE keys, stored digit-major (digit d of block b at d * B + b),
//      so that one exclusive scan gives every (digit, block) its first
//      output position;
//   2. that scan;
//   3. k_rs_scatter: each block ranks its keys in tile order: in rounds of
//      256 keys, the lanes of a wave with equal digits find each other
//      with eight ballots (one per digit bit), count their lower peers, and
//      the waves' counts per digit are combined through LDS.
#include <hip/hip_runtime.h>

#include "eag_internal.h"

namespace eag {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;
constexpr int RS_BITS = 8;
constexpr int RS_BINS = 1 << RS_BITS;
constexpr int RS_WAVES = RS_THREADS / 64;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Exclusive scan of one value per thread over a block of SCAN_THREADS
// threads (four waves); the block total goes to *total.
template <class T>
__device__ __forceinline__ T block_exclusive(T v, T* lds, T* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T t = __shfl_up(x, o);
    if (lane >= o) x += t;
  }
  if (lane == 63) lds[w] = x;
  T ex = __shfl_up(x, 1);   // the lower lanes' sum, exactly as added above
  if (lane == 0) ex = T(0);
  __syncthreads();
  T before = T(0);
  for (int k = 0; k < w; ++k) before += lds[k];
  *total = ((lds[0] + lds[1]) + lds[2]) + lds[3];
  __syncthreads();
  return before + ex;
}

template <class T>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(const T* in, int64_t n, T* sums) {
  __shared__ T lds[SCAN_THREADS / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  T s = T(0);
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k)
    if (base + k < n) s += in[base + k];
  T total;
  block_exclusive(s, lds, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// offsets: the exclusive scan of the block sums (null for one block).
template <class T>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_tile(const T* in, T* out, int64_t n, const T* offsets,
                                                            int inclusive) {
  __shared__ T lds[SCAN_THREADS / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  T v[SCAN_ITEMS];
  T s = T(0);
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = base + k < n ? in[base + k] : T(0);
    s += v[k];
  }
  T total;
  T run = block_exclusive(s, lds, &total);
  if (offsets) run = offsets[blockIdx.x] + run;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const T next = run + v[k];
    if (base + k < n) out[base + k] = inclusive ? next : run;
    run = next;
  }
}

template <class T>
size_t scan_bytes(int64_t n) {
  const int64_t b = ceil_div(n, SCAN_TILE);
  if (b <= 1) return 0;
  return align_up((size_t)b * sizeof(T)) + scan_bytes<T>(b);
}

template <class T>
void scan(const T* in, T* out, int64_t n, bool inclusive, void* tmp, size_t tmp_bytes, hipStream_t st) {
  if (n <= 0) return;
  const int64_t b = ceil_div(n, SCAN_TILE);
  if (tmp_bytes < scan_bytes<T>(n)) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "scan workspace too small");
  if (b > 0x7fffffff) fail(EAG_ERR_INVALID_ARGUMENT, "scan too long");
  if (b == 1) {
    hipLaunchKernelGGL(k_scan_tile<T>, dim3(1), dim3(SCAN_THREADS), 0, st, in, out, n, (const T*)nullptr,
                       inclusive ? 1 : 0);
    return;
  }
  T* sums = static_cast<T*>(tmp);
  const size_t own = align_up((size_t)b * sizeof(T));
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)b), dim3(SCAN_THREADS), 0, st, in, n, sums);
  scan<T>(sums, sums, b, false, static_cast<char*>(tmp) + own, tmp_bytes - own, st);
  hipLaunchKernelGGL(k_scan_tile<T>, dim3((unsigned)b), dim3(SCAN_THREADS), 0, st, in, out, n, (const T*)sums,
                     inclusive ? 1 : 0);
}

__device__ __forceinline__ uint32_t digit_of(uint64_t key, int shift, uint32_t mask) {
  return (uint32_t)(key >> shift) & mask;
}

__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const uint64_t* keys, int64_t n, int shift, uint32_t mask,
                                                       uint32_t* hist, int64_t blocks) {
  __shared__ uint32_t cnt[RS_BINS];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = base + r * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&cnt[digit_of(keys[i], shift, mask)], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * blocks + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(const uint64_t* kin, const uint32_t* vin, uint64_t* kout,
                                                          uint32_t* vout, int64_t n, int shift, uint32_t mask,
                                                          const uint32_t* offs, int64_t blocks, unsigned int* status) {
  __shared__ uint32_t run[RS_BINS];
  __shared__ uint32_t cnt[RS_WAVES][RS_BINS];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  run[t] = offs[(int64_t)t * blocks + blockIdx.x];
  const uint64_t below = (1ull << lane) - 1ull;
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
#pragma unroll
    for (int k = 0; k < RS_WAVES; ++k) cnt[k][t] = 0;
    __syncthreads();
    const int64_t i = base + r * RS_THREADS + t;
    const bool valid = i < n;
    uint64_t key = 0;
    uint32_t val = 0;
    if (valid) {
      key = kin[i];
      val = vin[i];
    }
    const uint32_t d = digit_of(key, shift, mask);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < RS_BITS; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & below);
    const bool last = valid && (peers >> lane) == 1ull;   // highest lane of its group
    if (last) cnt[w][d] = rank + 1;
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank;
      for (int k = 0; k < w; ++k) pos += cnt[k][d];
      if (pos < (uint64_t)n) {
        kout[pos] = key;
        vout[pos] = val;
      } else {
        __hip_atomic_fetch_or(status, EAG_DEVICE_SORT_RANGE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
    __syncthreads();
    run[t] += cnt[0][t] + cnt[1][t] + cnt[2][t] + cnt[3][t];
    __syncthreads();
  }
}

struct SortWs {
  uint64_t* keys;
  uint32_t* vals;
  uint32_t* hist;
  void* scan_tmp;
  size_t scan_bytes;
  size_t bytes;
};

SortWs sort_ws(void* base, int64_t n) {
  Carver c(base, ~size_t(0));
  SortWs w;
  const int64_t blocks = ceil_div(n, RS_TILE);
  w.keys = c.take<uint64_t>(n);
  w.vals = c.take<uint32_t>(n);
  w.hist = c.take<uint32_t>(RS_BINS * blocks);
  w.scan_bytes = scan_bytes<uint32_t>(RS_BINS * blocks);
  w.scan_tmp = c.take<char>(w.scan_bytes);
  w.bytes = c.bytes();
  return w;
}

}  // namespace

size_t scan_u32_bytes(int64_t n) { return scan_bytes<uint32_t>(n); }
size_t scan_f64_bytes(int64_t n) { return scan_bytes<double>(n); }

void scan_u32(const uint32_t* in, uint32_t* out, int64_t n, bool inclusive, void* tmp, size_t tmp_bytes,
              hipStream_t st) {
  scan<uint32_t>(in, out, n, inclusive, tmp, tmp_bytes, st);
  check_hip(hipGetLastError(), "scan launch");
}

void scan_f64(const double* in, double* out, int64_t n, bool inclusive, void* tmp, size_t tmp_bytes,
              hipStream_t st) {
  scan<double>(in, out, n, inclusive, tmp, tmp_bytes, st);
  check_hip(hipGetLastError(), "scan launch");
}

size_t sort_pairs_bytes(int64_t n) { return sort_ws(nullptr, n).bytes; }

void sort_pairs_u64(const uint64_t* keys_in, uint64_t* keys_out, const uint32_t* vals_in, uint32_t* vals_out,
                    int64_t n, int end_bit, void* tmp, size_t tmp_bytes, hipStream_t st) {
  if (n <= 0) return;
  if (n > 0x7fffffff) fail(EAG_ERR_INVALID_ARGUMENT, "sort too long");
  if (end_bit < 1 || end_bit > 64) fail(EAG_ERR_INVALID_ARGUMENT, "sort bit range must be in [1, 64]");
  const SortWs w = sort_ws(tmp, n);
  if (tmp_bytes < w.bytes) fail(EAG_ERR_WORKSPACE_TOO_SMALL, "sort workspace too small");
  const int64_t blocks = ceil_div(n, RS_TILE);
  const int passes = (end_bit + RS_BITS - 1) / RS_BITS;
  unsigned int* status = device_status_word();
  // ping-pong so that the last pass writes the output
  const uint64_t* ks = keys_in;
  const uint32_t* vs = vals_in;
  bool to_out = (passes & 1) != 0;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * RS_BITS;
    const int bits = end_bit - shift < RS_BITS ? end_bit - shift : RS_BITS;
    const uint32_t mask = (1u << bits) - 1u;
    uint64_t* kd = to_out ? keys_out : w.keys;
    uint32_t* vd = to_out ? vals_out : w.vals;
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)blocks), dim3(RS_THREADS), 0, st, ks, n, shift, mask, w.hist,
                       blocks);
    scan<uint32_t>(w.hist, w.hist, RS_BINS * blocks, false, w.scan_tmp, w.scan_bytes, st);
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)blocks), dim3(RS_THREADS), 0, st, ks, vs, kd, vd, n, shift,
                       mask, (const uint32_t*)w.hist, blocks, status);
    ks = kd;
    vs = vd;
    to_out = !to_out;
  }
  check_hip(hipGetLastError(), "sort launch");
}

}  // namespace eag
