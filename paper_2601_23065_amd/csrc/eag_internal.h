// Host-side internals shared by the library's translation units: the BVH
// handle, memory carving helpers, launch wrappers and error plumbing.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/eag.h"

namespace eag {

struct Node;
struct Node4;
struct Record;
struct Attr;
struct CamDev;

// Thrown inside the library, converted to a status at the C boundary.
struct Error {
  eag_status status;
  std::string msg;
};
[[noreturn]] void fail(eag_status s, const std::string& msg);
void set_last_error(const std::string& msg);
void check_hip(hipError_t e, const char* what);

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Sequential carving of a caller-provided buffer into aligned pieces.
struct Carver {
  char* base;
  size_t used = 0;
  size_t cap;
  Carver(void* p, size_t c) : base(static_cast<char*>(p)), cap(c) {}
  template <class T>
  T* take(size_t count) {
    size_t off = align_up(used);
    used = off + count * sizeof(T);
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
  size_t bytes() const { return align_up(used); }
};

// Device-side header of a BVH allocation.
struct BvhHeader {
  uint32_t plo[3], phi[3];   // ordered-uint encoded centre bounds (Morton frame)
  uint32_t blo[3], bhi[3];   // ordered-uint encoded box bounds
  int32_t max_depth;
  int32_t n_nodes4;     // 4-wide nodes written by the collapse
  int32_t depth4;       // levels of the 4-wide tree
  int32_t pad;
};

}  // namespace eag

// Host handle of a BVH. Build and refit only enqueue work: the fields marked
// "synced" are filled from the device header by bvh_sync_host (which waits
// for the `built` event) and are read by host code that may wait.
struct eag_bvh {
  int64_t n;
  int32_t idx_bits;
  int32_t max_depth;      // synced
  int32_t root;
  float lo[3], hi[3];     // synced
  void* mem;
  size_t mem_bytes;
  eag::BvhHeader* hdr;
  eag::Node* nodes;
  eag::Node4* nodes4;
  int32_t n_nodes4;       // synced
  int32_t depth4;         // synced
  eag::Record* recs;
  int32_t* perm;
  int32_t* leaf_parent;
  int32_t* node_parent;
  int32_t* levels;        // internal nodes made before each clustering iteration
  hipEvent_t built = nullptr;   // recorded after the last build or refit
};

namespace eag {

// Device status codes (bits of the mapped status word).
constexpr unsigned int EAG_DEVICE_KEY_RANGE = 1u;
constexpr unsigned int EAG_DEVICE_SORT_RANGE = 2u;
unsigned int* device_status_word();     // allocates the word on first use
bool device_status_allocated();
void check_device_status();
// The no-allocation entry point's static scratch on the current device:
// setup looks its address up (once per device), the other returns it, or
// null before setup.
void noalloc_setup_current_device();
Attr* noalloc_scratch_current_device();
// Waits for the last build or refit and fills the handle's synced fields.
void bvh_sync_host(eag_bvh* b);
// Decodes a bound of the header (floats stored as order-preserving uints).
inline float header_float(uint32_t e) {
  const uint32_t bits = (e & 0x80000000u) ? (e & 0x7fffffffu) : ~e;
  float f;
  __builtin_memcpy(&f, &bits, 4);
  return f;
}

// Device-wide primitives (eag_prim.hip), deterministic, enqueued on the
// stream; tmp is a workspace of at least the size the *_bytes function
// gives for n. A scan may run in place (out == in). The sort is stable,
// orders by the keys' low end_bit bits and leaves its inputs unchanged.
size_t scan_u32_bytes(int64_t n);
size_t scan_f64_bytes(int64_t n);
void scan_u32(const uint32_t* in, uint32_t* out, int64_t n, bool inclusive, void* tmp, size_t tmp_bytes,
              hipStream_t st);
void scan_f64(const double* in, double* out, int64_t n, bool inclusive, void* tmp, size_t tmp_bytes,
              hipStream_t st);
size_t sort_pairs_bytes(int64_t n);
void sort_pairs_u64(const uint64_t* keys_in, uint64_t* keys_out, const uint32_t* vals_in, uint32_t* vals_out,
                    int64_t n, int end_bit, void* tmp, size_t tmp_bytes, hipStream_t st);

// Pieces of a BVH allocation of n surfels (base may be null to size it).
struct BvhLayout {
  BvhHeader* hdr;
  Node* nodes;
  Node4* nodes4;
  Record* recs;
  int32_t* perm;
  int32_t* leaf_parent;
  int32_t* node_parent;
  int32_t* levels;
  size_t bytes;
};
BvhLayout bvh_layout(void* base, int64_t n);
// Points a handle's device arrays at the pieces of its allocation.
void bvh_attach(eag_bvh* b, const BvhLayout& l);

size_t build_ws_bytes(int64_t n);
void validate_surfels(const eag_surfels* s);
void build_bvh(const eag_surfels* s, eag_bvh* b, void* ws, size_t ws_bytes, hipStream_t st);
void refit_bvh(const eag_surfels* s, eag_bvh* b, void* ws, size_t ws_bytes, hipStream_t st);

// Attribute records in sorted order (rho, e, r), refreshed by every render call.
void pack_attrs(const eag_surfels* s, const eag_bvh* b, Attr* attrs, hipStream_t st);

// Trace context parameters derived from a BVH and trace params.
struct TraceSetup {
  int32_t idx_bits;
  uint32_t max_bucket;
  double inv_dq;
};
TraceSetup trace_setup(const eag_bvh* b, const eag_trace_params* p);
void validate_params(const eag_trace_params* p);
CamDev make_cam(const eag_camera& c, uint32_t id);

void launch_trace_rays(const eag_bvh* b, const Attr* attrs, const eag_trace_params* p, const TraceSetup& ts,
                       int64_t n_rays, const double* o, const double* d, float* out, int32_t* hit_idx,
                       int32_t* hit_count, int32_t max_hits, int32_t* stats, hipStream_t st);

}  // namespace eag
