// In-place attribute edits (relighting, switching lights off, recolouring):
// one thread per edited surfel.
#include "eag_device.h"
#include "eag_internal.h"
#include "eag_render.h"

namespace eag {

namespace {

__global__ void k_edit(eag_edit e, eag_surfel_attrs a) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= e.count) return;
  const int64_t i = e.idx[k];
  if (i < 0 || i >= a.n) return;  // out-of-range indices are ignored
  const int64_t n = a.n;
  switch (e.kind) {
    case EAG_EDIT_SET_RADIANCE:
      a.radiance[i] = e.value[0]; a.radiance[n + i] = e.value[1]; a.radiance[2 * n + i] = e.value[2];
      break;
    case EAG_EDIT_SCALE_RADIANCE:
      a.radiance[i] *= e.value[0]; a.radiance[n + i] *= e.value[1]; a.radiance[2 * n + i] *= e.value[2];
      break;
    case EAG_EDIT_SET_ALBEDO:
      a.albedo[i] = e.value[0]; a.albedo[n + i] = e.value[1]; a.albedo[2 * n + i] = e.value[2];
      break;
    case EAG_EDIT_SET_EMISSIVE:
      a.emissive[i] = e.value[0];
      break;
    default:
      break;
  }
}

}  // namespace

void launch_apply_edit(const eag_edit& e, const eag_surfel_attrs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_edit, dim3((unsigned)((e.count + 255) / 256)), dim3(256), 0, st, e, a);
  check_hip(hipGetLastError(), "edit launch");
}

}  // namespace eag
