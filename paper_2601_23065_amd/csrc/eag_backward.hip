// Single-bounce adjoint (placeholder until the adjoint kernels land).
#include "eag_device.h"
#include "eag_internal.h"
#include "eag_render.h"

namespace eag {

void launch_single_bounce_backward(const TraceCtx&, const eag_surfels&, const CamBatch&, int64_t, int32_t,
                                   const SbParams&, const float*, const float*, const float*,
                                   const eag_surfel_grads&, float*, hipStream_t) {
  fail(EAG_ERR_INTERNAL, "single-bounce backward is not available in this build");
}

}  // namespace eag
