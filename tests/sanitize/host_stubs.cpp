// Kernel launchers replaced for a host-only build of the C-ABI (argument
// checks, the float64 camera composition, error reporting), compiled with
// the address and undefined-behaviour sanitizers: every launch reports a
// failure, so only host code runs.
#include <hip/hip_runtime.h>

#include "uf_params.h"

namespace qk {
hipError_t launch_update_fuse(const UFParams &, int, int, int, bool, hipStream_t) {
    return hipErrorInvalidValue;
}
hipError_t launch_update_fuse_batch(const UFParams *, const UFBatch &, int, int, int, bool,
                                    hipStream_t) {
    return hipErrorInvalidValue;
}
hipError_t launch_fp8_scales(const F8Params &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_fold_weights(const FoldParams &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_composite(const CompParams &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_composite_backward(const CompBwdParams &, hipStream_t) {
    return hipErrorInvalidValue;
}
hipError_t launch_update_fuse_backward(const BwdParams &, hipStream_t) {
    return hipErrorInvalidValue;
}
hipError_t launch_ldm_init(const InitParams &, bool, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_render_ibr(const RenderParams &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_render_to_views(const ViewsParams &, hipStream_t) {
    return hipErrorInvalidValue;
}
hipError_t launch_residual_conv(const ConvParams &, int, bool, hipStream_t) {
    return hipErrorInvalidValue;
}
hipError_t launch_layer_collapse(const CollapseParams &, int, hipStream_t) {
    return hipErrorInvalidValue;
}
hipError_t launch_ray_encoding(const RayParams &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_upsample2x(const Up2Params &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_ldm_decode(const DecodeParams &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t scratch_address(int, float **out) {
    *out = nullptr;
    return hipErrorInvalidValue;
}
}  // namespace qk
