// knn_wide.hip -- instantiations of the 32x32-tile Euclidean kernel with
// register-resident lists (knn_wide.h): 16-bit tiles for dp = 32, 64, 96,
// 128 and k' <= 128 (one or two list keys per lane), also as the one-launch
// batched kernel.  The float32 tiles (dp = 16..128, k' <= 64) are built in
// knn_wide_f32.hip.
#include "knn_wide.h"

namespace knn {

template <int KIND>
static hipError_t dispatch_half(const FusedParams& p, hipStream_t stream) {
  switch (p.ng) {
    case 2: return launch_wide_one<KIND, 2>(p, stream);
    case 4: return launch_wide_one<KIND, 4>(p, stream);
    case 6: return launch_wide_one<KIND, 6>(p, stream);
    case 8: return launch_wide_one<KIND, 8>(p, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_wide(int kind, const FusedParams& p, hipStream_t stream) {
  if (kind == TILE_L2_F32) return p.kc_max <= kWideMaxKc1 ? launch_wide_f32(p, stream) : hipErrorInvalidValue;
  if (p.kc_max > kWideMaxKc) return hipErrorInvalidValue;
  if (p.counter) {
    if (!p.items) return hipErrorInvalidValue;
    if (kind == TILE_L2_BF16) return launch_wide_batch_one<TILE_L2_BF16>(p, stream);
    if (kind == TILE_L2_F16) return launch_wide_batch_one<TILE_L2_F16>(p, stream);
    return hipErrorInvalidValue;
  }
  if (kind == TILE_L2_BF16) return dispatch_half<TILE_L2_BF16>(p, stream);
  if (kind == TILE_L2_F16) return dispatch_half<TILE_L2_F16>(p, stream);
  return hipErrorInvalidValue;
}

}  // namespace knn
