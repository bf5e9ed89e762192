// knn_wide.hip -- instantiations of the 32x32-tile Euclidean kernel with
// register-resident lists (knn_wide.h): 16-bit tiles for dp = 32, 64, 96,
// 128 and k' <= 128 (one or two list keys per lane), also as the one-launch
// batched kernel; float32 tiles for dp = 16..128 and k' <= 64.
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

static hipError_t dispatch_f32(const FusedParams& p, hipStream_t stream) {
  switch (p.ng) {
    case 1: return launch_wide_one<TILE_L2_F32, 1>(p, stream);
    case 2: return launch_wide_one<TILE_L2_F32, 2>(p, stream);
    case 3: return launch_wide_one<TILE_L2_F32, 3>(p, stream);
    case 4: return launch_wide_one<TILE_L2_F32, 4>(p, stream);
    case 5: return launch_wide_one<TILE_L2_F32, 5>(p, stream);
    case 6: return launch_wide_one<TILE_L2_F32, 6>(p, stream);
    case 7: return launch_wide_one<TILE_L2_F32, 7>(p, stream);
    case 8: return launch_wide_one<TILE_L2_F32, 8>(p, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_wide(int kind, const FusedParams& p, hipStream_t stream) {
  if (kind == TILE_L2_F32) return p.kc_max <= kWideMaxKc1 ? dispatch_f32(p, stream) : hipErrorInvalidValue;
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
