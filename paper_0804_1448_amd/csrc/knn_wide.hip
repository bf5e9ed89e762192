// knn_wide.hip -- the 32x32-tile Euclidean kernel with register-resident
// lists (knn_wide.h): dispatch by tile kind, and the one-launch batched
// kernel (16-bit tiles, dp = 32..128, k' <= 128).  The single-instance
// kernels are built in knn_wide_bf16.hip, knn_wide_f16.hip (dp = 32, 64, 96,
// 128, k' <= 128) and knn_wide_f32.hip (dp = 16..128, k' <= 64).
#include "knn_wide.h"

namespace knn {

hipError_t launch_wide(int kind, const FusedParams& p, hipStream_t stream) {
  if (kind == TILE_L2_F32) return p.kc_max <= kWideMaxKc1 ? launch_wide_f32(p, stream) : hipErrorInvalidValue;
  if (p.kc_max > kWideMaxKc) return hipErrorInvalidValue;
  if (p.counter) {
    if (!p.items) return hipErrorInvalidValue;
    if (kind == TILE_L2_BF16) return launch_wide_batch_one<TILE_L2_BF16>(p, stream);
    if (kind == TILE_L2_F16) return launch_wide_batch_one<TILE_L2_F16>(p, stream);
    return hipErrorInvalidValue;
  }
  if (kind == TILE_L2_BF16) return launch_wide_bf16(p, stream);
  if (kind == TILE_L2_F16) return launch_wide_f16(p, stream);
  return hipErrorInvalidValue;
}

}  // namespace knn
