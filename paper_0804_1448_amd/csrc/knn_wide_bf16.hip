// knn_wide_bf16.hip -- instantiations of the 32x32-tile Euclidean kernel (knn_wide.h)
// for BF16 tiles: dp = 32, 64, 96, 128, k' <= 128 (a compile unit of its
// own, built beside knn_wide.hip).
#include "knn_wide.h"

namespace knn {

hipError_t launch_wide_bf16(const FusedParams& p, hipStream_t stream) { return dispatch_half<TILE_L2_BF16>(p, stream); }

}  // namespace knn
