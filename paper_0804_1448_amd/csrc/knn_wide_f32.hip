// knn_wide_f32.hip -- instantiations of the 32x32-tile Euclidean kernel
// (knn_wide.h) for float32 tiles: dp = 16..128, k' <= 64 (a compile unit of
// its own, built beside knn_wide.hip).
#include "knn_wide.h"

namespace knn {

hipError_t launch_wide_f32(const FusedParams& p, hipStream_t stream) {
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

}  // namespace knn
