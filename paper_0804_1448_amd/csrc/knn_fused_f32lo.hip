// knn_fused_f32lo.hip -- instantiations of the fused kernel (float32 Euclidean tiles).
#include "knn_fused.h"

namespace knn {

hipError_t launch_fused_f32lo(int ng, const FusedParams& p, hipStream_t stream) {
  switch (ng) {
    case 1: return launch_fused_one<TILE_L2_F32, 1>(p, stream);
    case 2: return launch_fused_one<TILE_L2_F32, 2>(p, stream);
    case 3: return launch_fused_one<TILE_L2_F32, 3>(p, stream);
    case 4: return launch_fused_one<TILE_L2_F32, 4>(p, stream);
    case 5: return launch_fused_one<TILE_L2_F32, 5>(p, stream);
    case 6: return launch_fused_one<TILE_L2_F32, 6>(p, stream);
    case 7: return launch_fused_one<TILE_L2_F32, 7>(p, stream);
    case 8: return launch_fused_one<TILE_L2_F32, 8>(p, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace knn
