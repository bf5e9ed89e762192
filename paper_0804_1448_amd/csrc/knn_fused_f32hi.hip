// knn_fused_f32hi.hip -- instantiations of the fused kernel (float32 Euclidean tiles).
#include "knn_fused.h"

namespace knn {

hipError_t launch_fused_f32hi(int ng, const FusedParams& p, hipStream_t stream) {
  switch (ng) {
    case 9: return launch_fused_one<TILE_L2_F32, 9>(p, stream);
    case 10: return launch_fused_one<TILE_L2_F32, 10>(p, stream);
    case 11: return launch_fused_one<TILE_L2_F32, 11>(p, stream);
    case 12: return launch_fused_one<TILE_L2_F32, 12>(p, stream);
    case 13: return launch_fused_one<TILE_L2_F32, 13>(p, stream);
    case 14: return launch_fused_one<TILE_L2_F32, 14>(p, stream);
    case 15: return launch_fused_one<TILE_L2_F32, 15>(p, stream);
    case 16: return launch_fused_one<TILE_L2_F32, 16>(p, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace knn
