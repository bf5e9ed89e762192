// knn_fused_half.hip -- instantiations of the fused kernel (bfloat16 / float16 Euclidean tiles).
#include "knn_fused.h"

namespace knn {

template <int KIND>
static hipError_t dispatch(int ng, const FusedParams& p, hipStream_t stream) {
  switch (ng) {
    case 1: return launch_fused_one<KIND, 1>(p, stream);
    case 2: return launch_fused_one<KIND, 2>(p, stream);
    case 3: return launch_fused_one<KIND, 3>(p, stream);
    case 4: return launch_fused_one<KIND, 4>(p, stream);
    case 5: return launch_fused_one<KIND, 5>(p, stream);
    case 6: return launch_fused_one<KIND, 6>(p, stream);
    case 7: return launch_fused_one<KIND, 7>(p, stream);
    case 8: return launch_fused_one<KIND, 8>(p, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fused_half(int kind, int ng, const FusedParams& p, hipStream_t stream) {
  if (kind == TILE_L2_BF16) return dispatch<TILE_L2_BF16>(ng, p, stream);
  if (kind == TILE_L2_F16) return dispatch<TILE_L2_F16>(ng, p, stream);
  return hipErrorInvalidValue;
}

}  // namespace knn
