// knn_fused_f16_s.hip -- fused kernel instantiations: float16 Euclidean; register merge only.
#include "knn_fused.h"

namespace knn {

hipError_t launch_fused_f16_s(const FusedParams& p, hipStream_t stream) {
  return dispatch_ng<TILE_L2_F16, true, 1,2,3,4,5,6,7,8>(p, stream);
}

}  // namespace knn
