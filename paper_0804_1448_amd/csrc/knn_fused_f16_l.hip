// knn_fused_f16_l.hip -- fused kernel instantiations: float16 Euclidean; rank merge for k' > 64.
#include "knn_fused.h"

namespace knn {

hipError_t launch_fused_f16_l(const FusedParams& p, hipStream_t stream) {
  return dispatch_ng<TILE_L2_F16, false, 1,2,3,4,5,6,7,8>(p, stream);
}

}  // namespace knn
