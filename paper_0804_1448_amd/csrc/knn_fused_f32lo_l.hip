// knn_fused_f32lo_l.hip -- fused kernel instantiations: float32 Euclidean, chunks of 1-8 groups; rank merge for k' > 64.
#include "knn_fused.h"

namespace knn {

hipError_t launch_fused_f32lo_l(const FusedParams& p, hipStream_t stream) {
  return dispatch_ng<TILE_L2_F32, false, 1,2,3,4,5,6,7,8>(p, stream);
}

}  // namespace knn
