// knn_fused_f32hi_l.hip -- fused kernel instantiations: float32 Euclidean, chunks of 9-16 groups; rank merge for k' > 64.
#include "knn_fused.h"

namespace knn {

hipError_t launch_fused_f32hi_l(const FusedParams& p, hipStream_t stream) {
  return dispatch_ng<TILE_L2_F32, false, 9,10,11,12,13,14,15,16>(p, stream);
}

}  // namespace knn
