// knn_fused_f32hi_s.hip -- fused kernel instantiations: float32 Euclidean, chunks of 9-16 groups; register merge only.
#include "knn_fused.h"

namespace knn {

hipError_t launch_fused_f32hi_s(const FusedParams& p, hipStream_t stream) {
  return dispatch_ng<TILE_L2_F32, true, 9,10,11,12,13,14,15,16>(p, stream);
}

}  // namespace knn
