// knn_fused_l1_s.hip -- fused kernel instantiations: Manhattan, vector ALU; register merge only.
#include "knn_fused.h"

namespace knn {

hipError_t launch_fused_l1_s(const FusedParams& p, hipStream_t stream) {
  return dispatch_ng<TILE_L1_F32, true, 1,2,3,4,5,6,7,8>(p, stream);
}

}  // namespace knn
