// knn_fused_linf_s.hip -- fused kernel instantiations: infinity norm, vector ALU; register merge only.
#include "knn_fused.h"

namespace knn {

hipError_t launch_fused_linf_s(const FusedParams& p, hipStream_t stream) {
  return dispatch_ng<TILE_LINF_F32, true, 1,2,3,4,5,6,7,8>(p, stream);
}

}  // namespace knn
