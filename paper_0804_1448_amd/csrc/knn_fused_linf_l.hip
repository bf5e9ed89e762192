// knn_fused_linf_l.hip -- fused kernel instantiations: infinity norm, vector ALU; rank merge for k' > 64.
#include "knn_fused.h"

namespace knn {

hipError_t launch_fused_linf_l(const FusedParams& p, hipStream_t stream) {
  return dispatch_ng<TILE_LINF_F32, false, 1,2,3,4,5,6,7,8>(p, stream);
}

}  // namespace knn
