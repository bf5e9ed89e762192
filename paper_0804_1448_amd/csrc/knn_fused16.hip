// knn_fused16.hip -- instantiations of the 16-bit Euclidean kernel with
// register-resident lists (knn_fused16.h): dp = 32, 64, 96, 128.
#include "knn_fused16.h"

namespace knn {

template <int KIND>
static hipError_t dispatch16(const FusedParams& p, hipStream_t stream) {
  switch (p.ng) {
    case 2: return launch_fused16_one<KIND, 2>(p, stream);
    case 4: return launch_fused16_one<KIND, 4>(p, stream);
    case 6: return launch_fused16_one<KIND, 6>(p, stream);
    case 8: return launch_fused16_one<KIND, 8>(p, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fused16(int kind, const FusedParams& p, hipStream_t stream) {
  if (kind == TILE_L2_BF16) return dispatch16<TILE_L2_BF16>(p, stream);
  if (kind == TILE_L2_F16) return dispatch16<TILE_L2_F16>(p, stream);
  return hipErrorInvalidValue;
}

}  // namespace knn
