// knn_lane.hip -- instantiations of the one-query-per-lane Manhattan and
// infinity-norm kernel (knn_lane.h) for padded dimensions 16 .. 128.
#include "knn_lane.h"

namespace knn {

template <int KIND>
static hipError_t dispatch_lane(const FusedParams& p, hipStream_t stream) {
  switch (p.ng) {
    case 1: return launch_lane_one<KIND, 1>(p, stream);
    case 2: return launch_lane_one<KIND, 2>(p, stream);
    case 3: return launch_lane_one<KIND, 3>(p, stream);
    case 4: return launch_lane_one<KIND, 4>(p, stream);
    case 5: return launch_lane_one<KIND, 5>(p, stream);
    case 6: return launch_lane_one<KIND, 6>(p, stream);
    case 7: return launch_lane_one<KIND, 7>(p, stream);
    case 8: return launch_lane_one<KIND, 8>(p, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_lane(int kind, const FusedParams& p, hipStream_t stream) {
  if (kind == TILE_L1_F32) return dispatch_lane<TILE_L1_F32>(p, stream);
  if (kind == TILE_LINF_F32) return dispatch_lane<TILE_LINF_F32>(p, stream);
  return hipErrorInvalidValue;
}

size_t lane_lds(int waves, int kc) { return lane_lds_bytes(waves, kc); }

}  // namespace knn
