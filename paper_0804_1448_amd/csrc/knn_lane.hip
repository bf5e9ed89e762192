// knn_lane.hip -- instantiations of the one-query-per-lane Manhattan and
// infinity-norm kernel (knn_lane.h) for padded dimensions 16 .. 128.
#include "knn_lane.h"

namespace knn {

template <int KIND, int T>
static hipError_t dispatch_ng(const FusedParams& p, hipStream_t stream) {
  switch (p.ng) {
    case 1: return launch_lane_one<KIND, 1, T>(p, stream);
    case 2: return launch_lane_one<KIND, 2, T>(p, stream);
    case 3: return launch_lane_one<KIND, 3, T>(p, stream);
    case 4: return launch_lane_one<KIND, 4, T>(p, stream);
    case 5: return launch_lane_one<KIND, 5, T>(p, stream);
    case 6: return launch_lane_one<KIND, 6, T>(p, stream);
    case 7: return launch_lane_one<KIND, 7, T>(p, stream);
    case 8: return launch_lane_one<KIND, 8, T>(p, stream);
    default: return hipErrorInvalidValue;
  }
}

// p.cb carries the queue size
template <int KIND>
static hipError_t dispatch_queue(const FusedParams& p, hipStream_t stream) {
  if (p.cb == 8) return dispatch_ng<KIND, 8>(p, stream);
  if (p.cb == 12) return dispatch_ng<KIND, 12>(p, stream);
  return hipErrorInvalidValue;
}

hipError_t launch_lane(int kind, const FusedParams& p, hipStream_t stream) {
  if (kind == TILE_L1_F32) return dispatch_queue<TILE_L1_F32>(p, stream);
  if (kind == TILE_LINF_F32) return dispatch_queue<TILE_LINF_F32>(p, stream);
  return hipErrorInvalidValue;
}

size_t lane_lds(int waves, int kc, int queue) { return lane_lds_bytes(waves, kc, queue); }

}  // namespace knn
