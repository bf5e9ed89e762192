// knn_lane_l2.hip -- instantiations of the float32 Euclidean kernel with
// per-lane selection (knn_lane_l2.h) for padded dimensions 16 .. 128.
#include "knn_lane_l2.h"

namespace knn {

template <int T, bool TILED>
static hipError_t dispatch_l2_ng(const FusedParams& p, hipStream_t stream) {
  switch (p.ng) {
    case 1: return launch_lane_l2_one<1, T, TILED>(p, stream);
    case 2: return launch_lane_l2_one<2, T, TILED>(p, stream);
    case 3: return launch_lane_l2_one<3, T, TILED>(p, stream);
    case 4: return launch_lane_l2_one<4, T, TILED>(p, stream);
    case 5: return launch_lane_l2_one<5, T, TILED>(p, stream);
    case 6: return launch_lane_l2_one<6, T, TILED>(p, stream);
    case 7: return launch_lane_l2_one<7, T, TILED>(p, stream);
    case 8: return launch_lane_l2_one<8, T, TILED>(p, stream);
    default: return hipErrorInvalidValue;
  }
}

// p.cb carries the queue size, p.tiled the reference layout
hipError_t launch_lane_l2(const FusedParams& p, hipStream_t stream) {
  if (p.cb == 8) return p.tiled ? dispatch_l2_ng<8, true>(p, stream) : dispatch_l2_ng<8, false>(p, stream);
  if (p.cb == 12) return p.tiled ? dispatch_l2_ng<12, true>(p, stream) : dispatch_l2_ng<12, false>(p, stream);
  return hipErrorInvalidValue;
}

}  // namespace knn
