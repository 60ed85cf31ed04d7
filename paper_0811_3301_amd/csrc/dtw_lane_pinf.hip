// Instantiations of the lane-per-pair DTW kernel for p = infinity, band half-widths 0..kLaneMaxW.
#include "dtw_lane.h"

namespace lbimp {

hipError_t launch_dtw_lane_pinf(int w, int num_cu, const DtwArgs &a, hipStream_t s) {
    static const auto table = dtw_lane_table<kPInf>(std::make_integer_sequence<int, kLaneMaxW + 1>{});
    if (w < 0 || w > kLaneMaxW) return hipErrorInvalidValue;
    table[w](num_cu, a, s);
    return hipGetLastError();
}

}  // namespace lbimp
