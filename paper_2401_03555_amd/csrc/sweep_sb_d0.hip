// sweep_sb_d0.hip -- state-box sweep kernels for grid dimensions other than 2, 3 and 5,
// with and without a disturbance player (for the latter: any dimension but 2 and 3).
#include "sweep_sb.hpp"

namespace impact {

template hipError_t launch_sb_d<0>(const SweepArgs&, int, int64_t, int32_t, hipStream_t);
template hipError_t launch_sb_dist<0>(const SweepArgs&, int, int64_t, int32_t, hipStream_t);
template hipError_t launch_mq_sb_d<0>(const QueryDesc*, const QueryCtrl*, const int32_t*,
                                       const int32_t*, int64_t, double*, int64_t, int32_t,
                                       hipStream_t);

}  // namespace impact
