// sweep_sb_d3.hip -- state-box sweep kernels for grid dimension 3 (with and without a
// disturbance player).
#include "sweep_sb.hpp"

namespace impact {

template hipError_t launch_sb_d<3>(const SweepArgs&, int, int64_t, int32_t, hipStream_t);
template hipError_t launch_sb_dist<3>(const SweepArgs&, int, int64_t, int32_t, hipStream_t);
template hipError_t launch_mq_sb_d<3>(const QueryDesc*, const QueryCtrl*, const int32_t*,
                                       const int32_t*, int64_t, double*, int64_t, int32_t,
                                       hipStream_t);

}  // namespace impact
