// Kernel instances (batched f64) of the templates in pk_pass.h, in a translation unit of
// their own so that the build compiles them in parallel.
#include "pk_pass.h"

namespace pk {
template hipError_t launch_batched_r<double, 4>(int, const KArgs&, const BatchArgs&, unsigned, hipStream_t);
template hipError_t launch_batched_r<double, 5>(int, const KArgs&, const BatchArgs&, unsigned, hipStream_t);
template int batched_occupancy_r<double, 4>(int);
template int batched_occupancy_r<double, 5>(int);
}  // namespace pk
