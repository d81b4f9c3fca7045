// Kernel instances (repeat f32) of the templates in pk_pass.h, in a translation unit of
// their own so that the build compiles them in parallel.
#include "pk_pass.h"

namespace pk {
template hipError_t launch_repeat_r<float, 4>(int, const KArgs&, const RepeatArgs&, unsigned, hipStream_t);
template hipError_t launch_repeat_r<float, 5>(int, const KArgs&, const RepeatArgs&, unsigned, hipStream_t);
template int repeat_occupancy_r<float, 4>(int);
template int repeat_occupancy_r<float, 5>(int);
}  // namespace pk
