// Kernel instances (pass f32r3) of the templates in pk_pass.h, in a translation unit of
// their own so that the build compiles them in parallel.
#include "pk_pass.h"

namespace pk {
template hipError_t launch_pass_r<float, 1, 3>(int, const KArgs&, int64_t, int64_t, hipStream_t);
}  // namespace pk
