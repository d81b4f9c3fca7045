// Kernel instances (pass f64) of the templates in pk_pass.h, in a translation unit of
// their own so that the build compiles them in parallel.  The 2^12- and 2^13-tile
// kernels, the largest, are compiled in pk_pass_f64t.hip.
#include "pk_pass.h"

namespace pk {
extern template hipError_t launch_pass_t<double, 1, 12, 4>(const KArgs&, int64_t, int64_t, hipStream_t);
extern template hipError_t launch_pass_t<double, 1, 13, 4>(const KArgs&, int64_t, int64_t, hipStream_t);
template hipError_t launch_pass_r<double, 1, 4>(int, const KArgs&, int64_t, int64_t, hipStream_t);
}  // namespace pk
