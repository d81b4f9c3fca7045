// Kernel instances (pass f64, 2^12- and 2^13-amplitude tiles with 4 register bits)
// of the templates in pk_pass.h, apart from the smaller tiles' so that the build
// compiles them in parallel.
#include "pk_pass.h"

namespace pk {
template hipError_t launch_pass_t<double, 1, 12, 4>(const KArgs&, int64_t, int64_t, hipStream_t);
template hipError_t launch_pass_t<double, 1, 13, 4>(const KArgs&, int64_t, int64_t, hipStream_t);
}  // namespace pk
