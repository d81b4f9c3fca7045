// Arguments of the pass and batched kernels, and the launchers of their
// template instances.  The instances are compiled in separate translation units
// (pk_pass_*.hip) so that the build runs them in parallel; pk_kernels.hip picks
// the instance at run time.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pk_desc.h"
#include "pk_launch.h"

namespace pk {

struct KArgs {
    const Pass* passes;
    const Stage* stages;
    const Flip* flips;
    const PhaseOp* phases;
    const double* twid;  // product tables of the controlled phases (re, im pairs)
    const URef* urefs;   // tile-part tables of each pass
    const double* mats;
    const double* mats4;  // 4x4 complex matrices of two-qubit gates, 32 doubles each
    const void* src0;  // vector 0 input of the first pass
    void* dst0;        // vector 0 output (and input of later passes)
    void* dst1;        // vector 1 (lambda) in/out, backward only
    double* partials;
    double* reads;
    double* gpart;
    const double* dL;
    int32_t pass;
    int32_t want_norm;
};

// Sum of one double per thread over the workgroup; result valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double x, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wave] = x;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < (NT + 63) / 64; ++w) s += red[w];
    }
    __syncthreads();
    return s;
}

// One vector (psi) with RB = 4 or 5 register bits, or two vectors (psi and
// lambda) with 4: every tile size kmax the precision allows.
template <typename R, int NV, int RB>
hipError_t launch_pass_r(int kmax, const KArgs& a, int64_t ntiles, int64_t cap, hipStream_t st);
template <typename R, int RB>
hipError_t launch_batched_r(int kmax, const KArgs& a, const BatchArgs& B, unsigned grid, hipStream_t st);
template <typename R, int RB>
int batched_occupancy_r(int kmax);
template <typename R, int RB>
hipError_t launch_repeat_r(int kmax, const KArgs& a, const RepeatArgs& r, unsigned grid, hipStream_t st);
template <typename R, int RB>
int repeat_occupancy_r(int kmax);

}  // namespace pk
