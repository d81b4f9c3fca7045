// The noise-free Grover search by the diffusion identity: a labelled variant of
// the HALL-based iteration, not the paper's form.
//
// One iteration is G = HALL . Inv . HALL . Oracle (Sec. 5.1).  With Inv =
// 2|0><0| - I (Eq. inversion) and HALL|0..0> = |s>, the uniform state (Eq.
// Shor1), HALL . Inv . HALL = 2|s><s| - I, so
//     (G C)_n = 2 m - (O C)_n,   m = mean over n of (O C)_n,
// where O flips the marked amplitudes.  A step is then one streaming pass: read
// C, write 2m - C, and sum the written values block by block for the next mean.
// The marked labels (a handful) are fixed afterwards by a one-workgroup kernel:
// the pass wrote w_x = 2m - C_x where 2m + C_x was due, so c_x = 4m - w_x, and the
// next mean is (sum of the pass - 4 m |M|) / N, since w_x + c_x = 4m.  Sums are
// FP64 (also for FP32 states) in a fixed order.
#include <hip/hip_runtime.h>

#include "pk_launch.h"

namespace pk {

namespace {

constexpr int kThreads = 256;
constexpr int kGrid = 2048;  // blocks of the streaming kernels (and partial sums)

template <typename T>
__device__ __forceinline__ double2 wide(const T& v) {
    return double2{(double)v.x, (double)v.y};
}

// Sum of a block's values (FP64), written to part[blockIdx.x] by thread 0.
__device__ __forceinline__ void block_sum2(double2 acc, double2* part) {
    __shared__ double2 red[kThreads / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        acc.x += __shfl_xor(acc.x, off, 64);
        acc.y += __shfl_xor(acc.y, off, 64);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double2 t = {0.0, 0.0};
        for (int w = 0; w < kThreads / 64; ++w) {
            t.x += red[w].x;
            t.y += red[w].y;
        }
        part[blockIdx.x] = t;
    }
}

// Block b owns the contiguous chunk [b * chunk, (b + 1) * chunk) of the state.
template <typename T>
__global__ void __launch_bounds__(kThreads) sum_kernel(const T* src, int64_t n, int64_t chunk, double2* part) {
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    double2 acc = {0.0, 0.0};
    for (int64_t e = lo + threadIdx.x; e < hi; e += kThreads) {
        const double2 v = wide(src[e]);
        acc.x += v.x;
        acc.y += v.y;
    }
    block_sum2(acc, part);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) diffuse_kernel(const T* src, T* dst, int64_t n, int64_t chunk,
                                                           const double2* mean, double2* part) {
    using R = decltype(src[0].x);
    const double2 m = *mean;
    const R mx = (R)(2.0 * m.x), my = (R)(2.0 * m.y);
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    double2 acc = {0.0, 0.0};
    for (int64_t e = lo + threadIdx.x; e < hi; e += kThreads) {
        const T v = src[e];
        T w;
        w.x = mx - v.x;
        w.y = my - v.y;
        dst[e] = w;
        acc.x += (double)w.x;
        acc.y += (double)w.y;
    }
    block_sum2(acc, part);
}

// mode 0 (start): m = (sum - 2 sum_x C_x) / N, the mean of O psi_in.
// mode 1 (after a pass): c_x = 4 m - w_x at the marked labels; m' = (sum - 4 m |M|) / N;
//                        L = sum_x |c_x|^2.
template <typename T>
__global__ void __launch_bounds__(kThreads) combine_kernel(const double2* part, int nparts, MarkedSet ms, T* state,
                                                           int64_t n, double2* mean, double* L, int mode) {
    using R = decltype(state[0].x);
    // the partial sums: lane l adds parts l, l + 64, ..., then a butterfly (fixed order);
    // all of a lane's loads are issued before the first add, so their latencies overlap
    constexpr int kPer = kGrid / 64;
    double2 pv[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int b = threadIdx.x + 64 * j;
        pv[j] = b < nparts ? part[b] : double2{0.0, 0.0};
    }
    double2 s = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < kPer; ++j)
        if (threadIdx.x + 64 * j < nparts) {
            s.x += pv[j].x;
            s.y += pv[j].y;
        }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        s.x += __shfl_xor(s.x, off, 64);
        s.y += __shfl_xor(s.y, off, 64);
    }
    if (threadIdx.x != 0) return;
    const double2 m = *mean;
    double l = 0.0;
    if (mode == 0) {
        for (int i = 0; i < ms.count; ++i) {
            const double2 c = wide(state[ms.label[i]]);
            s.x -= 2.0 * c.x;
            s.y -= 2.0 * c.y;
            l += c.x * c.x + c.y * c.y;
        }
    } else {
        for (int i = 0; i < ms.count; ++i) {
            const double2 w = wide(state[ms.label[i]]);
            T c;
            c.x = (R)(4.0 * m.x - w.x);
            c.y = (R)(4.0 * m.y - w.y);
            state[ms.label[i]] = c;
            l += (double)c.x * (double)c.x + (double)c.y * (double)c.y;
        }
        s.x -= 4.0 * m.x * ms.count;
        s.y -= 4.0 * m.y * ms.count;
    }
    *mean = double2{s.x / (double)n, s.y / (double)n};
    *L = l;
}

template <typename T>
hipError_t search_t(const void* psi_in, void* psi_out, int64_t n, const MarkedSet& ms, int64_t iters,
                    double2* part, double2* mean, double* L, hipStream_t st) {
    const int64_t chunk = (n + kGrid - 1) / kGrid;
    const int grid = (int)((n + chunk - 1) / chunk);
    const T* in = static_cast<const T*>(psi_in);
    T* out = static_cast<T*>(psi_out);
    hipLaunchKernelGGL(sum_kernel<T>, dim3(grid), dim3(kThreads), 0, st, in, n, chunk, part);
    hipLaunchKernelGGL(combine_kernel<T>, dim3(1), dim3(64), 0, st, part, grid, ms, const_cast<T*>(in), n, mean, L,
                       0);
    for (int64_t k = 0; k < iters; ++k) {
        hipLaunchKernelGGL(diffuse_kernel<T>, dim3(grid), dim3(kThreads), 0, st, k == 0 ? in : out, out, n, chunk,
                           mean, part);
        hipLaunchKernelGGL(combine_kernel<T>, dim3(1), dim3(64), 0, st, part, grid, ms, out, n, mean, L, 1);
    }
    return hipGetLastError();
}

}  // namespace

size_t search_workspace_bytes() { return (size_t)(kGrid + 2) * sizeof(double2); }

hipError_t launch_search(const void* psi_in, void* psi_out, int nq, bool fp64, const MarkedSet& ms, int64_t iters,
                         void* workspace, double* L, hipStream_t st) {
    double2* part = static_cast<double2*>(workspace);
    double2* mean = part + kGrid;
    const int64_t n = (int64_t)1 << nq;
    return fp64 ? search_t<double2>(psi_in, psi_out, n, ms, iters, part, mean, L, st)
                : search_t<float2>(psi_in, psi_out, n, ms, iters, part, mean, L, st);
}

}  // namespace pk
