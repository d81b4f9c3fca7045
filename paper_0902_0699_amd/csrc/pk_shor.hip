// Device kernels of Shor's data path (Sec. 5.2): the loaded two-register state
// (Step 3, Eq. Shor2) and the distribution of a measurement of register one
// (Step 6: p(n) = sum_k |C_{n,k}|^2).  The QFT between them (Step 5, App. A) is
// an ordinary gate list run by the pass kernels.
//
// Both kernels stream the state once at full width: the loader writes every
// amplitude (one 16- or 8-byte store per lane, lanes on consecutive labels), the
// marginal reads every amplitude the same way.  Neither needs LDS beyond a
// workgroup reduction, and neither touches the state twice.
#include <hip/hip_runtime.h>

#include "pk_launch.h"

namespace pk {

namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 16;  // stores per thread per block of the loader

// (a * b) mod M for a, b < M < 2^31: the product fits in 64 bits.
__device__ __forceinline__ uint64_t mulmod(uint64_t a, uint64_t b, uint64_t M) { return (a * b) % M; }

__device__ __forceinline__ uint64_t powmod(uint64_t x, uint64_t e, uint64_t M) {
    uint64_t r = 1 % M, b = x % M;
    while (e) {
        if (e & 1) r = mulmod(r, b, M);
        b = mulmod(b, b, M);
        e >>= 1;
    }
    return r;
}

// psi[n 2^n2 + k] = amp if k = f(n) = x^n mod M, else 0.  A block of the grid
// covers kThreads * kPerThread consecutive labels; thread t writes labels
// e0 + i * kThreads.  Along that sequence the register-one value n = e >> n2
// grows by 0 or 1 per step (rows longer than a block step) or by the constant
// g = kThreads >> n2 (shorter rows), so f follows by one multiplication by x or
// by xg = x^g mod M after a single modular power at the block's start.
template <typename T>
__global__ void __launch_bounds__(kThreads) shor_state_kernel(T* psi, int n2, uint64_t x, uint64_t xg, uint64_t M,
                                                              T amp, int64_t total) {
    using R = decltype(amp.x);
    const uint64_t mask = ((uint64_t)1 << n2) - 1;
    const int64_t step = (int64_t)kThreads * kPerThread;
    for (int64_t blk = (int64_t)blockIdx.x * step; blk < total; blk += (int64_t)gridDim.x * step) {
        const int64_t e0 = blk + threadIdx.x;
        uint64_t row = (uint64_t)e0 >> n2;
        uint64_t f = powmod(x, row, M);
#pragma unroll 4
        for (int i = 0; i < kPerThread; ++i) {
            const int64_t e = e0 + (int64_t)i * kThreads;
            if (e >= total) break;
            const uint64_t r = (uint64_t)e >> n2;
            if (r != row) {
                f = mulmod(f, r - row == 1 ? x % M : xg, M);
                row = r;
            }
            const bool hit = ((uint64_t)e & mask) == f;
            psi[e] = hit ? amp : T{(R)0, (R)0};
        }
    }
}

template <typename T>
__device__ __forceinline__ double norm2(const T& v) {
    const double x = (double)v.x, y = (double)v.y;
    return x * x + y * y;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// p[s] = sum over the 2^nl labels s 2^nl + k of |psi|^2, in FP64, in an order
// fixed by nl alone (deterministic).  Three shapes by segment length L = 2^nl:
//   L <= 64        each wave reads 64 consecutive amplitudes per step and sums
//                  groups of L lanes with butterflies;
//   64 < L < 2^14  one wave per segment, lanes striding by 64;
//   L >= 2^14      one workgroup per segment, then a workgroup reduction.
// Where segment s's sum goes: s, or s with its nh bits reversed (the register read
// in the opposite qubit order).
__device__ __forceinline__ int64_t out_index(int64_t s, int nh, bool bitrev) {
    if (!bitrev || nh == 0) return s;
    return (int64_t)(__brevll((unsigned long long)s) >> (64 - nh));
}

template <typename T>
__global__ void __launch_bounds__(kThreads) marginal_kernel(const T* psi, double* p, int nl, int64_t nseg, int nh,
                                                            bool bitrev) {
    __shared__ double red[kThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int nw = kThreads / 64;
    const int64_t L = (int64_t)1 << nl;
    if (nl <= 6) {
        const int64_t total = nseg << nl;
        for (int64_t base = ((int64_t)blockIdx.x * nw + wave) * 64; base < total;
             base += (int64_t)gridDim.x * nw * 64) {
            const int64_t e = base + lane;
            double v = e < total ? norm2(psi[e]) : 0.0;
            for (int off = 1; off < L; off <<= 1) v += __shfl_xor(v, off, 64);
            if ((lane & (L - 1)) == 0 && e < total) p[out_index(e >> nl, nh, bitrev)] = v;
        }
    } else if (nl < 14) {
        for (int64_t s = (int64_t)blockIdx.x * nw + wave; s < nseg; s += (int64_t)gridDim.x * nw) {
            const T* q = psi + (s << nl);
            double a0 = 0.0, a1 = 0.0;
            for (int64_t j = lane; j < L; j += 128) {  // L >= 128: both halves in range
                a0 += norm2(q[j]);
                a1 += norm2(q[j + 64]);
            }
            const double v = wave_sum(a0 + a1);
            if (lane == 0) p[out_index(s, nh, bitrev)] = v;
        }
    } else {
        for (int64_t s = blockIdx.x; s < nseg; s += gridDim.x) {
            const T* q = psi + (s << nl);
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            for (int64_t j = threadIdx.x; j < L; j += 4 * kThreads) {  // L >= 4 * kThreads
                a0 += norm2(q[j]);
                a1 += norm2(q[j + kThreads]);
                a2 += norm2(q[j + 2 * kThreads]);
                a3 += norm2(q[j + 3 * kThreads]);
            }
            const double v = wave_sum((a0 + a1) + (a2 + a3));
            if (lane == 0) red[wave] = v;
            __syncthreads();
            if (threadIdx.x == 0) {
                double t = 0.0;
                for (int w = 0; w < nw; ++w) t += red[w];
                p[out_index(s, nh, bitrev)] = t;
            }
            __syncthreads();
        }
    }
}

unsigned grid_for(int64_t work_blocks) {
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
    }
    const int64_t cap = (int64_t)ncu * 8;
    return (unsigned)(work_blocks < cap ? (work_blocks > 0 ? work_blocks : 1) : cap);
}

}  // namespace

hipError_t launch_shor_state(int n1, int n2, uint64_t x, uint64_t M, bool fp64, double amp, void* psi,
                             hipStream_t st) {
    const int64_t total = (int64_t)1 << (n1 + n2);
    const int64_t step = (int64_t)kThreads * kPerThread;
    const unsigned grid = grid_for((total + step - 1) / step);
    // x^(kThreads >> n2) mod M, the factor between the rows of consecutive steps when
    // rows are shorter than a step (unused otherwise)
    uint64_t xg = 1 % M;
    if (n2 < 8)
        for (int i = 0; i < (kThreads >> n2); ++i) xg = (xg * (x % M)) % M;
    if (fp64)
        hipLaunchKernelGGL(shor_state_kernel<double2>, dim3(grid), dim3(kThreads), 0, st,
                           static_cast<double2*>(psi), n2, x, xg, M, double2{amp, 0.0}, total);
    else
        hipLaunchKernelGGL(shor_state_kernel<float2>, dim3(grid), dim3(kThreads), 0, st, static_cast<float2*>(psi),
                           n2, x, xg, M, float2{(float)amp, 0.0f}, total);
    return hipGetLastError();
}

hipError_t launch_marginal(int nq, int nl, bool fp64, bool bitrev, const void* psi, double* p, hipStream_t st) {
    const int64_t nseg = (int64_t)1 << (nq - nl);
    int64_t blocks;
    if (nl <= 6)
        blocks = ((nseg << nl) + kThreads - 1) / kThreads;
    else if (nl < 14)
        blocks = (nseg + kThreads / 64 - 1) / (kThreads / 64);
    else
        blocks = nseg;
    const unsigned grid = grid_for(blocks);
    if (fp64)
        hipLaunchKernelGGL(marginal_kernel<double2>, dim3(grid), dim3(kThreads), 0, st,
                           static_cast<const double2*>(psi), p, nl, nseg, nq - nl, bitrev);
    else
        hipLaunchKernelGGL(marginal_kernel<float2>, dim3(grid), dim3(kThreads), 0, st,
                           static_cast<const float2*>(psi), p, nl, nseg, nq - nl, bitrev);
    return hipGetLastError();
}

}  // namespace pk
