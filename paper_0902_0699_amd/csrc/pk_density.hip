// The ensemble density matrix of Sec. 6.1 on FP64 matrix cores, and its spectrum.
//
//     <n|rho|n'> = sum_a P_a C_a(n) C_a^*(n')
//
// With C_a = X_a + i Y_a this is four real products over the universes a:
//     Re rho = (P X)^T X + (P Y)^T Y,     Im rho = (P Y)^T X - (P X)^T Y,
// a dense contraction of depth A (the number of universes), so it runs on
// v_mfma_f64_16x16x4f64.  rho is Hermitian: only blocks on or below the
// diagonal are computed, and each is written twice (as itself and as its
// conjugate transpose); on the diagonal the imaginary part is exactly zero and
// is written as such.
//
// Tiling: a workgroup of four waves owns a 64 x 64 block of rho.  The universes
// are consumed 8 at a time: the block's 64 row labels and 64 column labels of
// those 8 states are staged in LDS as separate real and imaginary planes (the
// row side already multiplied by P_a), and each wave then runs the MFMA chain
// for its 32 x 32 quarter, four 16 x 16 tiles, re and im accumulators each.
// Eight universes per stage keep the kernel within 128 VGPRs, so four waves
// share each SIMD's matrix pipe (16 per stage allowed three).
#include <hip/hip_runtime.h>

#include <cmath>

#include "pk_launch.h"

namespace pk {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kBM = 64;         // block of rho (rows and columns)
constexpr int kKC = 8;          // universes per LDS stage
constexpr int kLd = kBM + 2;    // LDS row length in doubles (padding spreads the rows over banks)
constexpr int kThreads = 256;

// v_mfma_f64_16x16x4f64 lane layout: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register r of lane l is D[4 r + l / 16][l % 16].
__global__ void __launch_bounds__(kThreads, 4) density_kernel(const double2* C, const double* P, double2* rho,
                                                           int64_t N, int A) {
    __shared__ double sAx[kKC][kLd], sAy[kKC][kLd], sBx[kKC][kLd], sBy[kKC][kLd];
    // block (bi, bj) with bi >= bj from the linear index
    const int64_t b = blockIdx.x;
    int64_t bi = (int64_t)((std::sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while (bi * (bi + 1) / 2 > b) --bi;
    while ((bi + 1) * (bi + 2) / 2 <= b) ++bi;
    const int64_t bj = b - bi * (bi + 1) / 2;
    const int64_t I0 = bi * kBM, J0 = bj * kBM;

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;  // the wave's quarter
    const int li = lane & 15, lk = lane >> 4;

    v4d re[2][2], im[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            re[x][y] = v4d{0, 0, 0, 0};
            im[x][y] = v4d{0, 0, 0, 0};
        }

    // The next stage's universes are fetched into registers before this stage's
    // MFMAs, so their HBM/L2 latency overlaps the matrix work; they go to LDS after.
    constexpr int kQ = kKC * kBM / kThreads;  // loads per thread per stage and side
    double2 pr[kQ], pc[kQ];
    double pw[kQ];
    const int c = t & 63;
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const int a = k0 + (t >> 6) + 4 * q;
            pr[q] = double2{0.0, 0.0};
            pc[q] = double2{0.0, 0.0};
            pw[q] = 0.0;
            if (a < A) {
                const double2* row = C + (int64_t)a * N;
                if (I0 + c < N) pr[q] = row[I0 + c];
                if (J0 + c < N) pc[q] = row[J0 + c];
                pw[q] = P[a];
            }
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < A; k0 += kKC) {
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const int kk = (t >> 6) + 4 * q;
            sAx[kk][c] = pw[q] * pr[q].x;
            sAy[kk][c] = pw[q] * pr[q].y;
            sBx[kk][c] = pc[q].x;
            sBy[kk][c] = pc[q].y;
        }
        __syncthreads();
        if (k0 + kKC < A) fetch(k0 + kKC);
#pragma unroll
        for (int k4 = 0; k4 < kKC; k4 += 4) {
            double ax[2], ay[2], bx[2], by[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                ax[x] = sAx[k4 + lk][wr + 16 * x + li];
                ay[x] = sAy[k4 + lk][wr + 16 * x + li];
                bx[x] = sBx[k4 + lk][wc + 16 * x + li];
                by[x] = sBy[k4 + lk][wc + 16 * x + li];
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    re[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[x], bx[y], re[x][y], 0, 0, 0);
                    re[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(ay[x], by[y], re[x][y], 0, 0, 0);
                    im[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(ay[x], bx[y], im[x][y], 0, 0, 0);
                    im[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ax[x], by[y], im[x][y], 0, 0, 0);
                }
        }
        __syncthreads();
    }

    // write back: (row, col) and its mirror (col, row); the strict upper part of a
    // diagonal block comes from the mirror of its lower part
    const bool diag = bi == bj;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = I0 + wr + 16 * x + 4 * r + lk;
                const int64_t col = J0 + wc + 16 * y + li;
                if (row >= N || col >= N) continue;
                if (diag && row < col) continue;
                const double vre = re[x][y][r], vim = im[x][y][r];
                if (row == col) {
                    rho[row * N + col] = double2{vre, 0.0};
                } else {
                    rho[row * N + col] = double2{vre, vim};
                    rho[col * N + row] = double2{vre, -vim};
                }
            }
}

// S = -sum lambda log2 lambda over lambda > 0, and Tr rho^2 = sum lambda^2, from
// the ascending eigenvalues; one workgroup, fixed order.
__global__ void __launch_bounds__(kThreads) spectrum_sums_kernel(const double* lam, int64_t n, double* out) {
    __shared__ double red[2][kThreads / 64];
    double s = 0.0, p = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kThreads) {
        const double v = lam[i];
        if (v > 0.0) s -= v * log2(v);
        p += v * v;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off, 64);
        p += __shfl_xor(p, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s;
        red[1][threadIdx.x >> 6] = p;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ts = 0.0, tp = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) {
            ts += red[0][w];
            tp += red[1][w];
        }
        out[0] = ts;
        out[1] = tp;
    }
}

}  // namespace

int64_t density_blocks(int64_t N) {
    const int64_t nb = (N + kBM - 1) / kBM;
    return nb * (nb + 1) / 2;
}

hipError_t launch_density(const void* C, const double* P, void* rho, int64_t N, int A, hipStream_t st) {
    const int64_t blocks = density_blocks(N);
    hipLaunchKernelGGL(density_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, st,
                       static_cast<const double2*>(C), P, static_cast<double2*>(rho), N, A);
    return hipGetLastError();
}

hipError_t launch_spectrum_sums(const double* lam, int64_t n, double* out, hipStream_t st) {
    hipLaunchKernelGGL(spectrum_sums_kernel, dim3(1), dim3(kThreads), 0, st, lam, n, out);
    return hipGetLastError();
}

}  // namespace pk
