// Device kernels for gfx950: table preparation, the final FP64 combine and the
// pair-index map; and the run-time choice of the pass and batched kernel
// instances (compiled in pk_pass_*.hip).
#include <hip/hip_runtime.h>

#include "pk_kargs.h"

namespace pk {

// D^(1/2): five 2x2 matrices D, D^H, dD/dalpha, dD/dbeta, dD/dgamma with
// D = R_z(alpha) R_y(beta) R_z(gamma) written out element by element.
__device__ void build_d2(double* m, double al, double be, double ga) {
    double c, s, cp, sp, cm, sm;
    sincos(0.5 * be, &s, &c);
    sincos(0.5 * (al + ga), &sp, &cp);  // e^{i(al+ga)/2}
    sincos(0.5 * (al - ga), &sm, &cm);  // e^{i(al-ga)/2}
    // D00 = e^{-i(a+g)/2} c, D01 = -e^{-i(a-g)/2} s, D10 = e^{i(a-g)/2} s, D11 = e^{i(a+g)/2} c
    const double D[8] = {cp * c, -sp * c, -cm * s, sm * s, cm * s, sm * s, cp * c, sp * c};
    for (int e = 0; e < 8; ++e) m[e] = D[e];
    // D^H[a][b] = conj(D[b][a])
    const double H[8] = {D[0], -D[1], D[4], -D[5], D[2], -D[3], D[6], -D[7]};
    for (int e = 0; e < 8; ++e) m[8 + e] = H[e];
    // dD/dalpha = diag(-i/2, i/2) D : row 0 times -i/2, row 1 times i/2
    const double Da[8] = {0.5 * D[1], -0.5 * D[0], 0.5 * D[3], -0.5 * D[2],
                          -0.5 * D[5], 0.5 * D[4], -0.5 * D[7], 0.5 * D[6]};
    for (int e = 0; e < 8; ++e) m[16 + e] = Da[e];
    // dD/dbeta: c -> -s/2 and s -> c/2 in every element
    const double Db[8] = {-0.5 * cp * s, 0.5 * sp * s, -0.5 * cm * c, 0.5 * sm * c,
                          0.5 * cm * c, 0.5 * sm * c, -0.5 * cp * s, -0.5 * sp * s};
    for (int e = 0; e < 8; ++e) m[24 + e] = Db[e];
    // dD/dgamma = D diag(-i/2, i/2) : column 0 times -i/2, column 1 times i/2
    const double Dg[8] = {0.5 * D[1], -0.5 * D[0], -0.5 * D[3], 0.5 * D[2],
                          0.5 * D[5], -0.5 * D[4], -0.5 * D[7], 0.5 * D[6]};
    for (int e = 0; e < 8; ++e) m[32 + e] = Dg[e];
}

// D^(3/2): five 4x4 matrices.  D_{m'm} = e^{-i m' alpha} d_{m'm}(beta) e^{-i m gamma}
// on rows/columns m = 3/2, 1/2, -1/2, -3/2, with the j = 3/2 small-d entries in
// c = cos(beta/2), s = sin(beta/2) and their beta derivatives written out.
__device__ void build_d4(double* m, double al, double be, double ga) {
    double s, c;
    sincos(0.5 * be, &s, &c);
    const double r3 = 1.7320508075688772;  // sqrt(3)
    const double c2 = c * c, s2 = s * s, c3 = c2 * c, s3 = s2 * s;
    const double d[16] = {c3,           -r3 * c2 * s,       r3 * c * s2,        -s3,
                          r3 * c2 * s,  c3 - 2.0 * c * s2,  s3 - 2.0 * c2 * s,  r3 * c * s2,
                          r3 * c * s2,  2.0 * c2 * s - s3,  c3 - 2.0 * c * s2,  -r3 * c2 * s,
                          s3,           r3 * c * s2,        r3 * c2 * s,        c3};
    const double u = r3 * (0.5 * c3 - c * s2);   // d/dbeta of r3 c^2 s
    const double w = r3 * (c2 * s - 0.5 * s3);   // d/dbeta of r3 c s^2
    const double dd[16] = {-1.5 * c2 * s,  -u,                    w,                     -1.5 * c * s2,
                           u,              -3.5 * c2 * s + s3,    3.5 * c * s2 - c3,     w,
                           w,              c3 - 3.5 * c * s2,     -3.5 * c2 * s + s3,    -u,
                           1.5 * c * s2,   w,                     u,                     -1.5 * c2 * s};
    const double mq[4] = {1.5, 0.5, -0.5, -1.5};
    for (int r = 0; r < 4; ++r)
        for (int col = 0; col < 4; ++col) {
            double sn, cs;
            sincos(mq[r] * al + mq[col] * ga, &sn, &cs);  // e^{-i phi} = cs - i sn
            const int e = 2 * (4 * r + col);
            const double Dr = d[4 * r + col] * cs, Di = -d[4 * r + col] * sn;
            m[e] = Dr;
            m[e + 1] = Di;
            // D^H[col][r] = conj(D[r][col])
            m[32 + 2 * (4 * col + r)] = Dr;
            m[32 + 2 * (4 * col + r) + 1] = -Di;
            // dD/dalpha = -i m' D, dD/dgamma = -i m D: (-i k)(x + i y) = k y - i k x
            m[64 + e] = mq[r] * Di;
            m[64 + e + 1] = -mq[r] * Dr;
            m[96 + e] = dd[4 * r + col] * cs;
            m[96 + e + 1] = -dd[4 * r + col] * sn;
            m[128 + e] = mq[col] * Di;
            m[128 + e + 1] = -mq[col] * Dr;
        }
}

// Copies the static operators (2x2 and 4x4) into the workspace, clears the
// launch counters, and builds every rotation's five matrices from its angles.
__global__ void prep_kernel(PrepArgs p) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < p.n_counters) p.counters[t] = 0u;
    if (t < p.n_smats) p.mats[t] = p.smats[t];
    if (t < p.n_smats4) p.mats4[t] = p.smats4[t];
    if (t < p.n_params) {
        const ParamRef r = p.params[t];
        const double al = p.angles[3 * t], be = p.angles[3 * t + 1], ga = p.angles[3 * t + 2];
        if (r.kind == 0)
            build_d2(p.mats + p.n_smats + 40 * r.slot, al, be, ga);
        else
            build_d4(p.mats4 + p.n_smats4 + 160 * r.slot, al, be, ga);
    }
}

// Final FP64 combine, one workgroup per output, fixed summation order.
__global__ void __launch_bounds__(256) reduce_kernel(const Reduction* red, int32_t n, const double* ws,
                                                     double* L_out, double* norm_out, double* grad_out) {
    __shared__ double sred[16];
    const int e = blockIdx.x;
    if (e >= n) return;
    const Reduction r = red[e];
    double* out = r.target == 0 ? L_out : (r.target == 1 ? norm_out : grad_out);
    if (!out) return;
    // thread t adds partials t, t + 256, ... in that order; eight loads are issued
    // before their adds so that their latencies overlap (same order, same result)
    constexpr int kBatch = 8;
    double s = 0.0;
    for (int64_t t0 = threadIdx.x; t0 < r.count; t0 += 256 * kBatch) {
        double v[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            const int64_t t = t0 + 256 * j;
            v[j] = t < r.count ? ws[r.src + t] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kBatch; ++j)
            if (t0 + 256 * j < r.count) s += v[j];
    }
    const double tot = block_sum<256>(s, sred);
    if (threadIdx.x == 0) out[r.index] = tot;
}

// Partner pairs of qubit i_s (Eqs. pair0 / pair1): the r-th label with bit
// (nq - i_s) clear is r with a zero bit inserted at that position.
__global__ void pair_index_kernel(int32_t nq, int32_t i_s, int64_t first, int64_t count, int64_t* n0,
                                  int64_t* n1) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count) return;
    const int b = nq - i_s;
    const int64_t q = first + r;
    const int64_t lo = q & (((int64_t)1 << b) - 1);
    const int64_t m0 = ((q >> b) << (b + 1)) | lo;
    n0[r] = m0;
    n1[r] = m0 + ((int64_t)1 << b);
}

// ---------------------------------------------------------------------------- host launchers

static KArgs kargs(const PassLaunch& L) {
    KArgs a;
    a.passes = L.passes;
    a.stages = L.stages;
    a.flips = L.flips;
    a.phases = L.phases;
    a.twid = L.twid;
    a.urefs = L.urefs;
    a.mats = L.mats;
    a.mats4 = L.mats4;
    a.src0 = L.src0;
    a.dst0 = L.dst0;
    a.dst1 = L.dst1;
    a.partials = L.partials;
    a.reads = L.reads;
    a.gpart = L.gpart;
    a.dL = L.dL;
    a.pass = L.pass;
    a.want_norm = L.want_norm;
    return a;
}

hipError_t launch_pass(const PassLaunch& L, hipStream_t st) {
    const KArgs a = kargs(L);
    if (L.nv == 2) {
        if (L.rbits != 4) return hipErrorInvalidValue;
        return L.fp64 ? launch_pass_r<double, 2, 4>(L.kmax, a, L.ntiles, L.grid_cap, st)
                      : launch_pass_r<float, 2, 4>(L.kmax, a, L.ntiles, L.grid_cap, st);
    }
    if (L.rbits == 5)
        return L.fp64 ? launch_pass_r<double, 1, 5>(L.kmax, a, L.ntiles, L.grid_cap, st)
                      : launch_pass_r<float, 1, 5>(L.kmax, a, L.ntiles, L.grid_cap, st);
    if (L.rbits == 3)
        return L.fp64 ? launch_pass_r<double, 1, 3>(L.kmax, a, L.ntiles, L.grid_cap, st)
                      : launch_pass_r<float, 1, 3>(L.kmax, a, L.ntiles, L.grid_cap, st);
    return L.fp64 ? launch_pass_r<double, 1, 4>(L.kmax, a, L.ntiles, L.grid_cap, st)
                  : launch_pass_r<float, 1, 4>(L.kmax, a, L.ntiles, L.grid_cap, st);
}

hipError_t launch_batched(const PassLaunch& L, const BatchArgs& B, unsigned grid, hipStream_t st) {
    KArgs a = kargs(L);
    a.dst1 = nullptr;
    a.gpart = nullptr;
    a.dL = nullptr;
    a.pass = 0;
    if (L.rbits == 5)
        return L.fp64 ? launch_batched_r<double, 5>(L.kmax, a, B, grid, st)
                      : launch_batched_r<float, 5>(L.kmax, a, B, grid, st);
    return L.fp64 ? launch_batched_r<double, 4>(L.kmax, a, B, grid, st)
                  : launch_batched_r<float, 4>(L.kmax, a, B, grid, st);
}

hipError_t launch_repeat(const PassLaunch& L, const RepeatArgs& r, unsigned grid, hipStream_t st) {
    KArgs a = kargs(L);
    a.dst1 = nullptr;
    a.gpart = nullptr;
    a.dL = nullptr;
    a.pass = 0;
    if (L.rbits == 5)
        return L.fp64 ? launch_repeat_r<double, 5>(L.kmax, a, r, grid, st)
                      : launch_repeat_r<float, 5>(L.kmax, a, r, grid, st);
    return L.fp64 ? launch_repeat_r<double, 4>(L.kmax, a, r, grid, st)
                  : launch_repeat_r<float, 4>(L.kmax, a, r, grid, st);
}

int repeat_blocks_per_cu(int kmax, int rbits, bool fp64) {
    if (rbits == 5) return fp64 ? repeat_occupancy_r<double, 5>(kmax) : repeat_occupancy_r<float, 5>(kmax);
    return fp64 ? repeat_occupancy_r<double, 4>(kmax) : repeat_occupancy_r<float, 4>(kmax);
}

int batched_blocks_per_cu(int kmax, int rbits, bool fp64) {
    if (rbits == 5) return fp64 ? batched_occupancy_r<double, 5>(kmax) : batched_occupancy_r<float, 5>(kmax);
    return fp64 ? batched_occupancy_r<double, 4>(kmax) : batched_occupancy_r<float, 4>(kmax);
}

hipError_t launch_prep(const PrepArgs& p, hipStream_t st) {
    int n = p.n_smats;
    if (p.n_smats4 > n) n = p.n_smats4;
    if (p.n_params > n) n = p.n_params;
    if (p.n_counters > n) n = p.n_counters;
    if (n < 1) n = 1;
    hipLaunchKernelGGL(prep_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_reduce(const Reduction* red, int n, const double* ws, double* L_out, double* norm_out,
                         double* grad_out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_kernel, dim3(n), dim3(256), 0, st, red, n, ws, L_out, norm_out, grad_out);
    return hipGetLastError();
}

hipError_t launch_pairs(int nq, int i_s, int64_t first, int64_t count, int64_t* n0, int64_t* n1,
                        hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(pair_index_kernel, dim3((unsigned)blocks), dim3(256), 0, st, nq, i_s, first, count, n0,
                       n1);
    return hipGetLastError();
}

}  // namespace pk
