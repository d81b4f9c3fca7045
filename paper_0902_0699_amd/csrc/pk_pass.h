// The fused tile pass and the batched multiverse launch (gfx950): device code
// and the templated launchers that the pk_pass_*.hip units instantiate.
//
// One workgroup owns one tile of 2^k amplitudes (labels that differ only in the
// pass's k tile bits).  Thread t holds 16 amplitudes in registers; in stage s
// their local labels are jt(s) | roff_s(i), i = 0..15, where register bit a of
// i sits on local tile bit rb[a] and the thread index fills the other bits in
// ascending order.  A one-qubit gate on a register bit is then a butterfly over
// register pairs (i, i | 2^a): the 2x2 pair update of Sec. 3 (Eq. resmat1) on
// every partner pair of the tile at once.  Between stages the tile goes through
// LDS to bring the next four bits into registers.  The first and last stages
// keep the lowest tile bits on the lane index, so HBM is read and written in
// contiguous runs.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "pk_kargs.h"

// Descriptor tables are read through the constant address space so that the
// uniform reads become scalar loads: they then never wait on vector memory
// traffic (the prefetched tile, the previous tile's stores).
#define PK_CONST __attribute__((address_space(4)))

namespace pk {

template <typename R>
struct Cplx;
template <>
struct Cplx<double> {
    using T = double2;
};
template <>
struct Cplx<float> {
    using T = float2;
};


template <typename X>
__device__ __forceinline__ const PK_CONST X* cptr(const X* p) {
    return (const PK_CONST X*)(p);
}

// LDS bank swizzle on element slots: the label's higher W-bit groups are XORed
// into its low W bits, with 2^W elements = 256 bytes, one pass over the LDS
// banks.  Whatever bits a stage puts on the lane index, any 256 contiguous
// bytes' worth of lanes then hit distinct banks.  Linear over XOR, so
// phys(a ^ b) = phys(a) ^ phys(b).
template <int ESZ>
__device__ __forceinline__ unsigned phys(unsigned j) {
    constexpr int W = ESZ == 16 ? 4 : 5;
    constexpr unsigned M = (1u << W) - 1u;
    return j ^ (((j >> W) ^ (j >> (2 * W)) ^ (j >> (3 * W))) & M);
}

// Layout of one stage: per-thread label base and the uniform offsets of the
// four register bits (as labels and as LDS slots).
struct Layout {
    unsigned jt;               // thread's label base
    unsigned pj;               // phys(jt)
    unsigned r[kMaxRegBits];   // 1 << rb[a] (0 for missing bits)
    unsigned p[kMaxRegBits];   // phys(1 << rb[a])
};

template <int ESZ>
__device__ __forceinline__ Layout make_layout(const PK_CONST Stage* S, int nrb, unsigned tid) {
    Layout L;
    unsigned t = tid;
    if (S->nlanes == 0) {
        // spread the thread index over the local bits that are not register bits
        for (int q = 0; q < nrb; ++q) {
            const int p = S->rbs[q];
            t = ((t >> p) << (p + 1)) | (t & ((1u << p) - 1u));
        }
    } else {
        // the low W thread bits to the chosen local bits, one per swizzle group bit,
        // the others in order to the remaining free bits (the masks are uniform)
        constexpr int W = ESZ == 16 ? 4 : 5;
        const unsigned lanes = S->lanes;
        t = 0u;
#pragma unroll
        for (int i = 0; i < W; ++i) t |= ((tid >> i) & 1u) << ((lanes >> (4 * i)) & 15u);
        unsigned rest = S->lanes_rest, x = tid >> W;
        while (rest != 0u) {
            const unsigned low = rest & (0u - rest);
            if (x & 1u) t |= low;
            x >>= 1;
            rest ^= low;
        }
    }
    L.jt = t;
    L.pj = phys<ESZ>(t);
#pragma unroll
    for (int a = 0; a < kMaxRegBits; ++a) {
        L.r[a] = a < nrb ? (1u << S->rb[a]) : 0u;
        L.p[a] = phys<ESZ>(L.r[a]);
    }
    return L;
}

__device__ __forceinline__ unsigned roff(const Layout& L, int i) {
    return ((i & 1) ? L.r[0] : 0u) | ((i & 2) ? L.r[1] : 0u) | ((i & 4) ? L.r[2] : 0u) |
           ((i & 8) ? L.r[3] : 0u) | ((i & 16) ? L.r[4] : 0u);
}
__device__ __forceinline__ unsigned poff(const Layout& L, int i) {
    return ((i & 1) ? L.p[0] : 0u) ^ ((i & 2) ? L.p[1] : 0u) ^ ((i & 4) ? L.p[2] : 0u) ^
           ((i & 8) ? L.p[3] : 0u) ^ ((i & 16) ? L.p[4] : 0u);
}

// Moves the bits of `x` along the runs (src, len, dst).
__device__ __forceinline__ int64_t deposit(int64_t x, const PK_CONST Run* run, int nrun) {
    int64_t r = 0;
    for (int q = 0; q < nrun; ++q) {
        const int src = run[q].src, len = run[q].len, dst = run[q].dst;
        r |= ((x >> src) & (((int64_t)1 << len) - 1)) << dst;
    }
    return r;
}

// State offsets of a stage used for HBM access: the thread's part (elements)
// and the uniform parts of the four register bits.
struct GOff {
    int64_t gt;
    int64_t g[kMaxRegBits];
};

// `store` selects the map the tile is written with (SWAPs done by relabelling
// make it differ from the map it is read with).
__device__ __forceinline__ GOff make_goff(const PK_CONST Pass* P, const PK_CONST Stage* S, const Layout& L,
                                          int nrb, bool store) {
    GOff G;
    G.gt = store ? deposit((int64_t)L.jt, P->strun, P->nstrun) : deposit((int64_t)L.jt, P->trun, P->ntrun);
    const PK_CONST int32_t* pos = store ? P->stpos : P->tpos;
#pragma unroll
    for (int a = 0; a < kMaxRegBits; ++a) G.g[a] = a < nrb ? ((int64_t)1 << pos[S->rb[a]]) : 0;
    return G;
}

__device__ __forceinline__ int64_t goff(const GOff& G, int i) {
    return ((i & 1) ? G.g[0] : 0) + ((i & 2) ? G.g[1] : 0) + ((i & 4) ? G.g[2] : 0) +
           ((i & 8) ? G.g[3] : 0) + ((i & 16) ? G.g[4] : 0);
}

// ---------------------------------------------------------------------------- gate bodies

// Hadamard butterfly (x, y) <- (x + y, x - y), unnormalised, written to update
// both registers in place: x += y, then y = x_new - 2 y (one rounding more than
// x - y, well inside the FP64 and FP32 tolerances).  In-place updates let the
// compiler keep the tile in one set of registers through the predicated steps.
template <int A, int NV, int NR, typename T>
__device__ __forceinline__ void op_h(T (&v)[NV][NR]) {
    using R = decltype(v[0][0].x);
#pragma unroll
    for (int n = 0; n < NV; ++n)
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (i & (1 << A)) continue;
            const int j = i | (1 << A);
            v[n][i].x += v[n][j].x;
            v[n][i].y += v[n][j].y;
            v[n][j].x = fma((R)-2, v[n][j].x, v[n][i].x);
            v[n][j].y = fma((R)-2, v[n][j].y, v[n][i].y);
        }
}

// (x, y) <- M (x, y) with M row-major complex [m0+i m1, m2+i m3; m4+i m5, m6+i m7]
template <typename T, typename R>
__device__ __forceinline__ void pair_mat(T& x, T& y, const R (&m)[8]) {
    const T a = x, b = y;
    x.x = m[0] * a.x - m[1] * a.y + m[2] * b.x - m[3] * b.y;
    x.y = m[0] * a.y + m[1] * a.x + m[2] * b.y + m[3] * b.x;
    y.x = m[4] * a.x - m[5] * a.y + m[6] * b.x - m[7] * b.y;
    y.y = m[4] * a.y + m[5] * a.x + m[6] * b.y + m[7] * b.x;
}

template <int A, int NV, int NR, typename T, typename R>
__device__ __forceinline__ void op_m(T (&v)[NV][NR], const R (&m)[8]) {
#pragma unroll
    for (int n = 0; n < NV; ++n)
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (i & (1 << A)) continue;
            pair_mat(v[n][i], v[n][i | (1 << A)], m);
        }
}

// Backward step through a D2 gate: psi <- D^H psi; then for every angle,
// g += Re( conj(lambda) . (dD/dtheta) psi ); then lambda <- D^H lambda.
// One derivative matrix at a time keeps the register footprint small.
template <int A, int NV, int NR, typename T, typename R>
__device__ __forceinline__ void op_d2bwd(T (&v)[NV][NR], const R (&mh)[8], const PK_CONST double* dmats,
                                         double (&g)[3]) {
    if constexpr (NV == 2) {
#pragma unroll
        for (int i = 0; i < NR; ++i)
            if (!(i & (1 << A))) pair_mat(v[0][i], v[0][i | (1 << A)], mh);
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            double m[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) m[e] = dmats[8 * t + e];
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                if (i & (1 << A)) continue;
                const int j = i | (1 << A);
                const double p0x = v[0][i].x, p0y = v[0][i].y, p1x = v[0][j].x, p1y = v[0][j].y;
                const double t0x = m[0] * p0x - m[1] * p0y + m[2] * p1x - m[3] * p1y;
                const double t0y = m[0] * p0y + m[1] * p0x + m[2] * p1y + m[3] * p1x;
                const double t1x = m[4] * p0x - m[5] * p0y + m[6] * p1x - m[7] * p1y;
                const double t1y = m[4] * p0y + m[5] * p0x + m[6] * p1y + m[7] * p1x;
                acc += (double)v[1][i].x * t0x + (double)v[1][i].y * t0y + (double)v[1][j].x * t1x +
                       (double)v[1][j].y * t1y;
            }
            g[t] += acc;
        }
#pragma unroll
        for (int i = 0; i < NR; ++i)
            if (!(i & (1 << A))) pair_mat(v[1][i], v[1][i | (1 << A)], mh);
    }
}

// A two-qubit gate on register bits 0 (qubit is1) and 1 (qubit is2): the
// registers i, i+2, i+1, i+3 (i = 0 mod 4) hold the amplitude quartet
// |q_is1 q_is2> = |00>, |01>, |10>, |11> of one n_00 (Eqs. twoopB, resmat2) and
// are replaced by M times it.  M is row-major complex (32 doubles), read row by
// row through scalar loads.
template <typename T>
__device__ __forceinline__ void quartet_mat(T& x0, T& x1, T& x2, T& x3, const PK_CONST double* m) {
    using R = decltype(x0.x);
    const T in[4] = {x0, x1, x2, x3};
    T out[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        R re = 0, im = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const R mr = (R)m[2 * (4 * r + c)], mi = (R)m[2 * (4 * r + c) + 1];
            re += mr * in[c].x - mi * in[c].y;
            im += mr * in[c].y + mi * in[c].x;
        }
        out[r].x = re;
        out[r].y = im;
    }
    x0 = out[0];
    x1 = out[1];
    x2 = out[2];
    x3 = out[3];
}

template <int NV, int NR, typename T>
__device__ __forceinline__ void op_mat4(T (&v)[NV][NR], const PK_CONST double* m) {
#pragma unroll
    for (int n = 0; n < NV; ++n)
#pragma unroll
        for (int i = 0; i < NR; i += 4) quartet_mat(v[n][i], v[n][i + 2], v[n][i + 1], v[n][i + 3], m);
}

// The same on register bits 2 (qubit is1) and 3 (qubit is2): a second qubit pair,
// disjoint from the first, in the same stage.  Registers i, i+8, i+4, i+12 (bits
// 2 and 3 of i clear) hold its quartet |00>, |01>, |10>, |11>.
template <int NV, int NR, typename T>
__device__ __forceinline__ void op_mat4_hi(T (&v)[NV][NR], const PK_CONST double* m) {
#pragma unroll
    for (int n = 0; n < NV; ++n)
#pragma unroll
        for (int i = 0; i < NR; ++i)
            if ((i & 12) == 0) quartet_mat(v[n][i], v[n][i + 8], v[n][i + 4], v[n][i + 12], m);
}

// Backward step through a D4 gate, as op_d2bwd with 4x4 matrices: psi <- D^H psi;
// for every angle g += Re( conj(lambda) . (dD/dtheta) psi ); lambda <- D^H lambda.
// `m` holds D, D^H, dD/dalpha, dD/dbeta, dD/dgamma (32 doubles each).
template <int NV, int NR, typename T>
__device__ __forceinline__ void op_d4bwd(T (&v)[NV][NR], const PK_CONST double* m, double (&g)[3]) {
    if constexpr (NV == 2) {
#pragma unroll
        for (int i = 0; i < NR; i += 4) quartet_mat(v[0][i], v[0][i + 2], v[0][i + 1], v[0][i + 3], m + 32);
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const PK_CONST double* dm = m + 64 + 32 * t;
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < NR; i += 4) {
                const int idx[4] = {i, i + 2, i + 1, i + 3};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double re = 0.0, im = 0.0;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const double mr = dm[2 * (4 * r + c)], mi = dm[2 * (4 * r + c) + 1];
                        const double px = v[0][idx[c]].x, py = v[0][idx[c]].y;
                        re += mr * px - mi * py;
                        im += mr * py + mi * px;
                    }
                    acc += (double)v[1][idx[r]].x * re + (double)v[1][idx[r]].y * im;
                }
            }
            g[t] += acc;
        }
#pragma unroll
        for (int i = 0; i < NR; i += 4) quartet_mat(v[1][i], v[1][i + 2], v[1][i + 1], v[1][i + 3], m + 32);
    }
}

// The controlled phases of one sub-stage (CPHASE, CPHASEK; Eq. cphasek).  For
// each accumulator slot, the factors of its phases are multiplied together,
// each switched to 1 unless the tile index and the thread's part of the label
// have the phase's other bits set; every register whose index holds the slot's
// register bits then takes the product once.  The loop over a slot's phases is
// branch-free: a phase's factor is (1 + on (c - 1), on s) with on = 0 or 1, a
// product the compiler cannot turn into a select (which it would lower to a
// branch around a late scalar load of c), so every table read is unconditional
// and the loads of several phases are in flight together.  Two independent
// product chains halve the dependent multiply latency.
//
// A slot's product multiplies the registers whose index holds the slot's register
// bits.  The mask is uniform but not known at compile time, so each register's
// test is a scalar branch around its multiply.  The empty volatile statement in
// the branch keeps the compiler from speculating the multiply into a product for
// every register followed by a select, and because each branch updates one
// register in place, no other register is copied where the paths join.
template <int NV, int NR, typename T, typename R>
__device__ __forceinline__ void apply_slot(T (&v)[NV][NR], int pm, R c, R s) {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        if ((i & pm) != pm) continue;
        __asm__ volatile("");
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            const R x = v[m][i].x, y = v[m][i].y;
            v[m][i].x = x * c - y * s;
            v[m][i].y = x * s + y * c;
        }
    }
}

// Bits of x at the positions set in m, packed (bit k of the result is the k-th
// set bit of m, counted from the least significant).
__device__ __forceinline__ unsigned extract_bits(uint64_t x, uint64_t m) {
    unsigned r = 0;
    for (int k = 0; m; ++k) {
        const int b = __builtin_ctzll(m);
        r |= (unsigned)((x >> b) & 1u) << k;
        m &= m - 1;
    }
    return r;
}

// A tile's entries of the pass's tile-part product tables: lane r of every wave
// holds the entry of table r (entry 0, the factor 1, where the pass has no table r).
template <typename R>
struct TileRefs {
    R c, s;
};

template <typename R>
__device__ __forceinline__ TileRefs<R> load_refs(const KArgs& a, const PK_CONST Pass* P, int64_t tile) {
    const int lane = (int)(threadIdx.x & 63u);
    int e = 0;
    if (lane < P->nuref) {
        const URef r = a.urefs[P->uref_begin + lane];
        e = r.base + (int)extract_bits((uint64_t)tile, (uint64_t)r.mask);
    }
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 x = *reinterpret_cast<const d2*>(a.twid + 2 * e);
    return {(R)x.x, (R)x.y};
}

__device__ __forceinline__ float lane_value(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

__device__ __forceinline__ double lane_value(double x, int l) {
    const long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The leading phase_ucnt[u] phases of a slot are in its product tables: the
// tile part is one or two of the tile's entries held by the lanes (U), the thread
// part one entry indexed by the thread's label bits.  The remaining phases
// multiply in one factor each.
// The lanes are read with every lane of the wave active (a lane that is inactive
// at a cross-lane read need not hold its value there); only the rest of the step
// runs under `active`.
template <int NV, int NR, typename T, typename R>
__device__ __forceinline__ void apply_phases(const KArgs& a, const PK_CONST Stage* S, T (&v)[NV][NR],
                                             const Layout& L, int64_t tile, const TileRefs<R>& U, bool active) {
    const PK_CONST PhaseOp* ph = cptr(a.phases) + S->phase_first;
    // the sub-stage's slot table in 16-byte loads issued together (reading the
    // fields where they are used costs one scalar round trip per field and slot)
    typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
    const i32x4 pms = *reinterpret_cast<const PK_CONST i32x4*>(S->phase_pm);
    const i32x4 cnts = *reinterpret_cast<const PK_CONST i32x4*>(S->phase_cnt);
    const i32x4 ucnts = *reinterpret_cast<const PK_CONST i32x4*>(S->phase_ucnt);
    const i32x4 tts = *reinterpret_cast<const PK_CONST i32x4*>(S->phase_tt);
    const i32x4 ut0s = *reinterpret_cast<const PK_CONST i32x4*>(S->phase_ut0);
    const i32x4 ut1s = *reinterpret_cast<const PK_CONST i32x4*>(S->phase_ut1);
    const i32x4 ttms = *reinterpret_cast<const PK_CONST i32x4*>(S->phase_ttm);
#pragma unroll
    for (int u = 0; u < kPhaseSlots; ++u) {
        const int cnt = cnts[u];
        if (cnt == 0) continue;
        R c0 = 1, s0 = 0, c1 = 1, s1 = 0;
        if (ut0s[u] >= 0) {
            c0 = lane_value(U.c, ut0s[u]);
            s0 = lane_value(U.s, ut0s[u]);
            if (ut1s[u] >= 0) {
                const R cf = lane_value(U.c, ut1s[u]), sf = lane_value(U.s, ut1s[u]);
                const R x = c0, y = s0;
                c0 = x * cf - y * sf;
                s0 = x * sf + y * cf;
            }
        }
        const PK_CONST PhaseOp* ps = ph;
        ph += cnt;
        if (!active) continue;
        if (tts[u] >= 0) {
            const unsigned ix = extract_bits((uint64_t)L.jt, (uint64_t)(unsigned)ttms[u]);
            const double* e = a.twid + 2 * (tts[u] + (int)ix);
            c1 = (R)e[0];
            s1 = (R)e[1];
        }
        int q = ucnts[u];
#pragma unroll 2
        for (; q + 1 < cnt; q += 2) {
            const int64_t fa = ps[q].fmask, fb = ps[q + 1].fmask;
            const unsigned ta = ps[q].tmask, tb = ps[q + 1].tmask;
            const R oa = (R)(((tile & fa) == fa) & ((L.jt & ta) == ta));
            const R ob = (R)(((tile & fb) == fb) & ((L.jt & tb) == tb));
            const R ca = fma(oa, (R)ps[q].cm1, (R)1), sa = oa * (R)ps[q].s;
            const R cb = fma(ob, (R)ps[q + 1].cm1, (R)1), sb = ob * (R)ps[q + 1].s;
            R x = c0, y = s0;
            c0 = x * ca - y * sa;
            s0 = x * sa + y * ca;
            x = c1;
            y = s1;
            c1 = x * cb - y * sb;
            s1 = x * sb + y * cb;
        }
        if (q < cnt) {
            const int64_t fa = ps[q].fmask;
            const unsigned ta = ps[q].tmask;
            const R oa = (R)(((tile & fa) == fa) & ((L.jt & ta) == ta));
            const R ca = fma(oa, (R)ps[q].cm1, (R)1), sa = oa * (R)ps[q].s;
            const R x = c0, y = s0;
            c0 = x * ca - y * sa;
            s0 = x * sa + y * ca;
        }
        const R c = c0 * c1 - s0 * s1, s = c0 * s1 + s0 * c1;
        apply_slot<NV, NR>(v, pms[u], c, s);
    }
}

// Hadamards on the register bits set in `mask` (distinct bits commute).
template <int NV, int NR, typename T>
__device__ __forceinline__ void apply_hmask(T (&v)[NV][NR], int mask) {
    if (mask & 1) op_h<0, NV, NR>(v);
    if (mask & 2) op_h<1, NV, NR>(v);
    if (mask & 4) op_h<2, NV, NR>(v);
    if constexpr (NR > 8)
        if (mask & 8) op_h<3, NV, NR>(v);
    if constexpr (NR > 16)
        if (mask & 16) op_h<4, NV, NR>(v);
}

template <int NV, int NR, typename T, typename R>
__device__ __forceinline__ void apply_mat(T (&v)[NV][NR], int a, const R (&m)[8]) {
    if (a == 0) op_m<0, NV, NR>(v, m);
    if (a == 1) op_m<1, NV, NR>(v, m);
    if (a == 2) op_m<2, NV, NR>(v, m);
    if constexpr (NR > 8)
        if (a == 3) op_m<3, NV, NR>(v, m);
    if constexpr (NR > 16)
        if (a == 4) op_m<4, NV, NR>(v, m);
}

template <int NV, int NR, typename T, typename R>
__device__ __forceinline__ void apply_d2bwd(T (&v)[NV][NR], int a, const R (&mh)[8], const PK_CONST double* dmats,
                                            double (&g)[3]) {
    if (a == 0) op_d2bwd<0, NV, NR>(v, mh, dmats, g);
    if (a == 1) op_d2bwd<1, NV, NR>(v, mh, dmats, g);
    if (a == 2) op_d2bwd<2, NV, NR>(v, mh, dmats, g);
    if constexpr (NR > 8)
        if (a == 3) op_d2bwd<3, NV, NR>(v, mh, dmats, g);
    if constexpr (NR > 16)
        if (a == 4) op_d2bwd<4, NV, NR>(v, mh, dmats, g);
}

// ---------------------------------------------------------------------------- one tile

// Per-pass constants of a workgroup: they do not depend on the tile.
struct PassCtx {
    int nrb, nreg, flags, nstages;
    bool active;
    Layout L0, Ll;  // first (load) and last (store) stage layouts
    GOff G0, Gl;
};

template <int ESZ, int RB>
__device__ __forceinline__ PassCtx make_ctx(const KArgs& a, const PK_CONST Pass* P) {
    PassCtx C;
    const int k = P->k;
    C.nrb = k < RB ? k : RB;
    C.nreg = 1 << C.nrb;
    C.flags = P->flags;
    C.nstages = P->nstages;
    const unsigned nact = k >= RB ? (1u << (k - RB)) : 1u;
    C.active = threadIdx.x < nact;
    const PK_CONST Stage* S0 = cptr(a.stages) + P->stage_begin;
    const PK_CONST Stage* Sl = S0 + (C.nstages - 1);
    C.L0 = make_layout<ESZ>(S0, C.nrb, threadIdx.x);
    C.Ll = make_layout<ESZ>(Sl, C.nrb, threadIdx.x);
    C.G0 = make_goff(P, S0, C.L0, C.nrb, false);
    C.Gl = make_goff(P, Sl, C.Ll, C.nrb, true);
    return C;
}

// Nontemporal (streaming) 16- or 8-byte accesses of one complex amplitude.
template <typename T>
__device__ __forceinline__ void store_stream(T* p, const T& v) {
    using R = decltype(v.x);
    typedef R V __attribute__((ext_vector_type(2)));
    V w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<V*>(p));
}

template <typename T>
__device__ __forceinline__ T load_stream(const T* p) {
    using R = decltype(p->x);
    typedef R V __attribute__((ext_vector_type(2)));
    const V w = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
    T r;
    r.x = w.x;
    r.y = w.y;
    return r;
}

// HBM -> registers in the first stage's layout.  `base` is the tile's first
// state label.  The uniform part (tile base + register offset) and the thread's
// part stay apart, so each load is a 64-bit scalar base plus a 32-bit lane
// offset; a wide pass (lane offsets beyond 32 bits) adds in 64 bits.  NT: the
// one-vector loads are nontemporal.
template <typename R, int NV, int NR, bool NT = false>
__device__ __forceinline__ void load_tile(const KArgs& a, const PassCtx& C, int64_t base,
                                          typename Cplx<R>::T (&v)[NV][NR]) {
    using T = typename Cplx<R>::T;
    if (C.nreg < NR || NV == 2) {
#pragma unroll
        for (int n = 0; n < NV; ++n)
#pragma unroll
            for (int i = 0; i < NR; ++i) v[n][i] = T{0, 0};
    }
    if (!C.active) return;
    const char* in0 = reinterpret_cast<const char*>((C.flags & PASS_FIRST) ? a.src0 : a.dst0);
    const char* in1 = reinterpret_cast<const char*>(a.dst1);
    const bool read1 = NV == 2 && !(C.flags & PASS_SEED_V1);
    if (!(C.flags & PASS_WIDE)) {
        const uint32_t lane = (uint32_t)C.G0.gt * (uint32_t)sizeof(T);
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (i >= C.nreg) continue;
            const int64_t u = (base + goff(C.G0, i)) * (int64_t)sizeof(T);
            if constexpr (NT)
                v[0][i] = load_stream(reinterpret_cast<const T*>(in0 + u + lane));
            else
                v[0][i] = *reinterpret_cast<const T*>(in0 + u + lane);
            if constexpr (NV == 2)
                if (read1) v[1][i] = *reinterpret_cast<const T*>(in1 + u + lane);
        }
    } else {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (i >= C.nreg) continue;
            const int64_t e = base + C.G0.gt + goff(C.G0, i);
            v[0][i] = reinterpret_cast<const T*>(in0)[e];
            if constexpr (NV == 2)
                if (read1) v[1][i] = reinterpret_cast<const T*>(in1)[e];
        }
    }
}

// Registers -> HBM in the last stage's layout (NT: nontemporal one-vector stores).
template <typename R, int NV, int NR, bool NT = false>
__device__ __forceinline__ void store_tile(const KArgs& a, const PassCtx& C, int64_t base,
                                           const typename Cplx<R>::T (&v)[NV][NR]) {
    using T = typename Cplx<R>::T;
    if (!C.active) return;
    char* out0 = reinterpret_cast<char*>(a.dst0);
    char* out1 = reinterpret_cast<char*>(a.dst1);
    const bool write0 = !(C.flags & PASS_SKIP_V0);
    if (!(C.flags & PASS_WIDE)) {
        const uint32_t lane = (uint32_t)C.Gl.gt * (uint32_t)sizeof(T);
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (i >= C.nreg) continue;
            const int64_t u = (base + goff(C.Gl, i)) * (int64_t)sizeof(T);
            if constexpr (NT) {
                if (write0) store_stream(reinterpret_cast<T*>(out0 + u + lane), v[0][i]);
            } else {
                if (write0) *reinterpret_cast<T*>(out0 + u + lane) = v[0][i];
            }
            if constexpr (NV == 2) *reinterpret_cast<T*>(out1 + u + lane) = v[1][i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (i >= C.nreg) continue;
            const int64_t e = base + C.Gl.gt + goff(C.Gl, i);
            if (write0) reinterpret_cast<T*>(out0)[e] = v[0][i];
            if constexpr (NV == 2) reinterpret_cast<T*>(out1)[e] = v[1][i];
        }
    }
}

// One-amplitude steps on the element flips[f] when it lies in this tile and
// thread: KIND 0 negates it (Oracle, Inv's C_0), 1 stores |C|^2 to its readout
// slot, 2 seeds lambda = dL * psi there.  Written as selects, so the register
// tile is updated in place.
template <int NV, int NR, int KIND, typename T>
__device__ __forceinline__ void element_op(const KArgs& a, T (&v)[NV][NR], const Layout& L, int f, int64_t tile,
                                           int nreg, bool active) {
    const PK_CONST Flip* fl = cptr(a.flips) + f;
    if (fl->tile != tile || !active) return;
    const unsigned jrel = (unsigned)fl->j ^ L.jt;
    unsigned rmask = 0;
#pragma unroll
    for (int q = 0; q < kMaxRegBits; ++q) rmask |= L.r[q];
    if ((jrel & ~rmask) != 0u) return;
    const int slot = fl->slot;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        if (i >= nreg) continue;
        const bool hit = roff(L, i) == jrel;
        if constexpr (KIND == 0) {
#pragma unroll
            for (int n = 0; n < NV; ++n) {
                v[n][i].x = hit ? -v[n][i].x : v[n][i].x;
                v[n][i].y = hit ? -v[n][i].y : v[n][i].y;
            }
        } else if constexpr (KIND == 1) {
            if (hit) {
                const double x = v[0][i].x, y = v[0][i].y;
                a.reads[slot] = x * x + y * y;
            }
        } else if constexpr (NV == 2) {
            const auto d = (decltype(v[0][0].x))a.dL[slot];
            v[1][i].x = hit ? d * v[0][i].x : v[1][i].x;
            v[1][i].y = hit ? d * v[0][i].y : v[1][i].y;
        }
    }
}

// Every stage of the pass on one tile held in registers, then the norm partial.
template <typename R, int NV, int KMAX, int RB>
__device__ __forceinline__ void compute_tile(const KArgs& a, const PK_CONST Pass* P, const PassCtx& C,
                                             int64_t tile, typename Cplx<R>::T (&v)[NV][1 << RB],
                                             const TileRefs<R>& U, typename Cplx<R>::T* lds, double* red) {
    constexpr int NT = 1 << (KMAX - RB);
    constexpr int NR = 1 << RB;
    const unsigned tid = threadIdx.x;
    const bool active = C.active;
    const int nreg = C.nreg;
    const PK_CONST Stage* S = cptr(a.stages) + P->stage_begin;
    Layout L = C.L0;
    for (int s = 0; s < C.nstages; ++s, ++S) {
        // one scalar word says which steps follow; only their parameters are loaded
        const int steps = S->steps;
        // the one-qubit steps' parameters (mat_pre_a .. mat_post) in two 16-byte loads
        // issued with the step word, not one scalar round trip per step
        typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
        const i32x4 sp0 = *reinterpret_cast<const PK_CONST i32x4*>(&S->mat_pre_a);
        const i32x4 sp1 = *reinterpret_cast<const PK_CONST i32x4*>(&S->hmask2);
        const int mat_pre_a = sp0.x, mat_pre = sp0.y, hmask1 = sp0.z, flip_mid = sp0.w;
        const int hmask2 = sp1.x, mat_post_a = sp1.y, mat_post = sp1.z;
        if (s > 0 && (steps & ST_EXCHANGE)) {
            // ---- LDS exchange: previous layout out, this layout in
            const Layout Ln = (s == C.nstages - 1) ? C.Ll : make_layout<(int)sizeof(R) * 2>(S, C.nrb, tid);
#pragma unroll
            for (int n = 0; n < NV; ++n) {
                if (active) {
#pragma unroll
                    for (int i = 0; i < NR; ++i)
                        if (i < nreg) lds[L.pj ^ poff(L, i)] = v[n][i];
                }
                __syncthreads();
                if (active) {
#pragma unroll
                    for (int i = 0; i < NR; ++i)
                        if (i < nreg) v[n][i] = lds[Ln.pj ^ poff(Ln, i)];
                }
                __syncthreads();
            }
            L = Ln;
        }
        // ---- the sub-stage's steps, in their fixed order
        if constexpr (NV == 2) {
            if (steps & ST_SEED) element_op<NV, NR, 2>(a, v, L, S->seed, tile, nreg, active);
        }
        if (steps & ST_FLIP_PRE) element_op<NV, NR, 0>(a, v, L, S->flip_pre, tile, nreg, active);
        if (steps & ST_PHASE) apply_phases<NV, NR>(a, S, v, L, tile, U, active);
        if (steps & ST_MAT_PRE) {
            R m[8];
            const PK_CONST double* mp = cptr(a.mats) + 8 * mat_pre;
#pragma unroll
            for (int e = 0; e < 8; ++e) m[e] = (R)mp[e];
            apply_mat<NV, NR>(v, mat_pre_a, m);
        }
        if (steps & ST_H1) apply_hmask<NV, NR>(v, hmask1);
        if (steps & ST_FLIP_MID) element_op<NV, NR, 0>(a, v, L, flip_mid, tile, nreg, active);
        if (steps & ST_H2) apply_hmask<NV, NR>(v, hmask2);
        if (steps & ST_MAT_POST) {
            R m[8];
            const PK_CONST double* mp = cptr(a.mats) + 8 * mat_post;
#pragma unroll
            for (int e = 0; e < 8; ++e) m[e] = (R)mp[e];
            apply_mat<NV, NR>(v, mat_post_a, m);
        }
        if ((steps & ST_MAT4) && active) op_mat4<NV, NR>(v, cptr(a.mats4) + 32 * S->mat4);
        if constexpr (NR > 8)
            if ((steps & ST_MAT4B) && active) op_mat4_hi<NV, NR>(v, cptr(a.mats4) + 32 * S->mat4b);
        if constexpr (NV == 2) {
            if (steps & ST_D2B) {
                R mh[8];
                const PK_CONST double* mp = cptr(a.mats) + 8 * S->d2b_mat;
#pragma unroll
                for (int e = 0; e < 8; ++e) mh[e] = (R)mp[8 + e];
                double g[3] = {0.0, 0.0, 0.0};
                if (active) apply_d2bwd<NV, NR>(v, S->d2b_a, mh, mp + 16, g);
                const double scale = 2.0 * (double)S->d2b_gscale;
                const int gslot = S->d2b_gslot;
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    const double tot = block_sum<NT>(g[t], red);
                    if (tid == 0) a.gpart[gslot + t * P->ntiles + tile] = scale * tot;
                }
            }
            if (steps & ST_D4B) {
                double g[3] = {0.0, 0.0, 0.0};
                if (active) op_d4bwd<NV, NR>(v, cptr(a.mats4) + 32 * S->d4b_mat, g);
                const double scale = 2.0 * (double)S->d4b_gscale;
                const int gslot = S->d4b_gslot;
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    const double tot = block_sum<NT>(g[t], red);
                    if (tid == 0) a.gpart[gslot + t * P->ntiles + tile] = scale * tot;
                }
            }
        }
        if (steps & ST_SCALE) {
            const R sc = (R)P->scale;
#pragma unroll
            for (int n = 0; n < NV; ++n)
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    v[n][i].x *= sc;
                    v[n][i].y *= sc;
                }
        }
        if (steps & ST_READ) element_op<NV, NR, 1>(a, v, L, S->read, tile, nreg, active);
    }

    // ---- norm partial of the final state (FP64 for FP64 data; Neumaier-
    //      compensated FP32 lane sums, then FP64, for FP32 data)
    if (a.want_norm && (C.flags & PASS_LAST)) {
        double part = 0.0;
        if (active) {
            if constexpr (sizeof(R) == 8) {
#pragma unroll
                for (int i = 0; i < NR; ++i)
                    if (i < nreg) part += v[0][i].x * v[0][i].x + v[0][i].y * v[0][i].y;
            } else {
                float s = 0.0f, c = 0.0f;
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    if (i >= nreg) continue;
                    const float term = v[0][i].x * v[0][i].x + v[0][i].y * v[0][i].y;
                    const float t = s + term;
                    c += (fabsf(s) >= fabsf(term)) ? ((s - t) + term) : ((term - t) + s);
                    s = t;
                }
                part = (double)s + (double)c;
            }
        }
        const double tot = block_sum<NT>(part, red);
        if (tid == 0) a.partials[P->part_base + tile] = tot;
    }
}

// Tiles first, first + stride, ... (below ntiles) of one pass.  With one vector, two register
// buffers alternate: the next tile's HBM loads are issued before the current
// tile's LDS stages, so memory traffic overlaps the exchange work of the one
// workgroup an LDS-sized tile leaves per CU.  The prefetch is unconditional
// (past the end it re-reads the current tile) so the wait counts stay static.
// PH: the pass has tile-part product tables, whose entries are loaded with the
// tile's amplitudes.  NT: the pass streams (PASS_STREAM).  FULL: the tile fills
// the workgroup (k == KMAX: every thread active, every register used) and lane
// offsets fit 32 bits, so every thread issues the same loads on every path; the
// compiler can then wait for exactly the current tile's loads (the next tile's
// stay in flight through the exchanges), where path-dependent load counts make
// it wait for all of them at the first LDS write.
template <typename R, int NV, int KMAX, int RB, bool PH, bool NT, bool FULL>
__device__ __forceinline__ void run_tiles_ph(const KArgs& a, const PK_CONST Pass* P, int64_t first,
                                             int64_t stride, int64_t ntiles, typename Cplx<R>::T* lds, double* red,
                                             int64_t chunk) {
    using T = typename Cplx<R>::T;
    constexpr int NR = 1 << RB;
    PassCtx C = make_ctx<(int)sizeof(R) * 2, RB>(a, P);
    if constexpr (FULL) {
        C.active = true;
        C.nreg = NR;
        C.flags &= ~PASS_WIDE;
    }
    const int64_t off = P->state_off;
    const int nfrun = P->nfrun;
    auto base_of = [&](int64_t t) { return off + deposit(t, P->frun, nfrun); };
    auto refs_of = [&](int64_t t) { return PH ? load_refs<R>(a, P, t) : TileRefs<R>{(R)1, (R)0}; };
    // the workgroup's tiles come in runs of `chunk` consecutive ones, the runs
    // `stride` runs apart (chunk 1: every stride-th tile)
    const int64_t jump = (stride - 1) * chunk;
    auto next = [&](int64_t t, int64_t& j) {
        if (j + 1 < chunk) {
            ++j;
            return t + 1;
        }
        j = 0;
        return t + 1 + jump;
    };
    if constexpr (NV == 2) {
        // two vectors already fill the register file: no second buffer
        int64_t j = 0;
        for (int64_t tile = first; tile < ntiles; tile = next(tile, j)) {
            T v[NV][NR];
            const int64_t base = base_of(tile);
            const TileRefs<R> u = refs_of(tile);
            load_tile<R, NV, NR, NT>(a, C, base, v);
            compute_tile<R, NV, KMAX, RB>(a, P, C, tile, v, u, lds, red);
            store_tile<R, NV, NR, NT>(a, C, base, v);
        }
    } else {
        T va[1][NR], vb[1][NR];
        int64_t ta = first, ja = 0;
        int64_t basea = base_of(ta);
        TileRefs<R> ua = refs_of(ta);
        load_tile<R, 1, NR, NT>(a, C, basea, va);
        for (;;) {
            int64_t jb = ja;
            const int64_t tb = next(ta, jb);
            const int64_t tbc = tb < ntiles ? tb : ta;
            const int64_t baseb = base_of(tbc);
            const TileRefs<R> ub = refs_of(tbc);
            load_tile<R, 1, NR, NT>(a, C, baseb, vb);
            compute_tile<R, 1, KMAX, RB>(a, P, C, ta, va, ua, lds, red);
            store_tile<R, 1, NR, NT>(a, C, basea, va);
            if (tb >= ntiles) break;
            int64_t jc = jb;
            const int64_t tc = next(tb, jc);
            const int64_t tcc = tc < ntiles ? tc : tb;
            const int64_t basec = base_of(tcc);
            ua = refs_of(tcc);
            load_tile<R, 1, NR, NT>(a, C, basec, va);
            compute_tile<R, 1, KMAX, RB>(a, P, C, tb, vb, ub, lds, red);
            store_tile<R, 1, NR, NT>(a, C, baseb, vb);
            if (tc >= ntiles) break;
            ta = tc;
            ja = jc;
            basea = basec;
        }
    }
}

// STREAM: a single-instance launch: honour PASS_STREAM and Pass::overlap (a
// batched launch's instances are small).
template <typename R, int NV, int KMAX, int RB, bool STREAM = false>
__device__ __forceinline__ void run_tiles(const KArgs& a, const PK_CONST Pass* P, int64_t first,
                                          int64_t stride, int64_t ntiles, typename Cplx<R>::T* lds, double* red,
                                          int64_t chunk = 1) {
    if (first >= ntiles) return;
    // Pass::overlap selects the FULL loop where it applies (single-instance launches).
    // Only the kernels with 4 register bits have it: there it keeps the occupancy
    // the other loops allow (FP64 2^13 tiles: 237 VGPRs either way; FP32: 146 -> 201,
    // one workgroup a CU either way), while the FP32 kernel with 5 would go from 241
    // to 359 VGPRs (one workgroup a CU instead of two, 17.7 -> 21.6 ms an iteration)
    // or spill under a 256 cap, and with 3 it spills under the 128 cap.
    constexpr bool kHasFull = STREAM && NV == 1 && RB == 4;
    const bool full = kHasFull && P->overlap && P->k == KMAX && !(P->flags & PASS_WIDE);
    if (P->nuref > 0) {
        if (full) run_tiles_ph<R, NV, KMAX, RB, true, false, true>(a, P, first, stride, ntiles, lds, red, chunk);
        else run_tiles_ph<R, NV, KMAX, RB, true, false, false>(a, P, first, stride, ntiles, lds, red, chunk);
        return;
    }
    if constexpr (STREAM && NV == 1) {
        if (P->flags & PASS_STREAM) {
            if (full) run_tiles_ph<R, NV, KMAX, RB, false, true, true>(a, P, first, stride, ntiles, lds, red, chunk);
            else run_tiles_ph<R, NV, KMAX, RB, false, true, false>(a, P, first, stride, ntiles, lds, red, chunk);
            return;
        }
    }
    if (full) run_tiles_ph<R, NV, KMAX, RB, false, false, true>(a, P, first, stride, ntiles, lds, red, chunk);
    else run_tiles_ph<R, NV, KMAX, RB, false, false, false>(a, P, first, stride, ntiles, lds, red, chunk);
}

// ---------------------------------------------------------------------------- kernels

// With 3 register bits the kernel is held to 128 VGPRs (four waves per SIMD): two
// 2^12-tile workgroups of 512 threads then share a CU, as their LDS allows.
template <typename R, int NV, int KMAX, int RB>
__global__ void __launch_bounds__(1 << (KMAX - RB)) __attribute__((amdgpu_waves_per_eu(RB == 3 ? 4 : 1)))
pass_kernel(KArgs a) {
    using T = typename Cplx<R>::T;
    __shared__ T lds[1 << KMAX];
    __shared__ double red[16];  // reduction scratch
    const PK_CONST Pass* P = cptr(a.passes) + a.pass;
    const int64_t ntiles = P->ntiles;
    const int64_t G = gridDim.x;
    const int walk = P->walk;
    if (walk == 0) {
        run_tiles<R, NV, KMAX, RB, true>(a, P, blockIdx.x, G, ntiles, lds, red);
    } else {
        // runs of c tiles that are neighbours in the tile index (the lowest free state
        // bits): a workgroup's next tile, whose loads are in flight, lies next to the
        // one it works on
        const int64_t c = walk > 0 ? walk : (ntiles + G - 1) / G;
        run_tiles<R, NV, KMAX, RB, true>(a, P, (int64_t)blockIdx.x * c, G, ntiles, lds, red, c);
    }
}

// Team barrier of the batched launch: every member adds one to the team's
// counter after its tiles, then waits until all team_size members of this
// round have.  Device-scope fences on both sides make the members' stores
// visible across CUs and XCDs.  The wait is bounded by `ticks` of the
// constant-rate wall clock: on time-out (the team's workgroups are not all
// resident) the barrier returns false, and a workgroup whose barrier failed
// once no longer waits at later ones, so every wave reaches the kernel's end.
__device__ __forceinline__ bool team_barrier(unsigned int* bar, unsigned int target, uint64_t ticks, bool broken,
                                             int* flag) {
    // every wave first waits for its own stores to reach the L2 (__syncthreads waits
    // only for LDS traffic), so that thread 0's fence below covers the whole tile
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(bar, 1u);
        int ok = 0;
        if (!broken) {
            const uint64_t t0 = wall_clock64();
            for (;;) {
                if (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) {
                    ok = 1;
                    break;
                }
                if (wall_clock64() - t0 > ticks) break;
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __threadfence();
        *flag = ok;
    }
    __syncthreads();
    return *flag != 0;
}

// Grid-wide barrier of the persistent repeat launch.  As team_barrier, but the
// workgroup whose arrival completes the round stores the round's target to a
// release word on another cache line, and the others poll that word: polling the
// arrival counter itself (hundreds of workgroups) delays the arrivals queued
// behind the polls on the same line.  bar[0] counts arrivals, bar[32] is the
// release word; both start at zero.
__device__ __forceinline__ bool grid_barrier(unsigned int* bar, unsigned int target, uint64_t ticks, bool broken,
                                             int* flag) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned int old = atomicAdd(bar, 1u);
        unsigned int* release = bar + 32;
        if (old + 1u == target) __hip_atomic_store(release, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 0;
        if (!broken) {
            const uint64_t t0 = wall_clock64();
            for (;;) {
                if (__hip_atomic_load(release, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) {
                    ok = 1;
                    break;
                }
                if (wall_clock64() - t0 > ticks) break;
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __threadfence();
        *flag = ok;
    }
    __syncthreads();
    return *flag != 0;
}

// L and the norm of one finished instance, written by one workgroup.
template <int NT>
__device__ __forceinline__ void finish_instance(const KArgs& a, const PK_CONST InstDesc* D, int inst, bool ok,
                                                double* L_out, double* norm_out, double* red) {
    if (threadIdx.x == 0) {
        double L = 0.0;
        for (int m = 0; m < D->nmarked; ++m) L += a.reads[D->read_base + m];
        L_out[inst] = ok ? L : __builtin_nan("");
    }
    if (norm_out) {
        double s = 0.0;
        const int64_t nt = D->ntiles_last, pb = D->part_base;
        for (int64_t t = threadIdx.x; t < nt; t += NT) s += a.partials[pb + t];
        const double tot = block_sum<NT>(s, red);
        if (threadIdx.x == 0) norm_out[inst] = ok ? tot : __builtin_nan("");
    }
    __syncthreads();
}

// Multiverse batch in one persistent launch.  First the teams: the j-th
// workgroup of XCD x (w = j * n_xcd + x) is member j mod team_size of team
// (j / team_size) * n_xcd + x; a team walks the passes of its large instances
// together, its members taking the tiles of each pass in turn, with a team
// barrier between passes.  Then every workgroup takes whole instances from the
// queue (largest first) and runs all their passes itself.
template <typename R, int KMAX, int RB>
__global__ void __launch_bounds__(1 << (KMAX - RB)) batched_kernel(KArgs a, BatchArgs b) {
    using T = typename Cplx<R>::T;
    constexpr int NT = 1 << (KMAX - RB);
    __shared__ T lds[1 << KMAX];
    __shared__ double red[16];  // reduction scratch
    __shared__ int item;
    __shared__ int flag;
    const PK_CONST InstDesc* idesc = cptr(b.idesc);
    const int w = blockIdx.x;
    const int xcd = w % b.n_xcd, j = w / b.n_xcd;
    const int team = b.team_size > 0 ? (j / b.team_size) * b.n_xcd + xcd : b.n_teams;
    if (team < b.n_teams) {
        const int member = j % b.team_size;
        unsigned int target = 0;
        bool broken = false;
        const int q0 = cptr(b.team_off)[team], q1 = cptr(b.team_off)[team + 1];
        for (int q = q0; q < q1; ++q) {
            const int inst = cptr(b.team_list)[q];
            const PK_CONST InstDesc* D = idesc + inst;
            bool ok = true;
            for (int p = 0; p < D->npass; ++p) {
                const PK_CONST Pass* P = cptr(a.passes) + D->first_pass + p;
                run_tiles<R, 1, KMAX, RB>(a, P, member, b.team_size, P->ntiles, lds, red);
                target += (unsigned int)b.team_size;
                const bool passed = team_barrier(b.bars + team, target, b.spin_ticks, broken, &flag);
                broken = broken || !passed;
                ok = ok && passed;
            }
            if (member == 0) finish_instance<NT>(a, D, inst, ok, b.L_out, b.norm_out, red);
        }
    }
    for (;;) {
        if (threadIdx.x == 0) item = (int)atomicAdd(b.queue, 1u);
        __syncthreads();
        const int it = item;
        __syncthreads();
        if (it >= b.n_solo) break;
        const int inst = cptr(b.order)[it];
        const PK_CONST InstDesc* D = idesc + inst;
        for (int p = 0; p < D->npass; ++p) {
            const PK_CONST Pass* P = cptr(a.passes) + D->first_pass + p;
            run_tiles<R, 1, KMAX, RB>(a, P, 0, 1, P->ntiles, lds, red);
            // this workgroup's stores must be visible to its own loads of the next pass:
            // every wave waits for its stores to complete before the barrier
            __builtin_amdgcn_s_waitcnt(0);
            __threadfence_block();
            __syncthreads();
        }
        finish_instance<NT>(a, D, inst, true, b.L_out, b.norm_out, red);
    }
}

// G^reps in one persistent launch (the full search of Sec. 5.1: n_t applications
// of one Grover iteration): every workgroup walks its tiles of each pass, then
// waits at a grid-wide barrier (grid_barrier) before the next pass.  The first application reads src0, the later ones work in place on
// dst0; the norm partials are written by the last application only.  Every
// workgroup of the grid must be resident at once (the grid is the occupancy
// limit); if a barrier times out, the workgroup stops waiting at later ones and
// the readouts and norm partials are overwritten with NaN, so a failed run is
// visible in L and the norm instead of hanging.
template <typename R, int KMAX, int RB>
__global__ void __launch_bounds__(1 << (KMAX - RB)) repeat_kernel(KArgs a, RepeatArgs r) {
    using T = typename Cplx<R>::T;
    __shared__ T lds[1 << KMAX];
    __shared__ double red[16];
    __shared__ int flag;
    unsigned int target = 0;
    bool broken = false;
    for (int64_t rep = 0; rep < r.reps; ++rep) {
        KArgs ar = a;
        if (rep > 0) ar.src0 = a.dst0;
        ar.want_norm = a.want_norm && rep == r.reps - 1;
        for (int p = 0; p < r.npass; ++p) {
            const PK_CONST Pass* P = cptr(a.passes) + r.pass0 + p;
            run_tiles<R, 1, KMAX, RB>(ar, P, blockIdx.x, gridDim.x, P->ntiles, lds, red);
            if (rep == r.reps - 1 && p == r.npass - 1) break;
            target += gridDim.x;
            broken = !grid_barrier(r.bar, target, r.spin_ticks, broken, &flag) || broken;
        }
    }
    if (broken) {
        const double nan = __builtin_nan("");
        for (int i = threadIdx.x; i < r.n_reads; i += blockDim.x) a.reads[i] = nan;
        for (int64_t i = threadIdx.x; i < r.n_part; i += blockDim.x) a.partials[r.part_base + i] = nan;
    }
}

// ---------------------------------------------------------------------------- host launchers

// Persistent launch: as many workgroups as fit on the device at once (capped by
// the tile count); each walks its tiles with the load of the next one in flight.
template <typename R, int NV, int KMAX, int RB>
hipError_t launch_pass_t(const KArgs& a, int64_t ntiles, int64_t wgs_per_cu, hipStream_t st) {
    static int ncu = 0, per_cu = 0;  // queried once per kernel instance
    if (ncu == 0) {
        int dev = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        auto kfn = pass_kernel<R, NV, KMAX, RB>;
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, 1 << (KMAX - RB), 0);
        if (ncu <= 0) ncu = 256;
        if (per_cu <= 0) per_cu = 1;
    }
    int64_t grid = (int64_t)ncu * (wgs_per_cu > 0 ? wgs_per_cu : per_cu);
    if (grid > ntiles) grid = ntiles;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((pass_kernel<R, NV, KMAX, RB>), dim3((unsigned)grid), dim3(1 << (KMAX - RB)), 0, st, a);
    return hipGetLastError();
}

// Kernel instances: one vector with 4 or 5 register bits, two vectors with 4.
template <typename R, int NV, int RB>
hipError_t launch_pass_r(int kmax, const KArgs& a, int64_t ntiles, int64_t cap, hipStream_t st) {
    if constexpr (RB == 3) {
        // 2^(KMAX - 3) threads: at most 1024, so at most 2^13-amplitude tiles
        switch (kmax) {
        case 9: return launch_pass_t<R, NV, 9, 3>(a, ntiles, cap, st);
        case 10: return launch_pass_t<R, NV, 10, 3>(a, ntiles, cap, st);
        case 11: return launch_pass_t<R, NV, 11, 3>(a, ntiles, cap, st);
        case 12: return launch_pass_t<R, NV, 12, 3>(a, ntiles, cap, st);
        case 13: return launch_pass_t<R, NV, 13, 3>(a, ntiles, cap, st);
        default: return hipErrorInvalidValue;
        }
    } else if constexpr (RB == 4) {
        switch (kmax) {
        case 10: return launch_pass_t<R, NV, 10, 4>(a, ntiles, cap, st);
        case 11: return launch_pass_t<R, NV, 11, 4>(a, ntiles, cap, st);
        case 12: return launch_pass_t<R, NV, 12, 4>(a, ntiles, cap, st);
        case 13: return launch_pass_t<R, NV, 13, 4>(a, ntiles, cap, st);
        case 14:
            if constexpr (sizeof(R) == 4) return launch_pass_t<R, NV, 14, 4>(a, ntiles, cap, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (kmax) {
        case 11: return launch_pass_t<R, NV, 11, 5>(a, ntiles, cap, st);
        case 12: return launch_pass_t<R, NV, 12, 5>(a, ntiles, cap, st);
        case 13: return launch_pass_t<R, NV, 13, 5>(a, ntiles, cap, st);
        case 14:
            if constexpr (sizeof(R) == 4) return launch_pass_t<R, NV, 14, 5>(a, ntiles, cap, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
        }
    }
}

template <typename R, int KMAX, int RB>
static hipError_t launch_batched_t(const KArgs& a, const BatchArgs& B, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL((batched_kernel<R, KMAX, RB>), dim3(grid), dim3(1 << (KMAX - RB)), 0, st, a, B);
    return hipGetLastError();
}

template <typename R, int KMAX, int RB>
static int batched_occupancy_t() {
    int per_cu = 0;
    auto kfn = batched_kernel<R, KMAX, RB>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, 1 << (KMAX - RB), 0) != hipSuccess) return 0;
    return per_cu;
}

// Kernel instances of the batched launch: KMAX 10..13 (14 for FP32), RB 4 or 5.
template <typename R, int RB, typename F>
static auto batched_instance(int kmax, F&& f) {
    switch (kmax) {
    case 10:
        if constexpr (RB == 4) return f(std::integral_constant<int, 10>{});
        break;
    case 11: return f(std::integral_constant<int, 11>{});
    case 12: return f(std::integral_constant<int, 12>{});
    case 13: return f(std::integral_constant<int, 13>{});
    case 14:
        if constexpr (sizeof(R) == 4) return f(std::integral_constant<int, 14>{});
        break;
    default: break;
    }
    return decltype(f(std::integral_constant<int, 13>{})){};
}

template <typename R, int RB>
hipError_t launch_batched_r(int kmax, const KArgs& a, const BatchArgs& B, unsigned grid, hipStream_t st) {
    bool found = false;
    hipError_t e = batched_instance<R, RB>(kmax, [&](auto K) {
        found = true;
        return launch_batched_t<R, decltype(K)::value, RB>(a, B, grid, st);
    });
    return found ? e : hipErrorInvalidValue;
}

template <typename R, int RB>
int batched_occupancy_r(int kmax) {
    return batched_instance<R, RB>(kmax, [&](auto K) { return batched_occupancy_t<R, decltype(K)::value, RB>(); });
}


template <typename R, int KMAX, int RB>
static hipError_t launch_repeat_t(const KArgs& a, const RepeatArgs& r, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL((repeat_kernel<R, KMAX, RB>), dim3(grid), dim3(1 << (KMAX - RB)), 0, st, a, r);
    return hipGetLastError();
}

template <typename R, int RB>
hipError_t launch_repeat_r(int kmax, const KArgs& a, const RepeatArgs& r, unsigned grid, hipStream_t st) {
    bool found = false;
    hipError_t e = batched_instance<R, RB>(kmax, [&](auto K) {
        found = true;
        return launch_repeat_t<R, decltype(K)::value, RB>(a, r, grid, st);
    });
    return found ? e : hipErrorInvalidValue;
}

template <typename R, int KMAX, int RB>
static int repeat_occupancy_t() {
    int per_cu = 0;
    auto kfn = repeat_kernel<R, KMAX, RB>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, 1 << (KMAX - RB), 0) != hipSuccess) return 0;
    return per_cu;
}

template <typename R, int RB>
int repeat_occupancy_r(int kmax) {
    return batched_instance<R, RB>(kmax, [&](auto K) { return repeat_occupancy_t<R, decltype(K)::value, RB>(); });
}

}  // namespace pk
