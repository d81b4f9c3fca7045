// Schedule tables shared by the host plan compiler and the device kernels.
//
// A plan lowers a gate list to passes.  One pass streams the whole state
// once: the state is cut into tiles of 2^k amplitudes whose labels differ only
// in k chosen bit positions (the tile bits, always including the lowest
// "carrier" bits so that every memory run is contiguous), every tile is loaded
// into one workgroup, the pass's gates are applied, and the tile is written
// back.  Inside a tile, each thread holds 16 (or 32) amplitudes in registers
// whose local labels differ in 4 (or 5) "register bits"; a stage applies the
// gates on those bits as butterflies in registers, and an LDS exchange moves the
// tile to the next stage's register bits.  This is the pair update of Sec. 3 (Eq. resmat1)
// applied to all partner pairs of a qubit at once, grouped so that the state
// is read from HBM once per group of qubits instead of once per gate.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace pk {

constexpr int kMaxRegBits = 5;       // register bits per stage (4 or 5): 16 or 32 amplitudes per thread
constexpr int kMaxTileBits = 14;     // fp32 limit (fp64: 13), LDS = 2^k * element
constexpr int kMaxQubits = 31;
constexpr int kMaxNV = 2;            // vectors carried by a pass: psi, or psi and lambda

enum OpKind : int32_t {
    OP_H = 0,      // unnormalised Hadamard butterfly (x+y, x-y) on register bit a
    OP_MAT = 1,    // 2x2 complex matrix mats[arg] on register bit a
    OP_FLIP = 2,   // negate the amplitude flips[arg] (Oracle items, Inv's C_0 fix)
    OP_SCALE = 3,  // multiply every amplitude by the pass scale
    OP_READ = 4,   // reads[flips[arg].slot] = |C|^2 of the amplitude flips[arg]
    OP_SEED = 5,   // lambda = dL * psi at the amplitude flips[arg] (backward start)
    OP_D2BWD = 6,  // backward D2: psi <- D^H psi, grad += Re<lambda|dD|psi>, lambda <- D^H lambda
    OP_MAT4 = 7,   // 4x4 complex matrix mats4[arg] on register bits a (qubit is1) and a + 1 (qubit is2), a = 0 or 2
    OP_D4BWD = 8,  // backward D4 on register bits 0 and 1, as OP_D2BWD with 4x4 matrices
    OP_PHASE = 9,  // controlled phase (CPHASE, CPHASEK): e^{i theta} where both bits are 1
};

constexpr int kPhaseSlots = 4;  // phase accumulators per sub-stage
constexpr int kTwidBits = 10;   // index bits of one product table (2^10 entries at most)
constexpr int kMaxURefs = 64;   // tile-part tables one pass reads (one per lane of a wave)

// One controlled phase as the kernel applies it in a sub-stage.  The amplitudes
// whose two qubits are both 1 get the factor c + i s.  Each qubit's bit sits on
// a register bit, on the thread's part of the local label, or in the tile index
// (a qubit outside the tile, so the same for the whole tile).  The register
// bits involved define the phase's accumulator slot (Stage::phase_pm); a thread
// multiplies the factors of a slot together and applies the product once to
// every register whose index has the slot's register bits set.  A sub-stage's
// phases are stored grouped by slot (Stage::phase_cnt).
//
// Product tables.  The factors of a slot's phases that depend only on the tile
// index (tmask == 0) multiply to a function of the tile-index bits they name,
// and those that depend only on the thread (fmask == 0) to a function of the
// thread's label bits.  The host tabulates both (Plan::twid): up to two tables
// for the tile part, indexed by the named tile-index bits (at most kTwidBits
// each; bits tied by one phase share a table), and one for the thread part.
// A pass lists its tile-part tables (URef, at most kMaxURefs); when a wave
// issues a tile's loads, lane r also loads the entry of the pass's table r for
// that tile, and the phase step reads it back from the lane.  The thread part
// is one vector load per slot.  The phases left over, and every phase that did
// not fit a table, run in a branch-free loop.
struct PhaseOp {
    int32_t slot;    // accumulator slot of the sub-stage (within a slot, the phases
                     // in the product tables come first: see Stage::phase_ucnt)
    uint32_t tmask;  // local label bits held by the thread index that must be 1
    int64_t fmask;   // tile-index bits that must be 1
    double cm1, s;   // the factor as (c - 1, s): 1 + on * (c - 1) and on * s give the
                     // factor or 1 without a select (c - 1 is exact for c >= 1/2)
};

// One step of a stage's op list, as the plan compiler schedules it on the host;
// the list is then packed into sub-stages (Stage) for the device.
struct Op {
    int32_t kind;
    int32_t a;      // register bit for OP_H / OP_MAT / OP_D2BWD
    int32_t arg;    // matrix index (OP_MAT, OP_MAT4; D2BWD, D4BWD: first of five), flip index (FLIP/READ/SEED)
    int32_t gslot;  // OP_D2BWD, OP_D4BWD: base of this gate's gradient partials
    float gscale;   // OP_D2BWD, OP_D4BWD: 1/s^2 for the deferred scale s carried at that point
    int32_t pad;
};

// Device tables below: all fields are 32- or 64-bit so that the kernels read
// them with scalar loads from the constant address space.
//
// One sub-stage: a fixed sequence of optional steps applied to the registers,
// in this order: seed, flip, controlled phases, matrix, Hadamards (mask 1),
// flip, Hadamards (mask 2), matrix, 4x4 matrix on register bits 0 and 1, 4x4
// matrix on register bits 2 and 3, backward D2, backward D4, scale, read.  A stage's op list is packed into
// as many sub-stages as its order needs; only the first of them exchanges the
// tile through LDS (`exchange`), the others keep the layout.  Straight-line
// steps instead of an op loop let the compiler update the register tile in
// place.
// Steps present in a sub-stage (Stage::steps): the kernel reads this one word
// and loads the parameters of the present steps only.
enum StepBits : int32_t {
    ST_EXCHANGE = 1, ST_SEED = 2, ST_FLIP_PRE = 4, ST_PHASE = 8, ST_MAT_PRE = 16, ST_H1 = 32, ST_FLIP_MID = 64,
    ST_H2 = 128, ST_MAT_POST = 256, ST_MAT4 = 512, ST_D2B = 1024, ST_D4B = 2048, ST_SCALE = 4096, ST_READ = 8192,
    ST_MAT4B = 16384,
};

// 16-byte aligned so that the slot table (phase_pm .. phase_tt) can be read as
// four aligned 16-byte words.
struct alignas(16) Stage {
    int32_t steps;            // StepBits of the steps below that are present
    int32_t rb[kMaxRegBits];  // local tile bit held by register bit a (-1 when unused)
    int32_t rbs[kMaxRegBits]; // the same bits sorted ascending (-1 entries last)
    int32_t exchange;         // 1: move the tile into this layout through LDS first
    int32_t seed;             // flip index of a SEED (backward start) or -1
    int32_t flip_pre;         // flip index or -1
    int32_t phase_first;      // first PhaseOp of this sub-stage's controlled phases
    int32_t phase_count;      // number of them (diagonal: any order)
    int32_t phase_pm[kPhaseSlots];   // register-bit mask of each accumulator slot, -1 when unused
    int32_t phase_cnt[kPhaseSlots];  // phases of each slot, stored slot after slot
    int32_t phase_ucnt[kPhaseSlots]; // of them, the leading ones whose factors the slot's product
                                     // tables hold (the kernel loops over the rest)
    int32_t phase_tt[kPhaseSlots];   // Plan::twid entry of the slot's thread-part table, or -1
    int32_t mat_pre_a;        // register bit of a matrix before the Hadamards, or -1
    int32_t mat_pre;          // its matrix index
    int32_t hmask1;           // register bits that get a Hadamard
    int32_t flip_mid;         // flip index between the two Hadamard masks, or -1
    int32_t hmask2;
    int32_t mat_post_a;       // register bit of a matrix after the Hadamards, or -1
    int32_t mat_post;
    int32_t d2b_a;            // backward D2 on this register bit, or -1
    int32_t d2b_mat;          // first of its five matrices
    int32_t d2b_gslot;        // base of its gradient partials
    float d2b_gscale;         // 1/s^2 for the deferred scale s at that point
    int32_t mat4;             // 4x4 matrix on register bits 0 (qubit is1) and 1 (qubit is2), or -1
    int32_t d4b_mat;          // backward D4 on register bits 0 and 1: first of its five matrices, or -1
    int32_t d4b_gslot;
    float d4b_gscale;
    int32_t scale;            // 1: multiply by the pass scale
    int32_t read;             // flip index of a READ or -1
    int32_t mat4b;            // 4x4 matrix on register bits 2 (qubit is1) and 3 (qubit is2), or -1: a
                              // second, disjoint qubit pair of the same stage
    // product tables of the slots (see PhaseOp): the tile part's first and second
    // table (index into the pass's URef list, or -1), the thread part's local
    // label bits
    alignas(16) int32_t phase_ut0[kPhaseSlots];
    int32_t phase_ut1[kPhaseSlots];
    uint32_t phase_ttm[kPhaseSlots];
    // Thread -> local label map of the layout.  nlanes == 0: the thread index's bits
    // go to the local bits that are not register bits, in ascending order.  Else
    // thread bit i < nlanes goes to local bit (lanes >> 4 i) & 15 and the thread's
    // higher bits to the bits of lanes_rest in ascending order: the planner picks
    // the low bits so that the lanes sharing an LDS access cycle hit distinct banks
    // under the slot swizzle (only for layouts that neither load nor store HBM).
    int32_t nlanes;
    uint32_t lanes;
    uint32_t lanes_rest;
};
static_assert(offsetof(Stage, phase_pm) % 16 == 0 && offsetof(Stage, phase_cnt) == offsetof(Stage, phase_pm) + 16 &&
                  offsetof(Stage, phase_ucnt) == offsetof(Stage, phase_pm) + 32 &&
                  offsetof(Stage, phase_tt) == offsetof(Stage, phase_pm) + 48 &&
                  offsetof(Stage, phase_ut0) % 16 == 0 && offsetof(Stage, phase_ut1) == offsetof(Stage, phase_ut0) + 16 &&
                  offsetof(Stage, phase_ttm) == offsetof(Stage, phase_ut0) + 32,
              "slot table must be four consecutive aligned 16-byte words");
static_assert(offsetof(Stage, mat_pre_a) % 16 == 0 && offsetof(Stage, mat_pre) == offsetof(Stage, mat_pre_a) + 4 &&
                  offsetof(Stage, hmask1) == offsetof(Stage, mat_pre_a) + 8 &&
                  offsetof(Stage, flip_mid) == offsetof(Stage, mat_pre_a) + 12 &&
                  offsetof(Stage, hmask2) == offsetof(Stage, mat_pre_a) + 16 &&
                  offsetof(Stage, mat_post_a) == offsetof(Stage, mat_pre_a) + 20 &&
                  offsetof(Stage, mat_post) == offsetof(Stage, mat_pre_a) + 24,
              "one-qubit step parameters must be two consecutive aligned 16-byte words");

// One amplitude addressed by (tile, local label) in a given pass.
struct Flip {
    int64_t tile;
    int32_t j;
    int32_t slot; // READ: readout slot; SEED: instance index
};

enum PassFlags : int32_t {
    PASS_FIRST = 1,    // read from the input buffers
    PASS_LAST = 2,     // final pass of the instance
    PASS_NORM = 4,     // (reserved)
    PASS_SKIP_V0 = 8,  // do not store vector 0 (backward: the recovered psi_in is not needed)
    PASS_SEED_V1 = 16, // vector 1 is not read: it starts as zero and is seeded (backward start)
    PASS_WIDE = 32,    // a thread's byte offset inside a tile may exceed 32 bits
    PASS_STREAM = 64,  // loads and stores are nontemporal (streaming): the last forward pass of
                       // an FP64 instance far larger than the memory-side cache, when it
                       // writes the tile back in the layout it read
};

// State size from which an FP64 instance's last forward pass streams
// (PASS_STREAM).  Measured at n_q = 30 (16 GiB): the last pass of the Grover
// iteration went from 6.7 to 5.9 ms (the iteration from 35.1 to 34.4 ms);
// streaming the other passes made two of them slower, and in FP32 (8-byte
// accesses) the last pass too, as did the last pass of the QFT, which writes the
// tile back in another layout (relabelled SWAPs; 8.05 -> 8.37 ms).  Small states
// are left alone: their next launch re-reads them from the caches.
constexpr int64_t kStreamBytes = (int64_t)1 << 30;

constexpr int kMaxRuns = 16;

// A run (src, len, dst) moves bits src..src+len-1 of a label to dst..dst+len-1.
struct Run {
    int32_t src, len, dst, pad;
};

// A tile-part product table of a pass: its first Plan::twid entry and the
// tile-index bits that index it.
struct URef {
    int32_t base;
    int32_t pad;
    int64_t mask;
};

struct Pass {
    int32_t k;           // tile bits
    int32_t nstages;
    int32_t stage_begin;
    int32_t flags;
    int64_t ntiles;      // 2^(nq - k)
    int64_t state_off;   // element offset of the instance in the packed buffer
    double scale;        // applied by OP_SCALE
    int32_t part_base;   // norm partials: part_base + tile
    int32_t kmax;        // kernel instance (workgroup = 2^(kmax - rbits) threads)
    int32_t rbits;       // register bits per thread
    int32_t ntrun;       // runs of consecutive tile bits
    int32_t nfrun;       // runs of consecutive free bits
    int32_t nstrun;      // runs of the store map
    int32_t uref_begin;  // first URef of the pass
    int32_t nuref;       // number of them (at most kMaxURefs)
    int32_t walk;        // tiles of workgroup w in a single-instance launch over a grid of G:
                         // 0: w, w + G, ...; c > 1: runs of c consecutive tiles starting at
                         // w c, (w + G) c, ...; -1: one contiguous block of ceil(ntiles / G)
    int32_t overlap;     // single-instance launch, forward pass of full tiles: 1 keeps the next
                         // tile's loads in flight through the LDS exchanges (see run_tiles)
    int32_t tpos[16];    // global bit position of local tile bit l when the tile is read
    int32_t stpos[16];   // ... when it is written (differs after SWAPs done by relabelling)
    Run trun[kMaxRuns];  // local tile label -> state label (read)
    Run strun[kMaxRuns]; // local tile label -> state label (write)
    Run frun[kMaxRuns];  // tile index -> state label
};

// Per-instance entry of a batched launch: one workgroup runs all passes of
// one instance, so no two workgroups ever depend on each other.
// A rotation parameter triple (alpha, beta, gamma) of the angle array: kind 0
// is a D2 gate (five 2x2 matrices at slot), kind 1 a D4 gate (five 4x4 matrices).
struct ParamRef {
    int32_t kind;
    int32_t slot;
};

struct InstDesc {
    int32_t first_pass;
    int32_t npass;
    int32_t read_base;
    int32_t nmarked;
    int64_t part_base;
    int64_t ntiles_last;
};

// One output of the final FP64 combine: out[index] = sum of count doubles at
// workspace + src (in doubles), summed in a fixed order.
struct Reduction {
    int32_t target;  // 0: L, 1: norm, 2: angle gradient
    int32_t index;
    int64_t src;
    int64_t count;
};

} // namespace pk
