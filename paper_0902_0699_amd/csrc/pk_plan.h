// Host-side plan: validated problems and their compiled pass schedules.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "pk_desc.h"
#include "paperkern.h"

namespace pk {

// A primitive operation of the gate list: a one- or two-qubit gate on state
// bits, a controlled phase, or a diagonal sign operation on the whole state.
struct Prim {
    enum Kind { GATE, ORACLE, INV } kind;
    int bit;  // GATE: state bit b = nq - i_s (bit 0 is qubit n_q, the least significant)
    enum GKind { GH, GMAT, GD2, GMAT4, GD4, GPHASE, GSWAP } gk;
    int idx;         // GMAT / GMAT4 / GSWAP: static matrix index; GD2 / GD4: global D2 / D4 index
    int bit2 = -1;   // two-qubit gates and phases: state bit of the second qubit is2
    int param = -1;  // GD2 / GD4: index of the gate's angle triple
    double pc = 1.0, ps = 0.0;  // GPHASE: the factor e^{i theta} = pc + i ps
};

// A controlled phase as scheduled in a pass: la / lb are its local tile bits (-1
// for a qubit outside the tile), fmask the tile-index bits of the qubits outside
// the tile, b1 / b2 the state bits of both qubits in the tile's read layout.
struct HostPhase {
    int la, lb;
    int64_t fmask;
    int b1, b2;
    double c, s;
};

struct HostStage {
    int rb[kMaxRegBits];
    std::vector<Op> ops;
};

struct HostPass {
    int k = 0;
    std::vector<int> tbits;  // state bits of the tile: local bit l is tbits[l], carriers first
    std::vector<int> sbits;  // state bit that local bit l is written to (tbits permuted by SWAPs)
    std::vector<HostStage> stages;
    std::vector<HostPhase> phases;  // the pass's controlled phases (OP_PHASE arg indexes this)
    std::vector<Stage> subs;  // the stages packed into fixed-slot sub-stages (device form)
    int flags = 0;
    double scale = 1.0;
    int64_t ntiles = 0;
    int part_base = 0;
    int kmax = 13;
    int rbits = 4;
    int uref_begin = 0;  // tile-part tables of the pass (Plan::urefs)
    int nuref = 0;
};

struct Instance {
    int nq = 0;
    int64_t off = 0;
    std::vector<int64_t> marked;
    std::vector<Prim> prims;
    int d2_base = 0;
    int n_d2 = 0;
    std::vector<HostPass> fwd;
    std::vector<HostPass> bwd;
    int read_base = 0;   // readout slots
    int gpart_base = 0;  // backward gradient partial base
};

struct Tiling {
    int tile_bits;
    int carrier_bits;
    int fuse;
    int wgs_per_cu = 0;  // resident workgroups per CU for pass launches (0 = occupancy limit)
    int reg_bits = 4;    // register bits per thread in forward passes (4 or 5)
    int lane_order = 1;  // 1: lanes cover tile bits of good DRAM stride next to the carriers
    int page_cap = 0;    // >0: prefer at most this many tile bits at >= 2 MiB byte stride
};

// log2 of the page size the per-CU address translation cache works in (2 MiB).
constexpr int kPageByteBit = 21;

// Default tile and register bits per precision, the fastest settings measured
// for the n_q = 30 Grover iteration: FP64 tiles of 2^13 amplitudes with 16 per
// thread (2^9 threads); FP32 tiles of 2^13 with 32 per thread (2^8 threads) -- the
// 2^14 FP32 tile with 16 per thread needs 1024 threads, whose 128-register cap
// spills the register tile.
inline int default_tile_bits(int /*prec*/) { return 13; }
inline int default_reg_bits(int prec) { return prec == PK_FP64 ? 4 : 5; }
// A tile spanning 2^8 pages (the pass holding Inv at n_q = 30) misses the per-CU
// translation cache on most loads; spreading those bits over the passes, at most 4
// per tile, gives every FP64 pass >= 4.4 TB/s.  FP32 measured faster without it.
inline int default_page_cap(int prec) { return prec == PK_FP64 ? 4 : 0; }

// Batched launch.  Workgroups that share an XCD (and so an L2) form teams of
// team_size; a team runs the passes of its large instances together, with a
// barrier between passes, so that an instance too large for one workgroup is
// still spread over many CUs.  An instance is large when its first pass has at
// least min_team_tiles * team_size tiles.  Every other instance is taken whole
// by one workgroup from a queue.  team_size 0 turns teams off.  The device-scope
// fences of a team barrier cost more than a single workgroup's sweep of an
// instance of up to ~2^20 amplitudes, hence the high default threshold.
struct BatchConfig {
    int team_size = 16;
    int min_team_tiles = 64;
};

constexpr int kMaxTeams = 512;

struct Plan;

struct TeamSchedule {
    int n_teams = 0;
    int team_size = 0;
    int n_xcd = 1;
    std::vector<int32_t> team_off;   // n_teams + 1 offsets into team_list
    std::vector<int32_t> team_list;  // the large instances of each team, largest first
    std::vector<int32_t> solo;       // the rest, largest first (the queue's order)
};

// Teams for a persistent grid of `grid` workgroups dispatched round-robin over
// n_xcd XCDs: workgroup w sits on XCD w mod n_xcd; the j-th workgroup of an XCD
// (j = w / n_xcd) is member j mod team_size of that XCD's team j / team_size.
// Large instances go to teams by longest-processing-time first.
TeamSchedule team_schedule(const Plan* plan, int64_t grid, int n_xcd);

struct Plan {
    uint32_t magic = 0x504b504cu;
    int prec = PK_FP64;
    std::vector<Instance> inst;
    std::vector<double> static_mats;   // 8 doubles per ONEOP matrix, then its adjoint
    std::vector<double> static_mats4;  // 32 doubles per fixed two-qubit matrix, then its adjoint
    std::vector<double> default_angles; // 3 per D2 or D4 gate, in order
    std::vector<ParamRef> params;      // what each angle triple drives
    std::vector<PhaseOp> phases;       // controlled phases as scheduled (device table)
    std::vector<double> twid;          // product tables of the controlled phases (re, im pairs);
                                       // entry 0 is 1 (what lanes without a table load)
    std::vector<URef> urefs;           // tile-part tables of every pass
    std::vector<int32_t> walk;         // Pass::walk of each forward pass of instance 0 (empty: all 0)
    std::vector<int32_t> overlap;      // Pass::overlap of each forward pass of instance 0 (empty: all 0)
    int lane_maps = 1;                 // 1: LDS-only layouts get bank-spreading lane maps (Stage::lanes)
    int n_d2 = 0;
    int n_d4 = 0;
    int n_static = 0;
    int n_static4 = 0;
    bool backward_ok = true;
    Tiling tiling{13, 4, 1};
    BatchConfig batch;
    TeamSchedule team;              // the schedule of the current device grid
    std::string last_error;

    // flattened tables (forward passes of all instances, then backward passes)
    std::vector<Pass> passes;
    std::vector<Stage> stages;
    std::vector<Flip> flips;
    std::vector<InstDesc> idesc;    // batched launch: per-instance pass ranges
    std::vector<int32_t> order;     // instances by decreasing size (largest first)
    struct D2Grad { int d; int64_t gslot; int64_t nt; };  // d: angle triple index
    std::vector<D2Grad> d2_grad;    // where each D2's or D4's backward partials live
    int n_fwd_passes = 0;
    int64_t n_partials = 0;         // norm partials (sum over instances of last-pass tiles)
    int64_t n_reads = 0;
    int64_t n_gpart = 0;
    int64_t total_elems = 0;
    int max_nq = 0;

    // device state (uploaded lazily)
    int device = -1;
    void* d_tables = nullptr;
    size_t d_tables_bytes = 0;
};

// Validates and compiles; returns PK_OK or an error code with plan->last_error set.
int compile_plan(Plan* plan, const pk_problem* probs, int n_inst, int prec, std::string* err);
int recompile(Plan* plan, std::string* err);
std::string describe(const Plan* plan);

// Byte offsets of the device table arrays inside plan->d_tables.
struct TableLayout {
    size_t passes, stages, flips, phases, twid, urefs, mats, mats4, params, idesc, order, team_off, team_list, red, total;
};
TableLayout table_layout(const Plan* plan);

// Final-combine lists (L and norm per instance; angle gradients) for a workspace layout.
std::vector<Reduction> eval_reductions(const Plan* plan);
std::vector<Reduction> backward_reductions(const Plan* plan);

// Workspace layout (byte offsets) for op = PK_OP_EVAL / PK_OP_BACKWARD.
struct WsLayout {
    size_t mats, mats4, partials, reads, gpart, counters, state, total;
};
WsLayout workspace_layout(const Plan* plan, int op);

} // namespace pk
