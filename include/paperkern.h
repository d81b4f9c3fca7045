/*
 * libpaperkern -- state-vector gate sweeps for MI355X (gfx950).
 *
 * The library applies gate lists to n_q-qubit state vectors as described in
 * Tabakin & Julia-Diaz, "QCMPI: a parallel environment for quantum computing":
 *   - amplitudes C_n, n = 0 .. 2^n_q - 1, in standard order, n = sum_i q_i 2^(n_q-i)
 *     (Sec. 2.2, Eq. staten): qubit 1 is the most significant bit;
 *   - a one-qubit operator on qubit i_s updates every partner pair
 *     (n_0, n_0 + 2^(n_q-i_s)) by its 2x2 matrix (Sec. 3, Eq. resmat1, routine OneOpA);
 *   - HALL is the Hadamard on every qubit (Sec. 4.3, Eq. HALL);
 *   - ORACLE flips the sign of the marked amplitudes (Sec. 5.1, Eq. oracle1);
 *   - INV = 2|0..0><0..0| - I flips every amplitude except C_0 (Sec. 5.1, Eq. inversion);
 *   - D2 is the Wigner rotation D^(1/2)(alpha, beta, gamma) used as one-qubit
 *     noise (Sec. 6.3), read as R_z(alpha) R_y(beta) R_z(gamma) with
 *     R_z(phi) = diag(e^{-i phi/2}, e^{+i phi/2}) and rows/columns m = +1/2 (|0>), -1/2 (|1>).
 * The scalar read out is L = sum_{n in M} |C_n|^2 over the marked set M, the
 * success probability of the Grover search (Sec. 5.1).
 *
 * Memory: every state-sized buffer (inputs, outputs, workspace) is allocated by
 * the caller on the current HIP device and stays owned by the caller; a plan owns
 * only its small gate/schedule tables and captured graphs.  States are arrays of
 * interleaved complex numbers (re, im) in standard order: double2 for PK_FP64,
 * float2 for PK_FP32.  All device pointers must be 16-byte aligned.
 *
 * Errors: every entry point returns PK_OK (0) or a negative code; nothing throws
 * or aborts across this boundary.  pk_last_error() gives the text of the last
 * failure on a plan (including the HIP error string for PK_EDEVICE).
 * Streams: calls enqueue work on `stream` (a hipStream_t, NULL = null stream) and
 * do not synchronise the host; a plan may be used by one stream at a time,
 * distinct plans are independent.
 */
#ifndef PAPERKERN_H
#define PAPERKERN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------------------- */
#define PK_OK 0
#define PK_EINVAL (-1)        /* an argument violates the documented contract          */
#define PK_ENOMEM (-2)        /* host allocation failed or a buffer is too small        */
#define PK_EDEVICE (-3)       /* a HIP call failed; see pk_last_error()                 */
#define PK_EUNSUPPORTED (-4)  /* well-formed request outside what this build computes   */

/* ---- precisions ------------------------------------------------------------------ */
#define PK_FP64 0 /* complex128 storage, FP64 arithmetic                                  */
#define PK_FP32 1 /* complex64 storage, FP32 arithmetic, FP64 final reductions            */

/* ---- gate kinds (one pk_gate each; applied in list order, first gate first) ------- */
#define PK_GATE_ONEOP 0  /* any 2x2 complex operator on qubit is1 (Sec. 3, Eq. resmat1)    */
#define PK_GATE_H 1      /* Hadamard on qubit is1 (Sec. 3, Eq. NOTH)                       */
#define PK_GATE_HALL 2   /* Hadamard on qubits 1..n_q (Sec. 4.3, Eq. HALL)                 */
#define PK_GATE_ORACLE 3 /* C_x -> -C_x for every x of the marked set (Sec. 5.1)          */
#define PK_GATE_INV 4    /* C_n -> -C_n for n != 0 (Sec. 5.1, Eq. inversion)              */
#define PK_GATE_D2 5     /* D^(1/2)(alpha, beta, gamma) on qubit is1 (Sec. 6.3)           */
/* Two-qubit gates act on qubits is1, is2 (distinct) in the basis |q_is1 q_is2> =
 * |00>, |01>, |10>, |11> of Sec. 4 (Eqs. twoopB, resmat2), whatever the order of
 * is1 and is2 in significance.                                                        */
#define PK_GATE_TWOOP 6   /* any 4x4 complex operator (Eq. resmat2, routine TwoOpA)          */
#define PK_GATE_CNOT 7    /* control is1, target is2 (Sec. 4.2)                              */
#define PK_GATE_CPHASE 8  /* diag(1, 1, 1, -1) (Sec. 4.2)                                    */
#define PK_GATE_CPHASEK 9 /* diag(1, 1, 1, e^{2 pi i / 2^k}), k = 1..62 (Eq. cphasek)        */
#define PK_GATE_SWAP 10   /* exchanges qubits is1 and is2 (the QFT reordering of App. A)     */
#define PK_GATE_D4 11     /* D^(3/2)(alpha, beta, gamma), the two-qubit noise of Sec. 6.3:
                             Wigner's j = 3/2 function with the D2 Euler convention, rows and
                             columns m = 3/2 - (2 q_is1 + q_is2)                               */
#define PK_GATE_QFT 12    /* quantum Fourier transform of the register of qubits is1 .. is1+k-1
                             (k >= 1, is2 = 0): <n|QFT|n'> = 2^(-k/2) e^{2 pi i n n' / 2^k}, n the
                             register's value with qubit is1 most significant (App. A).  Lowered
                             to the circuit App. A draws, derived from that definition: per qubit,
                             CPHASEK with each earlier qubit (exponent: their distance + 1), then
                             its Hadamard; then the pair swaps that restore standard order      */
#define PK_GATE_QFT_NOSWAP 13 /* a labelled variant, not the paper's circuit: PK_GATE_QFT without the
                             final pair swaps, so the register comes out with its qubit order
                             reversed (amplitude of value n at the bit-reversed value).  Read
                             register one's distribution with pk_marginal_bitrev              */

/* ---- workspace queries ----------------------------------------------------------- */
#define PK_OP_EVAL 0
#define PK_OP_BACKWARD 1

typedef struct pk_gate {
    int32_t kind;     /* PK_GATE_*                                                        */
    int32_t is1;      /* target qubit, 1..n_q (1 = most significant); ignored for
                         HALL, ORACLE and INV                                             */
    int32_t is2;      /* second qubit of a two-qubit gate, 1..n_q, != is1; else 0         */
    int32_t k;        /* CPHASEK: the exponent k (1..62); QFT: the register size; else 0   */
    double op[32];    /* ONEOP: row-major 2x2 complex in op[0..7], op[2*(2a+b)] = Re<a|Op|b>,
                         op[2*(2a+b)+1] = Im<a|Op|b>; TWOOP: row-major 4x4 complex in
                         op[0..31], op[2*(4a+b)] = Re<a|V|b> with a, b = 2 q_is1 + q_is2;
                         entries must be finite                                           */
    double angle[3];  /* D2 and D4: alpha, beta, gamma (radians, finite)                  */
} pk_gate;

typedef struct pk_problem {
    int32_t nq;             /* qubits: 1..30 for PK_FP64, 1..31 for PK_FP32             */
    int32_t n_gates;        /* >= 0                                                       */
    const pk_gate* gates;   /* host array of n_gates, copied by pk_create                 */
    int64_t n_marked;       /* size of the marked set M, 0..64                            */
    const int64_t* marked;  /* host array of distinct labels in [0, 2^nq); copied         */
} pk_problem;

typedef struct pk_plan pk_plan;

/*
 * pk_create -- validate n_inst problems and compile their pass schedules.
 * Gates on distinct qubits commute and diagonal gates commute with each other;
 * the compiler uses only those two facts to group gates into passes over the
 * state (each pass reads and writes every amplitude once).  Controlled phases
 * (CPHASE, CPHASEK) run in any pass their order allows, whatever the tile; a
 * SWAP of two qubits that are both inside a pass's tile moves no data (the
 * tile is written back with the two qubits exchanged).  The schedule is host
 * data; device tables are uploaded on first use.  Errors: PK_EINVAL for nq out of
 * range, a qubit label outside 1..nq, nonzero is2/k, non-finite op or angle,
 * duplicate or out-of-range marked labels, n_inst < 1, unknown prec or kind;
 * PK_ENOMEM if host allocation fails.  On error *out is set to NULL.
 */
int pk_create(const pk_problem* probs, int32_t n_inst, int32_t prec, pk_plan** out);

/*
 * pk_set_tiling -- choose the pass kernel's tile: 2^tile_bits amplitudes per
 * workgroup (fp64: 4..13, fp32: 4..14; tiles below 2^(reg_bits + 6) leave
 * threads of the smallest kernel idle), of which the carrier_bits lowest state
 * bits (0..6) are always part of a tile so that each memory run is
 * 2^carrier_bits contiguous amplitudes; fuse = 0 turns fusion off (one sweep per
 * gate, the plain form).  lane_order picks which other tile bits the lanes of
 * a wave cover next to the carriers when a tile is read or written: 0 the
 * lowest state bits, 1 (default) bits whose byte stride is below 4 KiB or at
 * least 4 MiB first -- on MI355X a wave-wide load whose lane groups lie 4 KiB
 * to 2 MiB apart streams up to a third slower.  Either order gives the same
 * result.  page_cap > 0: among tile bits the schedule could take equally, the
 * compiler takes bits at byte strides of 2 MiB or more first while a tile has
 * fewer than page_cap of them (0 = no preference, -1 = the default: 4 for FP64,
 * 0 for FP32) -- a tile whose amplitudes span many 2 MiB pages misses the
 * per-CU address translation cache on most loads, so these bits are best spread
 * over the passes.  Re-compiles the schedule and drops captured graphs.
 * Defaults: 2^13-amplitude tiles (FP64 and FP32), 4 carriers, fusion on,
 * lane_order 1, page_cap -1.  PK_EINVAL when out of range (page_cap -1..16).
 */
int pk_set_tiling(pk_plan* plan, int32_t tile_bits, int32_t carrier_bits, int32_t fuse, int32_t lane_order,
                  int32_t page_cap);

/*
 * pk_set_launch -- launch shape of the pass kernels: wgs_per_cu resident
 * workgroups per CU (1..8, or 0 for as many as the kernel's resources allow,
 * the default; more than fit only queue up), and reg_bits = 3, 4 or 5 register
 * bits per thread in forward passes (8, 16 or 32 amplitudes per thread, a
 * workgroup of 2^(tile_bits - reg_bits) threads, at most 1024; 0 selects the
 * default: 4 for FP64, 5 for FP32).  With 3, a stage holds one two-qubit pair
 * and pk_evaluate_batched returns PK_EUNSUPPORTED.  Backward passes always use
 * 4.  Changing reg_bits re-compiles the schedule.  Drops captured graphs.
 * PK_EINVAL when out of range.
 */
int pk_set_launch(pk_plan* plan, int32_t wgs_per_cu, int32_t reg_bits);

/*
 * pk_set_pass_walk -- the order in which a single-instance plan's passes hand
 * tiles to workgroups: one entry per forward pass (n = pk_plan_passes), or one
 * per forward pass followed by one per backward pass (pk_backward); n = 0
 * resets every pass to 0.  Over a grid of G workgroups,
 * workgroup w takes: 0, tiles w, w + G, ... (the default: the workgroups
 * resident at once cover neighbouring tiles); c in 2..65536, runs of c
 * consecutive tiles starting at tiles w c, (w + G) c, ...; -1, one contiguous
 * block of ceil(ntiles / G) tiles.  Results do not change; which walk is faster
 * depends on the pass's tile bits and is measured
 * (paper_0902_0699_amd.autotune.tune_walk).  Reset by pk_set_tiling and by a
 * register-bit change in pk_set_launch.  Drops captured graphs.  PK_EINVAL for a
 * batched plan, a wrong n or an entry out of range.
 */
int pk_set_pass_walk(pk_plan* plan, int32_t n, const int32_t* walk);

/*
 * pk_set_pass_overlap -- how a single-instance plan's forward passes pipeline
 * HBM and LDS: one entry per forward pass (n = pk_plan_passes) or n = 0 to reset
 * every pass to 0.  1: the pass keeps the next tile's loads in flight through
 * all of the current tile's LDS exchanges (the tile loop that issues the same
 * loads on every path, so that only the current tile's loads are waited for);
 * 0: they are waited for at the first exchange.  It applies to the FP64 kernels
 * with 4 register bits and to passes whose tiles fill the workgroup; elsewhere
 * it is accepted and changes nothing.  Results do not change; which setting is
 * faster depends on the pass and is measured
 * (paper_0902_0699_amd.autotune.tune_walk).  Reset by pk_set_tiling and by a
 * register-bit change in pk_set_launch.  Drops captured graphs.  PK_EINVAL for a
 * batched plan, a wrong n or an entry other than 0 or 1.
 */
int pk_set_pass_overlap(pk_plan* plan, int32_t n, const int32_t* on);

/*
 * pk_set_lane_maps -- on = 1 (the default): a stage layout that moves through LDS
 * only (neither a pass's first nor its last) gets a thread-to-label map whose low
 * thread bits sit on local bits of distinct residue modulo the LDS slot swizzle's
 * group width, so that the lanes of one LDS access cycle hit distinct banks; on =
 * 0: every layout takes the thread bits in ascending order.  Results do not
 * change (each amplitude meets the same arithmetic in either map).  Re-compiles
 * the schedule and drops captured graphs.  PK_EINVAL when on is not 0 or 1.
 */
int pk_set_lane_maps(pk_plan* plan, int32_t on);

/*
 * pk_set_batch -- shape of pk_evaluate_batched's persistent launch (Sec. 6.2:
 * independent multiverses).  Workgroups that share an XCD, and so an L2, form
 * teams of team_size; each team runs the passes of its large instances
 * together, with a device-scope barrier between passes, so that an instance
 * too large for one workgroup is spread over many CUs.  An instance is large
 * when its first pass has at least min_team_tiles * team_size tiles.  Every
 * other instance is taken whole by one workgroup from a queue, largest first.
 * team_size 0 turns teams off.  Defaults 16 and 64 (instances of 2^22 or more
 * amplitudes at the default tile: below that a single workgroup's sweep costs
 * less than the barriers' device-scope fences).  A team barrier that has not
 * completed within about half a second (the launch's workgroups are not all
 * resident, e.g. the GPU is shared) gives up: that instance's L_out and
 * norm_out entries are NaN.  Drops the plan's device tables and graphs.
 * PK_EINVAL when out of range (team_size 0..64, min_team_tiles 1..4096).
 */
int pk_set_batch(pk_plan* plan, int32_t team_size, int32_t min_team_tiles);

/*
 * pk_batch_teams -- the team split pk_evaluate_batched uses on the current
 * device: number of teams and of instances run by teams.  Uploads the plan's
 * tables to the current device if needed (no kernel runs).
 */
int pk_batch_teams(pk_plan* plan, int32_t* n_teams, int32_t* n_team_instances);

/* Number of passes (full sweeps over the state) one evaluation of instance `inst` makes. */
int pk_plan_passes(const pk_plan* plan, int32_t inst, int32_t* passes);

/*
 * pk_plan_describe -- JSON text of the compiled schedule (passes, tile bits,
 * stages and their gate lists).  Writes at most `cap` bytes including the NUL;
 * *needed receives the full size.  Host-only; for tests and tools.
 */
int pk_plan_describe(const pk_plan* plan, char* buf, int64_t cap, int64_t* needed);

/* Element offsets of each instance in a packed state buffer: offsets[n_inst + 1],
 * offsets[i] = sum_{j<i} 2^nq_j; states of a batch lie back to back in that order. */
int pk_plan_offsets(const pk_plan* plan, int64_t* offsets);

/* Number of rotation gates (D2 and D4) over all instances (instance order, then
 * gate order); the angle arrays below hold 3 doubles (alpha, beta, gamma) per
 * rotation gate in that order. */
int pk_plan_n_angles(const pk_plan* plan, int64_t* n_d2);

/*
 * pk_workspace_bytes -- device workspace that op (PK_OP_EVAL or PK_OP_BACKWARD)
 * needs.  EVAL needs small tables and partial sums; BACKWARD in addition one
 * state-sized buffer for the recomputed state.  Contents need not be initialised.
 */
int pk_workspace_bytes(const pk_plan* plan, int32_t op, int64_t* bytes);

/*
 * pk_evaluate -- apply the gate list of a single-instance plan (n_inst == 1).
 *   psi_in   device, 2^nq complex, read; may equal psi_out (in place, as the paper's psi)
 *   psi_out  device, 2^nq complex, written
 *   L_out    device double[1]: L = sum_{x in M} |C~_x|^2 (FP64 final combine)
 *   norm_out device double[1] or NULL: sum_n |C~_n|^2 (diagnostic)
 *   angles   device double[3 * n_rot] or NULL (n_rot = D2 and D4 gates; NULL = the
 *            angles given to pk_create)
 *   workspace device, >= pk_workspace_bytes(PK_OP_EVAL)
 * The launches are captured once into a hipGraph per pointer set and replayed.
 * Errors: PK_EINVAL (NULL/misaligned pointer, batched plan), PK_EDEVICE.
 */
int pk_evaluate(pk_plan* plan, const void* psi_in, void* psi_out, double* L_out, double* norm_out,
                const double* angles, void* workspace, void* stream);

/*
 * pk_evaluate_static -- pk_evaluate for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same kernels as pk_evaluate, but their workspace is a
 * static device buffer of the library, PK_STATIC_WORKSPACE_BYTES per GPU (held
 * by each GPU the library runs on until the process ends), and the launches go
 * to `stream` directly: the call allocates nothing and builds no graph.
 * Arguments as pk_evaluate, without `workspace`; the caller still owns
 * psi_in, psi_out, L_out and norm_out.
 * Set-up: the plan's tables must already be on the current device (any earlier
 * pk_evaluate or pk_batch_teams with that device current uploads them);
 * otherwise PK_EINVAL.  PK_EINVAL too when the plan's workspace
 * (pk_workspace_bytes(PK_OP_EVAL)) exceeds PK_STATIC_WORKSPACE_BYTES.
 * Every call on one GPU shares that GPU's buffer, which keeps the last call's
 * contents: calls that overlap on one GPU (other streams, other threads) race
 * and give wrong results; order them on one stream.  Nothing in the buffer needs
 * to start at zero.
 */
#define PK_STATIC_WORKSPACE_BYTES (8 << 20)
int pk_evaluate_static(pk_plan* plan, const void* psi_in, void* psi_out, double* L_out, double* norm_out,
                       const double* angles, void* stream);

/*
 * pk_evaluate_repeat -- apply the gate list of a single-instance plan `reps`
 * times in a row: psi_out = U^reps psi_in.  With the list of one Grover
 * iteration G = HALL . Inv . HALL . Oracle this is the whole search of Sec. 5.1,
 * G^{n_t} with n_t = floor((pi/4) sqrt(2^nq)) iterations.  For a plan without
 * angle parameters, 8 consecutive applications are scheduled as one gate list,
 * so that a pass can end one application and begin the next (a Grover iteration
 * at n_q = 20 takes 3 passes alone, 8 take 17); reps mod 8 applications run
 * alone, first.  The whole sequence of passes, one launch each, is captured into
 * one hipGraph, keyed by the pointers and reps, and replayed.  With the environment
 * variable PK_REPEAT_PERSISTENT=1 (and reps > 1, every pass on one kernel
 * instance) the passes run instead in one persistent launch of as many
 * workgroups as the GPU holds at once, with a grid-wide barrier between passes;
 * same results bit for bit, but on MI355X the barrier's device-scope fences cost
 * more than the kernel boundaries.  If its workgroups cannot all be resident (the
 * GPU is shared), a barrier gives up after about half a second and L_out and
 * norm_out are NaN.  L_out and norm_out refer to the final state.
 *   reps  1..2^24, with at most 2^20 passes in total
 * Other arguments and errors as pk_evaluate.
 */
int pk_evaluate_repeat(pk_plan* plan, int64_t reps, const void* psi_in, void* psi_out, double* L_out,
                       double* norm_out, const double* angles, void* workspace, void* stream);

/*
 * pk_repeat_launches -- the number of pass launches pk_evaluate_repeat(plan,
 * reps, ...) runs in its graph form (after the fusing described there).
 * Host-side only (the fused schedule is compiled, not uploaded).  Single-instance
 * plans; reps 1..2^24.  PK_EINVAL otherwise.
 */
int pk_repeat_launches(pk_plan* plan, int64_t reps, int64_t* launches);

/*
 * pk_search_diffusion -- a labelled variant of the noise-free search, not the
 * paper's HALL-based form: `iterations` applications of
 *     G = HALL . Inv . HALL . Oracle = (2|s><s| - I) . Oracle      (Sec. 5.1)
 * computed through that identity (Inv = 2|0><0| - I, HALL|0..0> = |s>), i.e.
 * C_n <- 2 mean(O C) - (O C)_n with O the Oracle's sign flips: one streaming pass
 * per iteration instead of the HALL sweeps.  Exact in exact arithmetic; it
 * applies only to the noise-free iteration (a noise rotation between the HALLs
 * breaks the identity).
 *   nq          1..30 (PK_FP64) or 1..31 (PK_FP32); prec as for plans
 *   marked      host int64[n_marked], distinct labels in [0, 2^nq), 0 <= n_marked <= 64
 *   iterations  >= 1 (the search: n_t = floor((pi/4) sqrt(2^nq)))
 *   psi_in      device, 2^nq complex, read; may equal psi_out
 *   psi_out     device, 2^nq complex, written
 *   L_out       device double[1]: sum_{x in M} |C_x|^2 of the final state
 *   workspace   device, >= pk_search_workspace_bytes() (FP64 partial sums and the mean)
 * Means are FP64 sums in a fixed order.  Not captured into a graph: 2 launches
 * per iteration go to `stream` directly.  PK_EINVAL on range or pointer errors.
 */
int pk_search_diffusion(int32_t nq, int32_t prec, const int64_t* marked, int32_t n_marked, int64_t iterations,
                        const void* psi_in, void* psi_out, double* L_out, void* workspace, void* stream);

/* Workspace pk_search_diffusion needs (bytes). */
int pk_search_workspace_bytes(int64_t* bytes);

/*
 * pk_evaluate_batched -- evaluate every instance of the plan ("multiverses",
 * Sec. 6.2) in one persistent launch replayed from a hipGraph.  States are
 * packed at pk_plan_offsets(); L_out and norm_out (or NULL) hold n_inst doubles.
 * Other arguments as pk_evaluate.
 */
int pk_evaluate_batched(pk_plan* plan, const void* psi_in, void* psi_out, double* L_out,
                        double* norm_out, const double* angles, void* workspace, void* stream);

/*
 * pk_backward -- gradient of sum_i dL[i] * L_i by the adjoint method with
 * recomputation: starting from psi_out (as produced by pk_evaluate with the same
 * angles) the state is walked back through the adjoint gates while
 * lambda = dL * P_M psi_out is propagated alongside; no intermediate state is stored.
 *   psi_out     device, read
 *   dL          device double[n_inst]
 *   grad_psi_in device complex, written: Re = dL/dRe psi_in, Im = dL/dIm psi_in
 *   grad_angles device double[3 * n_rot] or NULL, written (d/dalpha, d/dbeta, d/dgamma
 *               per D2 or D4 gate)
 *   angles      device double[3 * n_rot] or NULL, as for pk_evaluate
 *   workspace   device, >= pk_workspace_bytes(PK_OP_BACKWARD)
 * Single-instance plans only.  PK_EUNSUPPORTED when a ONEOP or TWOOP gate is
 * not unitary (its inverse is then not its adjoint and the state cannot be
 * walked back).
 */
int pk_backward(pk_plan* plan, const void* psi_out, const double* dL, void* grad_psi_in,
                double* grad_angles, const double* angles, void* workspace, void* stream);

/*
 * pk_pair_indices -- the partner pairs of qubit i_s (Sec. 2.2, Eqs. pair0/pair1):
 * for r = first .. first+count-1, n0[r] is the r-th label (ascending) whose qubit
 * i_s is 0 and n1[r] = n0[r] + 2^(nq - i_s).  Written to device arrays by a
 * kernel using the library's index arithmetic.  PK_EINVAL when nq is outside
 * 1..31, i_s outside 1..nq or the range exceeds 2^nq / 2 pairs.
 */
int pk_pair_indices(int32_t nq, int32_t i_s, int64_t first, int64_t count, int64_t* n0,
                    int64_t* n1, void* stream);

/*
 * pk_shor_state -- the loaded two-register state of Shor's algorithm (Sec. 5.2,
 * Step 3, Eq. Shor2): register one (n1 qubits, qubits 1..n1, the high bits)
 * holds every n < 2^n1 with equal weight and register two (n2 qubits, the low
 * bits) holds f(n) = xguess^n mod M:
 *     psi[n * 2^n2 + f(n)] = 2^(-n1/2),  every other amplitude 0.
 *   n1, n2   register sizes: n1, n2 >= 1, n1 + n2 <= 30 (PK_FP64) or 31 (PK_FP32)
 *   xguess   1 .. M-1 (Step 3 takes it coprime to M; not checked)
 *   M        2 <= M <= 2^n2, M < 2^31
 *   psi      device, 2^(n1+n2) complex of `prec`, written entirely (16-byte aligned)
 * f is exact (64-bit integer arithmetic); the amplitude is the correctly rounded
 * 2^(-n1/2) (FP32: that double rounded to float).  PK_EINVAL on any range error.
 * Errors are reported through pk_last_error(NULL).
 */
int pk_shor_state(int32_t n1, int32_t n2, int64_t xguess, int64_t M, int32_t prec, void* psi, void* stream);

/*
 * pk_marginal -- the distribution of a measurement of the high nq - n_low qubits
 * (Shor's register one, Step 6):
 *     p[n] = sum_{k < 2^n_low} |psi[n * 2^n_low + k]|^2,  n < 2^(nq - n_low).
 *   psi  device, 2^nq complex of `prec`, read (16-byte aligned)
 *   p    device double[2^(nq - n_low)], written (8-byte aligned)
 * FP64 sums (FP32 amplitudes are widened first) in an order fixed by n_low, so
 * results are reproducible.  One read of the state; with fewer than ~1000
 * segments of 2^14 or more amplitudes the launch cannot fill the GPU.
 * PK_EINVAL for nq out of range, n_low outside 0..nq, NULL or misaligned pointers.
 */
int pk_marginal(int32_t nq, int32_t n_low, int32_t prec, const void* psi, double* p, void* stream);

/*
 * pk_marginal_bitrev -- pk_marginal with the high register read in reversed qubit
 * order: p[rev(n)] = sum_{k < 2^n_low} |psi[n * 2^n_low + k]|^2, rev reversing the
 * nq - n_low bits of n.  After PK_GATE_QFT_NOSWAP on the high register this is the
 * distribution that pk_marginal gives after PK_GATE_QFT (Step 6 of Sec. 5.2) with
 * one pass fewer.  Same sums, order, arguments and errors as pk_marginal.
 */
int pk_marginal_bitrev(int32_t nq, int32_t n_low, int32_t prec, const void* psi, double* p, void* stream);

/*
 * pk_density_matrix -- the ensemble density matrix of Sec. 6.1:
 *     <n|rho|n'> = sum_a P_a C_a(n) C_a^*(n'),  n, n' < N = 2^nq,
 * over n_univ universes ("multiverses", Sec. 6.2) of the same size.
 *   nq       1..16 (rho takes N^2 * 16 bytes: 64 GiB at nq = 16)
 *   n_univ   >= 1
 *   states   device complex128, n_univ * N, universe after universe (the packed
 *            layout of pk_evaluate_batched for equal sizes), 16-byte aligned
 *   weights  device double[n_univ]: P_a (not normalised by the call)
 *   rho      device complex128[N * N], row-major rho[n * N + n'], written entirely
 * FP64 throughout, on the matrix cores.  rho is Hermitian by construction: each
 * element below the diagonal is computed once and written with its conjugate
 * above; diagonal elements are real.  PK_EINVAL on range or pointer errors.
 * Errors are reported through pk_last_error(NULL).
 */
int pk_density_matrix(int32_t nq, int32_t n_univ, const void* states, const double* weights, void* rho,
                      void* stream);

/*
 * pk_density_spectrum -- eigenvalues of a Hermitian rho (as written by
 * pk_density_matrix) and two sums over them (Sec. 6.1):
 *     sums[0] = S = -sum_{lambda > 0} lambda log2 lambda  (entropy in bits; the
 *               paper leaves the base open; eigenvalues <= 0 from rounding add 0)
 *     sums[1] = Tr rho^2 = sum lambda^2                   (purity)
 *   nq           1..15
 *   rho          device complex128[N * N]; only its lower triangle is read, and it
 *                is overwritten (used as the solver's workspace)
 *   eigenvalues  device double[N], ascending
 *   sums         device double[2]
 * The eigenvalues come from rocSOLVER (zheevd, no eigenvectors).  The call waits
 * for the stream to finish (to read the solver's convergence flag).  PK_EDEVICE
 * when the solver fails or does not converge.
 */
int pk_density_spectrum(int32_t nq, void* rho, double* eigenvalues, double* sums, void* stream);

/*
 * pk_time_passes -- measurement helper: runs one evaluation of a single-instance
 * plan pass by pass with HIP events around every kernel on `stream`, waits for
 * it, and writes the duration of each launch in milliseconds to ms[max_n]
 * (the count written goes to *n).  Arguments as pk_evaluate.
 */
int pk_time_passes(pk_plan* plan, const void* psi_in, void* psi_out, double* L_out,
                   const double* angles, void* workspace, void* stream, double* ms, int32_t max_n,
                   int32_t* n);

/* Frees plan-owned host and device tables and graphs.  NULL is a no-op. */
void pk_destroy(pk_plan* plan);

/* Static text for a return code. */
const char* pk_strerror(int code);

/* Text of the last error recorded on `plan` ("" when none); NULL plan gives the
 * last error of pk_create/pk_pair_indices on this thread. */
const char* pk_last_error(const pk_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* PAPERKERN_H */
