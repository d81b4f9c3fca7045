// Host-side launchers of the device kernels (defined in pk_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pk_desc.h"

namespace pk {

struct PassLaunch {
    const Pass* passes;
    const Stage* stages;
    const Flip* flips;
    const PhaseOp* phases;
    const double* twid;  // product tables of the controlled phases (re, im pairs)
    const URef* urefs;   // tile-part tables of each pass
    const double* mats;
    const double* mats4;
    const void* src0;
    void* dst0;
    void* dst1;
    double* partials;
    double* reads;
    double* gpart;
    const double* dL;
    int32_t pass;
    int32_t want_norm;
    int32_t kmax;
    int32_t nv;
    int32_t fp64;
    int32_t rbits;     // register bits per thread (4 or 5)
    int64_t ntiles;
    int64_t grid_cap;  // workgroups per CU of a pass launch; 0 = as many as fit
};

// Device arguments of the batched launch (see batched_kernel).
struct BatchArgs {
    const InstDesc* idesc;
    const int32_t* order;      // queue order: instances taken whole by one workgroup
    const int32_t* team_off;   // n_teams + 1 offsets into team_list
    const int32_t* team_list;  // large instances of each team
    unsigned int* queue;       // next queue position (cleared before the launch)
    unsigned int* bars;        // one barrier counter per team (cleared before the launch)
    double* L_out;
    double* norm_out;
    uint64_t spin_ticks;       // bound of one team barrier wait, in wall-clock ticks
    int32_t n_solo;
    int32_t n_teams;
    int32_t team_size;
    int32_t n_xcd;
};

// Device arguments of the persistent repeat launch (see repeat_kernel).
struct RepeatArgs {
    unsigned int* bar;     // grid barrier counter (cleared before the launch)
    int64_t reps;          // applications of the gate list
    int32_t pass0;         // first pass of the instance in the pass table
    int32_t npass;         // passes per application
    uint64_t spin_ticks;   // bound of one barrier wait, in wall-clock ticks
    int32_t n_reads;       // readout slots (set to NaN when a barrier timed out)
    int32_t pad;
    int64_t part_base;     // norm partials of the last pass (likewise)
    int64_t n_part;
};

hipError_t launch_pass(const PassLaunch& L, hipStream_t st);
// G^reps of a single-instance plan in one persistent launch of `grid` resident
// workgroups (L.kmax, L.rbits, L.fp64 select the kernel instance).
hipError_t launch_repeat(const PassLaunch& L, const RepeatArgs& r, unsigned grid, hipStream_t st);
// Resident workgroups per CU of that instance (0 if unknown).
int repeat_blocks_per_cu(int kmax, int rbits, bool fp64);
hipError_t launch_batched(const PassLaunch& L, const BatchArgs& B, unsigned grid, hipStream_t st);
// Resident workgroups per CU of the batched kernel instance (0 if unknown).
int batched_blocks_per_cu(int kmax, int rbits, bool fp64);
// Workspace matrices for one launch: the static 2x2 and 4x4 operators are
// copied, then each rotation's five matrices are built after them
// (D2: 40 doubles at mats + n_smats + 40 * slot; D4: 160 doubles at
// mats4 + n_smats4 + 160 * slot); n_counters launch counters are cleared.
struct PrepArgs {
    double* mats;
    const double* smats;
    int32_t n_smats;  // doubles
    double* mats4;
    const double* smats4;
    int32_t n_smats4;  // doubles
    const double* angles;
    const ParamRef* params;
    int32_t n_params;
    unsigned int* counters;
    int32_t n_counters;
};

hipError_t launch_prep(const PrepArgs& p, hipStream_t st);
hipError_t launch_reduce(const Reduction* red, int n, const double* ws, double* L_out, double* norm_out,
                         double* grad_out, hipStream_t st);
hipError_t launch_pairs(int nq, int i_s, int64_t first, int64_t count, int64_t* n0, int64_t* n1,
                        hipStream_t st);
// Shor's data path (pk_shor.hip): the loaded state of Eq. Shor2 and the marginal
// over the n_low low qubits.
hipError_t launch_shor_state(int n1, int n2, uint64_t x, uint64_t M, bool fp64, double amp, void* psi,
                             hipStream_t st);
hipError_t launch_marginal(int nq, int n_low, bool fp64, bool bitrev, const void* psi, double* p, hipStream_t st);
// The ensemble density matrix (pk_density.hip): rho = sum_a P_a C_a C_a^H for A
// universe states of N amplitudes (rows of C), and the entropy / purity sums of
// a spectrum.
int64_t density_blocks(int64_t N);
hipError_t launch_density(const void* C, const double* P, void* rho, int64_t N, int A, hipStream_t st);
hipError_t launch_spectrum_sums(const double* lam, int64_t n, double* out, hipStream_t st);
// The noise-free Grover search by the diffusion identity (pk_search.hip).
struct MarkedSet {
    int32_t count;
    int32_t pad;
    int64_t label[64];
};
size_t search_workspace_bytes();
hipError_t launch_search(const void* psi_in, void* psi_out, int nq, bool fp64, const MarkedSet& ms, int64_t iters,
                         void* workspace, double* L, hipStream_t st);

}  // namespace pk
