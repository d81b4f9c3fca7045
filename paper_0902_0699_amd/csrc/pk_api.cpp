// The C-ABI of libpaperkern: argument checks, device tables, graph capture.
#include <hip/hip_runtime.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "paperkern.h"
#include "pk_launch.h"
#include "pk_plan.h"

using namespace pk;

namespace {

thread_local std::string g_error;

enum GraphSlot { G_EVAL = 0, G_BATCH = 1, G_BWD = 2, G_REPEAT = 3, G_SLOTS = 4 };

struct DevPlan {
    Plan host;
    void* exec[G_SLOTS] = {nullptr, nullptr, nullptr, nullptr};
    const void* key[G_SLOTS][8] = {};
    hipStream_t cap = nullptr;
    int n_cu = 0;
    unsigned batch_grid = 0;  // persistent grid of the batched launch
    uint64_t spin_ticks = 0;  // half a second of the device wall clock
    DevPlan* fused = nullptr; // pk_evaluate_repeat: kRepeatFuse applications as one schedule
};

// pk_evaluate_repeat schedules this many consecutive applications of the gate list
// as one gate list: a pass can then finish one application and start the next
// (at n_q = 20 a Grover iteration takes 3 passes alone, 8 take 17).
constexpr int64_t kRepeatFuse = 8;

// MI355X has 8 XCDs and dispatches workgroups round-robin over them; the count
// only shapes the batched teams (which workgroups share an L2), not results.
constexpr int kXcds = 8;

int batched_kmax(const Plan& P) {
    int km = P.inst[0].fwd[0].rbits + 6;
    for (const auto& in : P.inst)
        for (const auto& hp : in.fwd) km = hp.kmax > km ? hp.kmax : km;
    return km;
}

DevPlan* dp(pk_plan* p) { return reinterpret_cast<DevPlan*>(p); }
const DevPlan* dp(const pk_plan* p) { return reinterpret_cast<const DevPlan*>(p); }

int fail(DevPlan* d, int code, const std::string& msg) {
    if (d)
        d->host.last_error = msg;
    else
        g_error = msg;
    return code;
}

int hip_fail(DevPlan* d, hipError_t e, const char* where) {
    return fail(d, PK_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

bool valid(const pk_plan* p) { return p && dp(p)->host.magic == 0x504b504cu; }

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

void drop_device(DevPlan* d);

// Captured graphs, and the fused repeat schedule (it copies the plan's settings).
void drop_graphs(DevPlan* d) {
    for (int s = 0; s < G_SLOTS; ++s) {
        if (d->exec[s]) hipGraphExecDestroy(reinterpret_cast<hipGraphExec_t>(d->exec[s]));
        d->exec[s] = nullptr;
        std::memset(d->key[s], 0, sizeof d->key[s]);
    }
    if (d->fused) {
        drop_device(d->fused);
        if (d->fused->cap) hipStreamDestroy(d->fused->cap);
        delete d->fused;
        d->fused = nullptr;
    }
}

void drop_device(DevPlan* d) {
    drop_graphs(d);
    if (d->host.d_tables) hipFree(d->host.d_tables);
    d->host.d_tables = nullptr;
    d->host.device = -1;
}

template <typename T>
void put(std::vector<char>& buf, size_t off, const std::vector<T>& v) {
    if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(T));
}

int ensure_device(DevPlan* d) {
    Plan& P = d->host;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(d, e, "hipGetDevice");
    if (P.d_tables) {
        if (dev != P.device) return fail(d, PK_EINVAL, "plan was first used on another device");
        return PK_OK;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) d->n_cu = prop.multiProcessorCount;
    if (d->n_cu <= 0) d->n_cu = 256;
    int wall_khz = 0;
    if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wall_khz <= 0)
        wall_khz = 100000;
    // bound of one barrier wait: 0.5 s, or PK_BARRIER_SPIN_US microseconds (tests
    // force the time-out path with a tiny value)
    uint64_t spin_us = 500000;
    if (const char* v = std::getenv("PK_BARRIER_SPIN_US")) spin_us = std::strtoull(v, nullptr, 10);
    d->spin_ticks = (uint64_t)wall_khz * spin_us / 1000;
    // batched launch: as many workgroups as are resident at once, in teams
    int per_cu = batched_blocks_per_cu(batched_kmax(P), P.inst[0].fwd[0].rbits, P.prec == PK_FP64);
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 8) per_cu = 8;
    d->batch_grid = (unsigned)(d->n_cu * per_cu);
    P.team = team_schedule(&P, d->batch_grid, d->n_cu % kXcds == 0 ? kXcds : 1);

    TableLayout t = table_layout(&P);
    std::vector<char> buf(t.total, 0);
    put(buf, t.passes, P.passes);
    put(buf, t.stages, P.stages);
    put(buf, t.flips, P.flips);
    put(buf, t.phases, P.phases);
    put(buf, t.twid, P.twid);
    put(buf, t.urefs, P.urefs);
    put(buf, t.mats, P.static_mats);
    put(buf, t.mats + P.static_mats.size() * sizeof(double), P.default_angles);
    put(buf, t.mats4, P.static_mats4);
    put(buf, t.params, P.params);
    put(buf, t.idesc, P.idesc);
    put(buf, t.order, P.team.solo);
    put(buf, t.team_off, P.team.team_off);
    put(buf, t.team_list, P.team.team_list);
    std::vector<Reduction> r = eval_reductions(&P);
    std::vector<Reduction> rb = backward_reductions(&P);
    r.insert(r.end(), rb.begin(), rb.end());
    put(buf, t.red, r);
    void* ptr = nullptr;
    e = hipMalloc(&ptr, t.total);
    if (e != hipSuccess) return hip_fail(d, e, "hipMalloc(plan tables)");
    e = hipMemcpy(ptr, buf.data(), t.total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(ptr);
        return hip_fail(d, e, "hipMemcpy(plan tables)");
    }
    P.d_tables = ptr;
    P.d_tables_bytes = t.total;
    P.device = dev;
    if (!d->cap) {
        e = hipStreamCreateWithFlags(&d->cap, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(d, e, "hipStreamCreate");
    }
    return PK_OK;
}

template <typename T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off);
}

struct EvalArgs {
    const void* psi_in;
    void* psi_out;
    double* L_out;
    double* norm_out;
    const double* angles;
    void* ws;
};

PassLaunch base_launch(DevPlan* d, void* ws, int op) {
    Plan& P = d->host;
    TableLayout t = table_layout(&P);
    WsLayout w = workspace_layout(&P, op);
    PassLaunch L{};
    L.passes = at<Pass>(P.d_tables, t.passes);
    L.stages = at<Stage>(P.d_tables, t.stages);
    L.flips = at<Flip>(P.d_tables, t.flips);
    L.phases = at<PhaseOp>(P.d_tables, t.phases);
    L.twid = at<double>(P.d_tables, t.twid);
    L.urefs = at<URef>(P.d_tables, t.urefs);
    L.mats = at<double>(ws, w.mats);
    L.mats4 = at<double>(ws, w.mats4);
    L.partials = at<double>(ws, w.partials);
    L.reads = at<double>(ws, w.reads);
    L.gpart = at<double>(ws, w.gpart);
    L.fp64 = P.prec == PK_FP64;
    return L;
}

const double* angle_src(DevPlan* d, const double* angles) {
    if (angles) return angles;
    TableLayout t = table_layout(&d->host);
    return at<double>(d->host.d_tables, t.mats + d->host.static_mats.size() * sizeof(double));
}

hipError_t enqueue_prep(DevPlan* d, void* ws, const double* angles, int op, int n_counters, hipStream_t st) {
    Plan& P = d->host;
    TableLayout t = table_layout(&P);
    WsLayout w = workspace_layout(&P, op);
    PrepArgs p{};
    p.mats = at<double>(ws, w.mats);
    p.smats = at<double>(P.d_tables, t.mats);
    p.n_smats = (int32_t)P.static_mats.size();
    p.mats4 = at<double>(ws, w.mats4);
    p.smats4 = at<double>(P.d_tables, t.mats4);
    p.n_smats4 = (int32_t)P.static_mats4.size();
    p.angles = angle_src(d, angles);
    p.params = at<ParamRef>(P.d_tables, t.params);
    p.n_params = (int32_t)P.params.size();
    p.counters = at<unsigned int>(ws, w.counters);
    p.n_counters = n_counters;
    return launch_prep(p, st);
}

// Evaluation of a single-instance plan: prep, every forward pass, final combine.
// One evaluation, or `reps` applications of the gate list in a row: the first
// reads psi_in, every later one works on psi_out in place; the matrices are
// built once, and the norm partials are written by the last application only.
hipError_t enqueue_eval(DevPlan* d, const EvalArgs& a, hipStream_t st, std::vector<hipEvent_t>* ev,
                        int64_t reps = 1) {
    Plan& P = d->host;
    hipError_t e = enqueue_prep(d, a.ws, a.angles, PK_OP_EVAL, 0, st);
    if (e != hipSuccess) return e;
    PassLaunch L = base_launch(d, a.ws, PK_OP_EVAL);
    L.dst0 = a.psi_out;
    L.nv = 1;
    const Instance& in = P.inst[0];
    for (int64_t r = 0; r < reps; ++r) {
        L.src0 = r == 0 ? a.psi_in : a.psi_out;
        L.want_norm = a.norm_out != nullptr && r == reps - 1;
        for (size_t p = 0; p < in.fwd.size(); ++p) {
            L.pass = (int)p;
            L.kmax = in.fwd[p].kmax;
            L.ntiles = in.fwd[p].ntiles;
            L.grid_cap = P.tiling.wgs_per_cu;
            L.rbits = in.fwd[p].rbits;
            if (ev) hipEventRecord((*ev)[2 * p], st);
            e = launch_pass(L, st);
            if (ev) hipEventRecord((*ev)[2 * p + 1], st);
            if (e != hipSuccess) return e;
        }
    }
    TableLayout t = table_layout(&P);
    return launch_reduce(at<Reduction>(P.d_tables, t.red), 2 * (int)P.inst.size(), static_cast<double*>(a.ws),
                         a.L_out, a.norm_out, nullptr, st);
}

// The gate list applied kRepeatFuse times, compiled as one plan with the same
// settings, or nullptr where that does not apply: a plan with angle parameters
// (each application would need its own), or one whose fused schedule would not use
// the same workspace layout.  Built on first use and kept until the plan's
// settings change.
DevPlan* fused_plan(DevPlan* d) {
    if (d->fused) return d->fused;
    const Plan& P = d->host;
    if (P.inst.size() != 1 || !P.params.empty()) return nullptr;
    DevPlan* f = new (std::nothrow) DevPlan();
    if (!f) return nullptr;
    f->host = P;
    f->host.d_tables = nullptr;
    f->host.d_tables_bytes = 0;
    f->host.device = -1;
    f->host.walk.clear();
    f->host.overlap.clear();
    std::vector<Prim>& prims = f->host.inst[0].prims;
    const std::vector<Prim> one = prims;
    for (int64_t r = 1; r < kRepeatFuse; ++r) prims.insert(prims.end(), one.begin(), one.end());
    std::string err;
    int rc;
    try {
        rc = recompile(&f->host, &err);
    } catch (...) {
        rc = PK_EINVAL;
    }
    bool same = false;
    if (rc == PK_OK) {
        const WsLayout wa = workspace_layout(&P, PK_OP_EVAL), wb = workspace_layout(&f->host, PK_OP_EVAL);
        same = wa.mats == wb.mats && wa.mats4 == wb.mats4 && wa.partials == wb.partials && wa.reads == wb.reads &&
               wa.counters == wb.counters && wa.total == wb.total && f->host.n_partials == P.n_partials &&
               f->host.n_reads == P.n_reads;
    }
    if (!same || f->host.inst[0].fwd.size() >= (size_t)kRepeatFuse * P.inst[0].fwd.size()) {
        delete f;
        return nullptr;
    }
    d->fused = f;
    return f;
}

// How pk_evaluate_repeat splits reps: `single` applications of the plan, then
// `rounds` of the fused schedule (none when it does not apply).
struct RepeatSplit {
    DevPlan* fused;
    int64_t single, rounds;
};

RepeatSplit repeat_split(DevPlan* d, int64_t reps) {
    DevPlan* f = reps >= kRepeatFuse ? fused_plan(d) : nullptr;
    if (!f) return {nullptr, reps, 0};
    return {f, reps % kRepeatFuse, reps / kRepeatFuse};
}

// The passes of one application of `src`'s forward schedule.
hipError_t enqueue_passes(DevPlan* src, void* ws, const void* in, void* out, bool want_norm, hipStream_t st) {
    Plan& P = src->host;
    PassLaunch L = base_launch(src, ws, PK_OP_EVAL);
    L.src0 = in;
    L.dst0 = out;
    L.nv = 1;
    L.want_norm = want_norm;
    const Instance& inst = P.inst[0];
    for (size_t p = 0; p < inst.fwd.size(); ++p) {
        L.pass = (int)p;
        L.kmax = inst.fwd[p].kmax;
        L.ntiles = inst.fwd[p].ntiles;
        L.grid_cap = P.tiling.wgs_per_cu;
        L.rbits = inst.fwd[p].rbits;
        hipError_t e = launch_pass(L, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// pk_evaluate_repeat with the fused schedule: prep, the single applications, the
// fused rounds, then the final combine of the last one (same workspace layout).
hipError_t enqueue_repeat_fused(DevPlan* d, const RepeatSplit& sp, const EvalArgs& a, hipStream_t st) {
    hipError_t e = enqueue_prep(d, a.ws, a.angles, PK_OP_EVAL, 0, st);
    if (e != hipSuccess) return e;
    int64_t done = 0;
    for (int64_t r = 0; r < sp.single; ++r, ++done) {
        e = enqueue_passes(d, a.ws, done == 0 ? a.psi_in : a.psi_out, a.psi_out, false, st);
        if (e != hipSuccess) return e;
    }
    for (int64_t r = 0; r < sp.rounds; ++r, ++done) {
        e = enqueue_passes(sp.fused, a.ws, done == 0 ? a.psi_in : a.psi_out, a.psi_out,
                           a.norm_out != nullptr && r == sp.rounds - 1, st);
        if (e != hipSuccess) return e;
    }
    Plan& F = sp.fused->host;
    TableLayout t = table_layout(&F);
    return launch_reduce(at<Reduction>(F.d_tables, t.red), 2, static_cast<double*>(a.ws), a.L_out, a.norm_out,
                         nullptr, st);
}

// The persistent form of pk_evaluate_repeat is opt-in (PK_REPEAT_PERSISTENT=1): on
// MI355X its grid barrier (device-scope fences in every workgroup) costs more than
// the kernel boundary it replaces.
bool repeat_persistent() {
    const char* v = std::getenv("PK_REPEAT_PERSISTENT");
    return v && v[0] && v[0] != '0';
}

// G^reps in one persistent launch when every forward pass runs on the same kernel
// instance; 0 when the plan needs the launch-per-pass form.
unsigned repeat_grid(DevPlan* d) {
    const Instance& in = d->host.inst[0];
    const int kmax = in.fwd[0].kmax, rbits = in.fwd[0].rbits;
    if (rbits == 3) return 0;  // the persistent kernel has 4 and 5 register bits
    int64_t tiles = 0;
    for (const auto& hp : in.fwd) {
        if (hp.kmax != kmax || hp.rbits != rbits) return 0;
        tiles = std::max<int64_t>(tiles, hp.ntiles);
    }
    int per_cu = repeat_blocks_per_cu(kmax, rbits, d->host.prec == PK_FP64);
    if (per_cu < 1) return 0;
    const int64_t grid = std::min<int64_t>((int64_t)d->n_cu * per_cu, tiles);
    return (unsigned)std::max<int64_t>(grid, 1);
}

// prep (clears the barrier counter), the persistent launch, the final combine.
hipError_t enqueue_repeat(DevPlan* d, const EvalArgs& a, hipStream_t st, int64_t reps, unsigned grid) {
    Plan& P = d->host;
    hipError_t e = enqueue_prep(d, a.ws, a.angles, PK_OP_EVAL, 64, st);  // arrival counter and release word
    if (e != hipSuccess) return e;
    PassLaunch L = base_launch(d, a.ws, PK_OP_EVAL);
    const Instance& in = P.inst[0];
    L.src0 = a.psi_in;
    L.dst0 = a.psi_out;
    L.nv = 1;
    L.want_norm = a.norm_out != nullptr;
    L.kmax = in.fwd[0].kmax;
    L.rbits = in.fwd[0].rbits;
    WsLayout w = workspace_layout(&P, PK_OP_EVAL);
    RepeatArgs r{};
    r.bar = at<unsigned int>(a.ws, w.counters);
    r.reps = reps;
    r.pass0 = 0;
    r.npass = (int32_t)in.fwd.size();
    r.spin_ticks = d->spin_ticks;
    r.n_reads = P.n_reads;
    r.part_base = in.fwd.back().part_base;
    r.n_part = in.fwd.back().ntiles;
    e = launch_repeat(L, r, grid, st);
    if (e != hipSuccess) return e;
    TableLayout t = table_layout(&P);
    return launch_reduce(at<Reduction>(P.d_tables, t.red), 2 * (int)P.inst.size(), static_cast<double*>(a.ws),
                         a.L_out, a.norm_out, nullptr, st);
}

hipError_t enqueue_batched(DevPlan* d, const EvalArgs& a, hipStream_t st) {
    Plan& P = d->host;
    const TeamSchedule& ts = P.team;
    hipError_t e = enqueue_prep(d, a.ws, a.angles, PK_OP_EVAL, 2 + ts.n_teams, st);
    if (e != hipSuccess) return e;
    PassLaunch L = base_launch(d, a.ws, PK_OP_EVAL);
    L.src0 = a.psi_in;
    L.dst0 = a.psi_out;
    L.want_norm = a.norm_out != nullptr;
    L.nv = 1;
    L.kmax = batched_kmax(P);
    L.rbits = P.inst[0].fwd[0].rbits;
    TableLayout t = table_layout(&P);
    WsLayout w = workspace_layout(&P, PK_OP_EVAL);
    BatchArgs B{};
    B.idesc = at<InstDesc>(P.d_tables, t.idesc);
    B.order = at<int32_t>(P.d_tables, t.order);
    B.team_off = at<int32_t>(P.d_tables, t.team_off);
    B.team_list = at<int32_t>(P.d_tables, t.team_list);
    B.queue = at<unsigned int>(a.ws, w.counters);
    B.bars = at<unsigned int>(a.ws, w.counters) + 2;
    B.L_out = a.L_out;
    B.norm_out = a.norm_out;
    B.n_solo = (int32_t)ts.solo.size();
    B.n_teams = ts.n_teams;
    B.team_size = ts.team_size;
    B.n_xcd = ts.n_xcd;
    B.spin_ticks = d->spin_ticks;
    return launch_batched(L, B, d->batch_grid, st);
}

struct BwdArgs {
    const void* psi_out;
    const double* dL;
    void* grad_psi;
    double* grad_angles;
    const double* angles;
    void* ws;
};

hipError_t enqueue_backward(DevPlan* d, const BwdArgs& a, hipStream_t st) {
    Plan& P = d->host;
    hipError_t e = enqueue_prep(d, a.ws, a.angles, PK_OP_BACKWARD, 0, st);
    if (e != hipSuccess) return e;
    WsLayout w = workspace_layout(&P, PK_OP_BACKWARD);
    PassLaunch L = base_launch(d, a.ws, PK_OP_BACKWARD);
    L.src0 = a.psi_out;
    L.dst0 = at<void>(a.ws, w.state);
    L.dst1 = a.grad_psi;
    L.dL = a.dL;
    L.want_norm = 0;
    L.nv = 2;
    const Instance& in = P.inst[0];
    for (size_t p = 0; p < in.bwd.size(); ++p) {
        L.pass = P.n_fwd_passes + (int)p;
        L.kmax = in.bwd[p].kmax;
        L.ntiles = in.bwd[p].ntiles;
        L.grid_cap = P.tiling.wgs_per_cu;
        L.rbits = in.bwd[p].rbits;
        e = launch_pass(L, st);
        if (e != hipSuccess) return e;
    }
    if (!a.grad_angles || P.d2_grad.empty()) return hipSuccess;
    TableLayout t = table_layout(&P);
    return launch_reduce(at<Reduction>(P.d_tables, t.red) + 2 * P.inst.size(), 3 * (int)P.d2_grad.size(),
                         static_cast<double*>(a.ws), nullptr, nullptr, a.grad_angles, st);
}

bool no_graph() {
    const char* v = std::getenv("PK_NO_GRAPH");
    return v && v[0] && v[0] != '0';
}

// Replays the cached graph for `slot` when the pointer set matches, else
// captures `fn` on the plan's capture stream and instantiates it.
template <typename Fn>
int run_graphed(DevPlan* d, int slot, const void* const (&key)[8], hipStream_t st, Fn fn) {
    if (no_graph()) {
        hipError_t e = fn(st);
        return e == hipSuccess ? PK_OK : hip_fail(d, e, "kernel launch");
    }
    if (!d->exec[slot] || std::memcmp(d->key[slot], key, sizeof key) != 0) {
        if (d->exec[slot]) hipGraphExecDestroy(reinterpret_cast<hipGraphExec_t>(d->exec[slot]));
        d->exec[slot] = nullptr;
        hipError_t e = hipStreamBeginCapture(d->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(d, e, "hipStreamBeginCapture");
        hipError_t le = fn(d->cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(d->cap, &g);
        if (le != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return hip_fail(d, le, "kernel launch (capture)");
        }
        if (e != hipSuccess) return hip_fail(d, e, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(d, e, "hipGraphInstantiate");
        d->exec[slot] = ex;
        std::memcpy(d->key[slot], key, sizeof key);
    }
    hipError_t e = hipGraphLaunch(reinterpret_cast<hipGraphExec_t>(d->exec[slot]), st);
    return e == hipSuccess ? PK_OK : hip_fail(d, e, "hipGraphLaunch");
}

int check_eval_args(DevPlan* d, const void* psi_in, void* psi_out, double* L_out, double* norm_out,
                    const double* angles, void* ws) {
    if (!psi_in || !psi_out || !L_out || !ws) return fail(d, PK_EINVAL, "NULL pointer argument");
    if (!aligned(psi_in, 16) || !aligned(psi_out, 16) || !aligned(ws, 256) || !aligned(L_out, 8) ||
        (norm_out && !aligned(norm_out, 8)) || (angles && !aligned(angles, 8)))
        return fail(d, PK_EINVAL, "misaligned pointer (states 16 B, workspace 256 B, doubles 8 B)");
    return PK_OK;
}


// Re-compiles after a tiling or launch change; on failure the previous
// settings and schedule come back, so the plan stays usable.
int recompile_or_restore(DevPlan* d, const Tiling& previous) {
    std::string err;
    int rc;
    try {
        rc = recompile(&d->host, &err);
    } catch (const std::bad_alloc&) {
        rc = PK_ENOMEM;
        err = "out of host memory";
    } catch (...) {
        rc = PK_EINVAL;
        err = "plan compilation failed";
    }
    if (rc == PK_OK) return PK_OK;
    d->host.tiling = previous;
    std::string ignored;
    try {
        recompile(&d->host, &ignored);
    } catch (...) {
    }
    return fail(d, rc, err);
}

// The workspace of pk_evaluate_static: a device array of fixed size that every
// call on a GPU shares (each GPU holds its own copy until the process ends).
// Host code never passes `scratch` itself to a kernel (its host-side name is not
// a device address): the device address comes from hipGetSymbolAddress, once per
// device, with that device current.
constexpr size_t kStaticWorkspaceBytes = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's `scratch` (looked up on the first call per device).
hipError_t static_workspace(int dev, void** out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

int pk_create(const pk_problem* probs, int32_t n_inst, int32_t prec, pk_plan** out) {
    if (!out) return fail(nullptr, PK_EINVAL, "out is NULL");
    *out = nullptr;
    DevPlan* d = new (std::nothrow) DevPlan();
    if (!d) return fail(nullptr, PK_ENOMEM, "out of host memory");
    std::string err;
    int rc;
    try {
        rc = compile_plan(&d->host, probs, n_inst, prec, &err);
    } catch (const std::bad_alloc&) {
        rc = PK_ENOMEM;
        err = "out of host memory";
    } catch (...) {
        rc = PK_EINVAL;
        err = "plan compilation failed";
    }
    if (rc != PK_OK) {
        delete d;
        return fail(nullptr, rc, err);
    }
    *out = reinterpret_cast<pk_plan*>(d);
    return PK_OK;
}

int pk_set_tiling(pk_plan* plan, int32_t tile_bits, int32_t carrier_bits, int32_t fuse, int32_t lane_order,
                  int32_t page_cap) {
    if (!valid(plan)) return fail(nullptr, PK_EINVAL, "invalid plan");
    DevPlan* d = dp(plan);
    const int kmax = d->host.prec == PK_FP64 ? 13 : 14;
    if (tile_bits < 4 || tile_bits > kmax) return fail(d, PK_EINVAL, "tile_bits out of range");
    if (carrier_bits < 0 || carrier_bits > 6 || carrier_bits > tile_bits - 1)
        return fail(d, PK_EINVAL, "carrier_bits out of range");
    if (fuse != 0 && fuse != 1) return fail(d, PK_EINVAL, "fuse must be 0 or 1");
    if (lane_order != 0 && lane_order != 1) return fail(d, PK_EINVAL, "lane_order must be 0 or 1");
    if (page_cap < -1 || page_cap > 16) return fail(d, PK_EINVAL, "page_cap must be -1..16");
    if (tile_bits - d->host.tiling.reg_bits > 10)
        return fail(d, PK_EINVAL, "tile_bits - reg_bits must be at most 10 (1024 threads a workgroup)");
    const Tiling previous = d->host.tiling;
    d->host.walk.clear();  // the passes change with the tiling
    d->host.overlap.clear();
    d->host.tiling = Tiling{tile_bits, carrier_bits, fuse, d->host.tiling.wgs_per_cu, d->host.tiling.reg_bits,
                            lane_order, page_cap < 0 ? default_page_cap(d->host.prec) : page_cap};
    drop_device(d);
    return recompile_or_restore(d, previous);
}

int pk_set_pass_walk(pk_plan* plan, int32_t n, const int32_t* walk) {
    if (!valid(plan)) return fail(nullptr, PK_EINVAL, "invalid plan");
    DevPlan* d = dp(plan);
    if (d->host.inst.size() != 1) return fail(d, PK_EINVAL, "pk_set_pass_walk needs a single-instance plan");
    const size_t nf = d->host.inst[0].fwd.size(), nb = d->host.inst[0].bwd.size();
    if (n != 0 && (size_t)n != nf && (size_t)n != nf + nb)
        return fail(d, PK_EINVAL, "walk needs one entry per forward pass (then, optionally, per backward pass), or n = 0");
    if (n > 0 && !walk) return fail(d, PK_EINVAL, "walk is NULL");
    std::vector<int32_t> w(walk, walk + n);
    for (int32_t c : w)
        if (c < -1 || c == 1 || c > (1 << 16)) return fail(d, PK_EINVAL, "walk entries are 0, -1 or 2..65536");
    if (w == d->host.walk) return PK_OK;
    const Tiling previous = d->host.tiling;
    const std::vector<int32_t> before = d->host.walk;
    d->host.walk = w;
    drop_device(d);
    const int rc = recompile_or_restore(d, previous);
    if (rc != PK_OK) d->host.walk = before;
    return rc;
}

int pk_set_pass_overlap(pk_plan* plan, int32_t n, const int32_t* on) {
    if (!valid(plan)) return fail(nullptr, PK_EINVAL, "invalid plan");
    DevPlan* d = dp(plan);
    if (d->host.inst.size() != 1) return fail(d, PK_EINVAL, "pk_set_pass_overlap needs a single-instance plan");
    const size_t nf = d->host.inst[0].fwd.size();
    if (n != 0 && (size_t)n != nf) return fail(d, PK_EINVAL, "overlap needs one entry per forward pass, or n = 0");
    if (n > 0 && !on) return fail(d, PK_EINVAL, "on is NULL");
    std::vector<int32_t> w(on, on + n);
    for (int32_t c : w)
        if (c != 0 && c != 1) return fail(d, PK_EINVAL, "overlap entries are 0 or 1");
    if (w == d->host.overlap) return PK_OK;
    const Tiling previous = d->host.tiling;
    const std::vector<int32_t> before = d->host.overlap;
    d->host.overlap = w;
    drop_device(d);
    const int rc = recompile_or_restore(d, previous);
    if (rc != PK_OK) d->host.overlap = before;
    return rc;
}

int pk_set_lane_maps(pk_plan* plan, int32_t on) {
    if (!valid(plan)) return fail(nullptr, PK_EINVAL, "invalid plan");
    DevPlan* d = dp(plan);
    if (on != 0 && on != 1) return fail(d, PK_EINVAL, "on must be 0 or 1");
    if (on == d->host.lane_maps) return PK_OK;
    const Tiling previous = d->host.tiling;
    d->host.lane_maps = on;
    drop_device(d);
    const int rc = recompile_or_restore(d, previous);
    if (rc != PK_OK) d->host.lane_maps = 1 - on;
    return rc;
}

int pk_set_launch(pk_plan* plan, int32_t wgs_per_cu, int32_t reg_bits) {
    if (!valid(plan)) return fail(nullptr, PK_EINVAL, "invalid plan");
    DevPlan* d = dp(plan);
    if (wgs_per_cu < 0 || wgs_per_cu > 8) return fail(d, PK_EINVAL, "wgs_per_cu must be 0..8");
    if (reg_bits != 0 && (reg_bits < 3 || reg_bits > 5)) return fail(d, PK_EINVAL, "reg_bits must be 0, 3, 4 or 5");
    const int rb = reg_bits == 0 ? default_reg_bits(d->host.prec) : reg_bits;
    if (d->host.tiling.tile_bits - rb > 10)
        return fail(d, PK_EINVAL, "tile_bits - reg_bits must be at most 10 (1024 threads a workgroup)");
    const bool recompile_needed = rb != d->host.tiling.reg_bits;
    const Tiling previous = d->host.tiling;
    d->host.tiling.wgs_per_cu = wgs_per_cu;
    d->host.tiling.reg_bits = rb;
    if (recompile_needed) {
        d->host.walk.clear();  // the passes change with the register bits
        d->host.overlap.clear();
        drop_device(d);
        return recompile_or_restore(d, previous);
    }
    drop_graphs(d);
    return PK_OK;
}

int pk_set_batch(pk_plan* plan, int32_t team_size, int32_t min_team_tiles) {
    if (!valid(plan)) return fail(nullptr, PK_EINVAL, "invalid plan");
    DevPlan* d = dp(plan);
    if (team_size < 0 || team_size > 64) return fail(d, PK_EINVAL, "team_size must be 0..64");
    if (min_team_tiles < 1 || min_team_tiles > 4096) return fail(d, PK_EINVAL, "min_team_tiles must be 1..4096");
    d->host.batch = BatchConfig{team_size, min_team_tiles};
    drop_device(d);  // the team schedule is part of the device tables
    return PK_OK;
}

int pk_batch_teams(pk_plan* plan, int32_t* n_teams, int32_t* n_team_instances) {
    if (!valid(plan) || !n_teams || !n_team_instances) return fail(nullptr, PK_EINVAL, "invalid argument");
    DevPlan* d = dp(plan);
    const int rc = ensure_device(d);
    if (rc != PK_OK) return rc;
    *n_teams = d->host.team.n_teams;
    *n_team_instances = (int32_t)d->host.team.team_list.size();
    return PK_OK;
}

int pk_plan_passes(const pk_plan* plan, int32_t inst, int32_t* passes) {
    if (!valid(plan) || !passes) return fail(nullptr, PK_EINVAL, "invalid argument");
    const Plan& P = dp(plan)->host;
    if (inst < 0 || inst >= (int)P.inst.size()) return PK_EINVAL;
    *passes = (int32_t)P.inst[inst].fwd.size();
    return PK_OK;
}

int pk_plan_describe(const pk_plan* plan, char* buf, int64_t cap, int64_t* needed) {
    if (!valid(plan)) return fail(nullptr, PK_EINVAL, "invalid plan");
    std::string s = describe(&dp(plan)->host);
    if (needed) *needed = (int64_t)s.size() + 1;
    if (buf && cap > 0) {
        size_t n = s.size() < (size_t)(cap - 1) ? s.size() : (size_t)(cap - 1);
        std::memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return PK_OK;
}

int pk_plan_offsets(const pk_plan* plan, int64_t* offsets) {
    if (!valid(plan) || !offsets) return fail(nullptr, PK_EINVAL, "invalid argument");
    const Plan& P = dp(plan)->host;
    for (size_t i = 0; i < P.inst.size(); ++i) offsets[i] = P.inst[i].off;
    offsets[P.inst.size()] = P.total_elems;
    return PK_OK;
}

int pk_plan_n_angles(const pk_plan* plan, int64_t* n_d2) {
    if (!valid(plan) || !n_d2) return fail(nullptr, PK_EINVAL, "invalid argument");
    *n_d2 = (int64_t)dp(plan)->host.params.size();
    return PK_OK;
}

int pk_workspace_bytes(const pk_plan* plan, int32_t op, int64_t* bytes) {
    if (!valid(plan) || !bytes) return fail(nullptr, PK_EINVAL, "invalid argument");
    if (op != PK_OP_EVAL && op != PK_OP_BACKWARD) return fail(nullptr, PK_EINVAL, "unknown op");
    *bytes = (int64_t)workspace_layout(&dp(plan)->host, op).total;
    return PK_OK;
}

int pk_evaluate(pk_plan* plan, const void* psi_in, void* psi_out, double* L_out, double* norm_out,
                const double* angles, void* workspace, void* stream) {
    if (!valid(plan)) return fail(nullptr, PK_EINVAL, "invalid plan");
    DevPlan* d = dp(plan);
    if (d->host.inst.size() != 1) return fail(d, PK_EINVAL, "pk_evaluate needs a single-instance plan");
    int rc = check_eval_args(d, psi_in, psi_out, L_out, norm_out, angles, workspace);
    if (rc != PK_OK) return rc;
    rc = ensure_device(d);
    if (rc != PK_OK) return rc;
    EvalArgs a{psi_in, psi_out, L_out, norm_out, angles, workspace};
    const void* const key[8] = {psi_in, psi_out, L_out, norm_out, angles, workspace, nullptr, nullptr};
    return run_graphed(d, G_EVAL, key, static_cast<hipStream_t>(stream),
                       [&](hipStream_t s) { return enqueue_eval(d, a, s, nullptr); });
}

int pk_evaluate_static(pk_plan* plan, const void* psi_in, void* psi_out, double* L_out, double* norm_out,
                       const double* angles, void* stream) {
    if (!valid(plan)) return fail(nullptr, PK_EINVAL, "invalid plan");
    DevPlan* d = dp(plan);
    if (d->host.inst.size() != 1) return fail(d, PK_EINVAL, "pk_evaluate_static needs a single-instance plan");
    const size_t need = workspace_layout(&d->host, PK_OP_EVAL).total;
    if (need > kStaticWorkspaceBytes)
        return fail(d, PK_EINVAL,
                    "the plan needs " + std::to_string(need) + " bytes of workspace; the static buffer holds " +
                        std::to_string(kStaticWorkspaceBytes) + " (use larger tiles, or pk_evaluate)");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(d, e, "hipGetDevice");
    if (!d->host.d_tables || d->host.device != dev)
        return fail(d, PK_EINVAL,
                    "the plan's tables are not on this device: upload them first (pk_evaluate or pk_batch_teams "
                    "with this device current)");
    void* ws = nullptr;
    e = static_workspace(dev, &ws);
    if (e != hipSuccess) return hip_fail(d, e, "hipGetSymbolAddress(scratch)");
    int rc = check_eval_args(d, psi_in, psi_out, L_out, norm_out, angles, ws);
    if (rc != PK_OK) return rc;
    EvalArgs a{psi_in, psi_out, L_out, norm_out, angles, ws};
    e = enqueue_eval(d, a, static_cast<hipStream_t>(stream), nullptr);
    return e == hipSuccess ? PK_OK : hip_fail(d, e, "pk_evaluate_static");
}

int pk_evaluate_repeat(pk_plan* plan, int64_t reps, const void* psi_in, void* psi_out, double* L_out,
                       double* norm_out, const double* angles, void* workspace, void* stream) {
    if (!valid(plan)) return fail(nullptr, PK_EINVAL, "invalid plan");
    DevPlan* d = dp(plan);
    if (d->host.inst.size() != 1) return fail(d, PK_EINVAL, "pk_evaluate_repeat needs a single-instance plan");
    if (reps < 1 || reps > ((int64_t)1 << 24)) return fail(d, PK_EINVAL, "reps out of 1..2^24");
    if ((int64_t)d->host.inst[0].fwd.size() * reps > ((int64_t)1 << 20))
        return fail(d, PK_EINVAL, "more than 2^20 pass launches in one graph");
    int rc = check_eval_args(d, psi_in, psi_out, L_out, norm_out, angles, workspace);
    if (rc != PK_OK) return rc;
    rc = ensure_device(d);
    if (rc != PK_OK) return rc;
    EvalArgs a{psi_in, psi_out, L_out, norm_out, angles, workspace};
    const unsigned grid = (reps > 1 && repeat_persistent()) ? repeat_grid(d) : 0u;
    const void* const key[8] = {psi_in, psi_out, L_out, norm_out, angles, workspace,
                                reinterpret_cast<const void*>((intptr_t)reps),
                                reinterpret_cast<const void*>((intptr_t)grid)};
    if (grid > 0)
        return run_graphed(d, G_REPEAT, key, static_cast<hipStream_t>(stream),
                           [&](hipStream_t s) { return enqueue_repeat(d, a, s, reps, grid); });
    const RepeatSplit sp = repeat_split(d, reps);
    if (sp.fused) {
        rc = ensure_device(sp.fused);
        if (rc != PK_OK) return fail(d, rc, sp.fused->host.last_error);
        return run_graphed(d, G_REPEAT, key, static_cast<hipStream_t>(stream),
                           [&](hipStream_t s) { return enqueue_repeat_fused(d, sp, a, s); });
    }
    return run_graphed(d, G_REPEAT, key, static_cast<hipStream_t>(stream),
                       [&](hipStream_t s) { return enqueue_eval(d, a, s, nullptr, reps); });
}

int pk_repeat_launches(pk_plan* plan, int64_t reps, int64_t* launches) {
    if (!valid(plan)) return fail(nullptr, PK_EINVAL, "invalid plan");
    DevPlan* d = dp(plan);
    if (!launches) return fail(d, PK_EINVAL, "NULL output");
    if (d->host.inst.size() != 1) return fail(d, PK_EINVAL, "pk_repeat_launches needs a single-instance plan");
    if (reps < 1 || reps > ((int64_t)1 << 24)) return fail(d, PK_EINVAL, "reps out of 1..2^24");
    const RepeatSplit sp = repeat_split(d, reps);
    *launches = sp.single * (int64_t)d->host.inst[0].fwd.size() +
                (sp.fused ? sp.rounds * (int64_t)sp.fused->host.inst[0].fwd.size() : 0);
    return PK_OK;
}

int pk_search_workspace_bytes(int64_t* bytes) {
    if (!bytes) return fail(nullptr, PK_EINVAL, "NULL output");
    *bytes = (int64_t)search_workspace_bytes();
    return PK_OK;
}

int pk_search_diffusion(int32_t nq, int32_t prec, const int64_t* marked, int32_t n_marked, int64_t iterations,
                        const void* psi_in, void* psi_out, double* L_out, void* workspace, void* stream) {
    if (prec != PK_FP64 && prec != PK_FP32) return fail(nullptr, PK_EINVAL, "prec must be PK_FP64 or PK_FP32");
    if (nq < 1 || nq > (prec == PK_FP64 ? 30 : 31)) return fail(nullptr, PK_EINVAL, "nq out of range");
    if (n_marked < 0 || n_marked > 64 || (n_marked > 0 && !marked))
        return fail(nullptr, PK_EINVAL, "marked set must hold 0..64 labels");
    if (iterations < 1) return fail(nullptr, PK_EINVAL, "iterations must be >= 1");
    if (!psi_in || !psi_out || !L_out || !workspace || (reinterpret_cast<uintptr_t>(psi_in) & 15) ||
        (reinterpret_cast<uintptr_t>(psi_out) & 15) || (reinterpret_cast<uintptr_t>(workspace) & 15))
        return fail(nullptr, PK_EINVAL, "NULL or misaligned pointer");
    MarkedSet ms{};
    ms.count = n_marked;
    for (int i = 0; i < n_marked; ++i) {
        if (marked[i] < 0 || marked[i] >= ((int64_t)1 << nq)) return fail(nullptr, PK_EINVAL, "marked label out of range");
        for (int j = 0; j < i; ++j)
            if (marked[j] == marked[i]) return fail(nullptr, PK_EINVAL, "duplicate marked label");
        ms.label[i] = marked[i];
    }
    hipError_t e = launch_search(psi_in, psi_out, nq, prec == PK_FP64, ms, iterations, workspace, L_out,
                                 static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PK_OK : hip_fail(nullptr, e, "diffusion search");
}

int pk_evaluate_batched(pk_plan* plan, const void* psi_in, void* psi_out, double* L_out, double* norm_out,
                        const double* angles, void* workspace, void* stream) {
    if (!valid(plan)) return fail(nullptr, PK_EINVAL, "invalid plan");
    DevPlan* d = dp(plan);
    if (d->host.tiling.reg_bits == 3)
        return fail(d, PK_EUNSUPPORTED, "the batched launch has 4 or 5 register bits (pk_set_launch)");
    int rc = check_eval_args(d, psi_in, psi_out, L_out, norm_out, angles, workspace);
    if (rc != PK_OK) return rc;
    rc = ensure_device(d);
    if (rc != PK_OK) return rc;
    EvalArgs a{psi_in, psi_out, L_out, norm_out, angles, workspace};
    const void* const key[8] = {psi_in, psi_out, L_out, norm_out, angles, workspace, nullptr, nullptr};
    return run_graphed(d, G_BATCH, key, static_cast<hipStream_t>(stream),
                       [&](hipStream_t s) { return enqueue_batched(d, a, s); });
}

int pk_backward(pk_plan* plan, const void* psi_out, const double* dL, void* grad_psi_in, double* grad_angles,
                const double* angles, void* workspace, void* stream) {
    if (!valid(plan)) return fail(nullptr, PK_EINVAL, "invalid plan");
    DevPlan* d = dp(plan);
    if (d->host.inst.size() != 1) return fail(d, PK_EINVAL, "pk_backward needs a single-instance plan");
    if (!d->host.backward_ok)
        return fail(d, PK_EUNSUPPORTED, "a ONEOP gate is not unitary: its adjoint is not its inverse");
    if (!psi_out || !dL || !grad_psi_in || !workspace) return fail(d, PK_EINVAL, "NULL pointer argument");
    if (!aligned(psi_out, 16) || !aligned(grad_psi_in, 16) || !aligned(workspace, 256) || !aligned(dL, 8) ||
        (grad_angles && !aligned(grad_angles, 8)) || (angles && !aligned(angles, 8)))
        return fail(d, PK_EINVAL, "misaligned pointer");
    int rc = ensure_device(d);
    if (rc != PK_OK) return rc;
    BwdArgs a{psi_out, dL, grad_psi_in, grad_angles, angles, workspace};
    const void* const key[8] = {psi_out, dL, grad_psi_in, grad_angles, angles, workspace, nullptr, nullptr};
    return run_graphed(d, G_BWD, key, static_cast<hipStream_t>(stream),
                       [&](hipStream_t s) { return enqueue_backward(d, a, s); });
}

int pk_pair_indices(int32_t nq, int32_t i_s, int64_t first, int64_t count, int64_t* n0, int64_t* n1,
                    void* stream) {
    if (nq < 1 || nq > 31) return fail(nullptr, PK_EINVAL, "nq out of 1..31");
    if (i_s < 1 || i_s > nq) return fail(nullptr, PK_EINVAL, "i_s out of 1..nq");
    const int64_t npairs = (int64_t)1 << (nq - 1);
    if (first < 0 || count < 0 || first + count > npairs) return fail(nullptr, PK_EINVAL, "pair range out of bounds");
    if (count > 0 && (!n0 || !n1)) return fail(nullptr, PK_EINVAL, "NULL output");
    hipError_t e = launch_pairs(nq, i_s, first, count, n0, n1, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PK_OK : hip_fail(nullptr, e, "pair_index_kernel");
}

int pk_shor_state(int32_t n1, int32_t n2, int64_t xguess, int64_t M, int32_t prec, void* psi, void* stream) {
    if (prec != PK_FP64 && prec != PK_FP32) return fail(nullptr, PK_EINVAL, "prec must be PK_FP64 or PK_FP32");
    const int nq_max = prec == PK_FP64 ? 30 : 31;
    if (n1 < 1 || n2 < 1 || n1 + n2 > nq_max) return fail(nullptr, PK_EINVAL, "register sizes out of range");
    if (M < 2 || M > ((int64_t)1 << n2) || M >= ((int64_t)1 << 31))
        return fail(nullptr, PK_EINVAL, "M must satisfy 2 <= M <= 2^n2 and M < 2^31");
    if (xguess < 1 || xguess >= M) return fail(nullptr, PK_EINVAL, "xguess must lie in 1..M-1");
    if (!psi || (reinterpret_cast<uintptr_t>(psi) & 15)) return fail(nullptr, PK_EINVAL, "psi NULL or not 16-byte aligned");
    // the correctly rounded 2^(-n1/2): an exact power of two, or sqrt(2) (correctly
    // rounded by IEEE sqrt) times one
    const double amp = (n1 % 2 == 0) ? std::ldexp(1.0, -n1 / 2) : std::ldexp(std::sqrt(2.0), -(n1 + 1) / 2);
    hipError_t e = launch_shor_state(n1, n2, (uint64_t)xguess, (uint64_t)M, prec == PK_FP64, amp, psi,
                                     static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PK_OK : hip_fail(nullptr, e, "shor_state_kernel");
}

namespace {
int marginal_entry(int32_t nq, int32_t n_low, int32_t prec, bool bitrev, const void* psi, double* p, void* stream) {
    if (prec != PK_FP64 && prec != PK_FP32) return fail(nullptr, PK_EINVAL, "prec must be PK_FP64 or PK_FP32");
    if (nq < 1 || nq > (prec == PK_FP64 ? 30 : 31)) return fail(nullptr, PK_EINVAL, "nq out of range");
    if (n_low < 0 || n_low > nq) return fail(nullptr, PK_EINVAL, "n_low out of 0..nq");
    if (!psi || !p || (reinterpret_cast<uintptr_t>(psi) & 15) || (reinterpret_cast<uintptr_t>(p) & 7))
        return fail(nullptr, PK_EINVAL, "NULL or misaligned pointer");
    hipError_t e = launch_marginal(nq, n_low, prec == PK_FP64, bitrev, psi, p, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PK_OK : hip_fail(nullptr, e, "marginal_kernel");
}
}  // namespace

int pk_marginal(int32_t nq, int32_t n_low, int32_t prec, const void* psi, double* p, void* stream) {
    return marginal_entry(nq, n_low, prec, false, psi, p, stream);
}

int pk_marginal_bitrev(int32_t nq, int32_t n_low, int32_t prec, const void* psi, double* p, void* stream) {
    return marginal_entry(nq, n_low, prec, true, psi, p, stream);
}

int pk_density_matrix(int32_t nq, int32_t n_univ, const void* states, const double* weights, void* rho,
                      void* stream) {
    if (nq < 1 || nq > 16) return fail(nullptr, PK_EINVAL, "nq out of 1..16");
    if (n_univ < 1) return fail(nullptr, PK_EINVAL, "need at least one universe");
    if (!states || !weights || !rho || (reinterpret_cast<uintptr_t>(states) & 15) ||
        (reinterpret_cast<uintptr_t>(rho) & 15) || (reinterpret_cast<uintptr_t>(weights) & 7))
        return fail(nullptr, PK_EINVAL, "NULL or misaligned pointer");
    hipError_t e = launch_density(states, weights, rho, (int64_t)1 << nq, n_univ, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PK_OK : hip_fail(nullptr, e, "density_kernel");
}

namespace {
// One rocBLAS handle per thread and device, kept for the process (creating one
// loads the library's kernels).
rocblas_handle solver_handle(int dev) {
    thread_local std::vector<rocblas_handle> handles;
    if ((int)handles.size() <= dev) handles.resize(dev + 1, nullptr);
    if (!handles[dev] && rocblas_create_handle(&handles[dev]) != rocblas_status_success) handles[dev] = nullptr;
    return handles[dev];
}
}  // namespace

int pk_density_spectrum(int32_t nq, void* rho, double* eigenvalues, double* sums, void* stream) {
    if (nq < 1 || nq > 15) return fail(nullptr, PK_EINVAL, "nq out of 1..15");
    if (!rho || !eigenvalues || !sums || (reinterpret_cast<uintptr_t>(rho) & 15))
        return fail(nullptr, PK_EINVAL, "NULL or misaligned pointer");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
    rocblas_handle h = solver_handle(dev);
    if (!h) return fail(nullptr, PK_EDEVICE, "rocblas_create_handle failed");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (rocblas_set_stream(h, st) != rocblas_status_success) return fail(nullptr, PK_EDEVICE, "rocblas_set_stream");
    const int64_t n = (int64_t)1 << nq;
    double* off = nullptr;  // the tridiagonal's off-diagonal, and the convergence flag
    e = hipMallocAsync(reinterpret_cast<void**>(&off), n * sizeof(double) + 256, st);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipMallocAsync");
    rocblas_int* info = reinterpret_cast<rocblas_int*>(off + n);
    // rho is Hermitian and row-major; read as column-major it is conj(rho), whose
    // eigenvalues are the same.  The lower triangle is read; rho is overwritten.
    rocblas_status rs = rocsolver_zheevd(h, rocblas_evect_none, rocblas_fill_lower, (rocblas_int)n,
                                         static_cast<rocblas_double_complex*>(rho), (rocblas_int)n, eigenvalues, off,
                                         info);
    rocblas_int hinfo = 0;
    if (rs == rocblas_status_success) {
        e = launch_spectrum_sums(eigenvalues, n, sums, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&hinfo, info, sizeof hinfo, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    hipError_t fe = hipFreeAsync(off, st);
    if (rs != rocblas_status_success) return fail(nullptr, PK_EDEVICE, std::string("rocsolver_zheevd: ") + rocblas_status_to_string(rs));
    if (e != hipSuccess) return hip_fail(nullptr, e, "spectrum");
    if (fe != hipSuccess) return hip_fail(nullptr, fe, "hipFreeAsync");
    if (hinfo != 0) return fail(nullptr, PK_EDEVICE, "rocsolver_zheevd did not converge");
    return PK_OK;
}

int pk_time_passes(pk_plan* plan, const void* psi_in, void* psi_out, double* L_out, const double* angles,
                   void* workspace, void* stream, double* ms, int32_t max_n, int32_t* n) {
    if (!valid(plan)) return fail(nullptr, PK_EINVAL, "invalid plan");
    DevPlan* d = dp(plan);
    if (d->host.inst.size() != 1) return fail(d, PK_EINVAL, "single-instance plans only");
    if (!ms || !n || max_n < 0) return fail(d, PK_EINVAL, "NULL output");
    int rc = check_eval_args(d, psi_in, psi_out, L_out, nullptr, angles, workspace);
    if (rc != PK_OK) return rc;
    rc = ensure_device(d);
    if (rc != PK_OK) return rc;
    const size_t np = d->host.inst[0].fwd.size();
    std::vector<hipEvent_t> ev(2 * np, nullptr);
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) return fail(d, PK_EDEVICE, "hipEventCreate");
    hipStream_t st = static_cast<hipStream_t>(stream);
    EvalArgs a{psi_in, psi_out, L_out, nullptr, angles, workspace};
    hipError_t e = enqueue_eval(d, a, st, &ev);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    int w = 0;
    if (e == hipSuccess) {
        for (size_t p = 0; p < np && w < max_n; ++p) {
            float t = 0.f;
            hipEventElapsedTime(&t, ev[2 * p], ev[2 * p + 1]);
            ms[w++] = t;
        }
    }
    for (auto& x : ev) hipEventDestroy(x);
    *n = w;
    return e == hipSuccess ? PK_OK : hip_fail(d, e, "pk_time_passes");
}

void pk_destroy(pk_plan* plan) {
    if (!valid(plan)) return;
    DevPlan* d = dp(plan);
    drop_device(d);
    if (d->cap) hipStreamDestroy(d->cap);
    d->host.magic = 0;
    delete d;
}

const char* pk_strerror(int code) {
    switch (code) {
    case PK_OK: return "success";
    case PK_EINVAL: return "invalid argument";
    case PK_ENOMEM: return "out of memory";
    case PK_EDEVICE: return "HIP device error";
    case PK_EUNSUPPORTED: return "unsupported request";
    default: return "unknown error code";
    }
}

const char* pk_last_error(const pk_plan* plan) {
    if (!plan) return g_error.c_str();
    if (!valid(plan)) return "invalid plan";
    return dp(plan)->host.last_error.c_str();
}

}  // extern "C"
