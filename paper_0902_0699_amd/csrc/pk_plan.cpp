// Plan compiler: validates gate lists and lowers them to pass / stage / op tables.
//
// Legality rests on two facts about the gates of the paper: gates on disjoint
// sets of qubits commute (each acts on its own tensor factors, Sec. 2.1), and
// diagonal operations (Oracle, Inv, Sec. 5.1; the controlled phases CPHASE and
// CPHASEK, Eq. cphasek) commute with each other.  Any order of the primitives
// that keeps every non-commuting pair in list order computes the same state, so
// the compiler may gather all gates on a set of qubits into one pass over the
// state.  A controlled phase needs no partner amplitude: each amplitude's
// factor follows from its own label, so it runs in whatever pass and stage its
// ordering allows, whether or not its qubits are tile or register bits.
#include "pk_plan.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <stdexcept>
#include <string>

namespace pk {

namespace {

constexpr int kWaveBits = 6;          // smallest kernel instance: one wavefront of 64 threads
constexpr int kBackwardMaxBits = 12;  // largest backward tile (psi and lambda in registers)

bool finite8(const double* v, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

bool is_unitary(const double* m) {
    // m row-major complex 2x2; check M^H M = I
    double a[2][2][2];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            a[r][c][0] = m[2 * (2 * r + c)];
            a[r][c][1] = m[2 * (2 * r + c) + 1];
        }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double re = 0, im = 0;
            for (int r = 0; r < 2; ++r) {  // conj(a[r][i]) * a[r][j]
                re += a[r][i][0] * a[r][j][0] + a[r][i][1] * a[r][j][1];
                im += a[r][i][0] * a[r][j][1] - a[r][i][1] * a[r][j][0];
            }
            if (std::fabs(re - (i == j ? 1.0 : 0.0)) > 1e-12 || std::fabs(im) > 1e-12) return false;
        }
    return true;
}

bool is_unitary4(const double* m) {
    // m row-major complex 4x4; check M^H M = I
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double re = 0, im = 0;
            for (int r = 0; r < 4; ++r) {
                const double ar = m[2 * (4 * r + i)], ai = m[2 * (4 * r + i) + 1];
                const double br = m[2 * (4 * r + j)], bi = m[2 * (4 * r + j) + 1];
                re += ar * br + ai * bi;
                im += ar * bi - ai * br;
            }
            if (std::fabs(re - (i == j ? 1.0 : 0.0)) > 1e-12 || std::fabs(im) > 1e-12) return false;
        }
    return true;
}

// Forward scan: which not-yet-scheduled primitives can run in a pass (or stage)
// whose register/tile bit set is `in_set`.  A gate is blocked by an earlier
// unscheduled gate or controlled phase on one of its bits, or an earlier
// unscheduled Oracle/Inv; Oracle/Inv are blocked by any earlier unscheduled
// gate; a controlled phase only by an earlier unscheduled gate on one of its
// bits (phases, Oracle and Inv are all diagonal).  Gates need their bits in the
// set, phases do not.  Two-qubit gates need both bits; `pair` further restricts
// them: PAIR_ANY (tiles), PAIR_NONE (a stage without two-qubit gates), or
// (b1 << 8 | b2), the ordered pair a stage holds on register bits 0 and 1;
// `pair2` is a second, disjoint pair on register bits 2 and 3 (or PAIR_NONE),
// which takes only the gates whose kernel step exists for those bits.
constexpr int PAIR_ANY = -1;
constexpr int PAIR_NONE = -2;

enum ItemType { IT_GATE = 0, IT_DIAG = 1, IT_PHASE = 2 };

struct ScanItem {
    int type;
    int bit;   // IT_GATE, IT_PHASE: first bit (for a phase, -1 when it is outside the tile)
    int bit2;  // second bit of a two-qubit gate or phase, -1 otherwise
    bool swap = false;  // a SWAP gate (done by relabelling bits when the pass allows)
    bool pair_b = true; // a two-qubit gate the second register pair (bits 2, 3) can take
};

int scan(const std::vector<ScanItem>& items, const std::vector<char>& done,
         const std::vector<char>& in_set, int nbits, int max_gates, std::vector<int>* out,
         int pair = PAIR_ANY, int pair2 = PAIR_NONE) {
    std::vector<char> blocked(nbits, 0);  // later gates on the bit must wait
    std::vector<char> nd(nbits, 0);       // later phases on the bit must wait (a non-diagonal gate is pending)
    bool blocked_gate = false, blocked_diag = false;
    int count = 0, gates = 0;
    for (size_t i = 0; i < items.size(); ++i) {
        if (done[i]) continue;
        const ScanItem& it = items[i];
        if (it.type == IT_DIAG) {
            if (!blocked_gate) {
                ++count;
                if (out) out->push_back((int)i);
            } else {
                blocked_diag = true;
            }
        } else if (it.type == IT_PHASE) {
            const bool ok = (it.bit < 0 || !nd[it.bit]) && (it.bit2 < 0 || !nd[it.bit2]) &&
                            (max_gates < 0 || gates < max_gates);
            if (ok) {
                ++count;
                ++gates;
                if (out) out->push_back((int)i);
            } else {
                if (it.bit >= 0) blocked[it.bit] = 1;
                if (it.bit2 >= 0) blocked[it.bit2] = 1;
            }
        } else {
            const bool two = it.bit2 >= 0;
            bool ok = !blocked[it.bit] && !blocked_diag && in_set[it.bit] &&
                      (max_gates < 0 || gates < max_gates);
            if (two) {
                const int code = (it.bit << 8) | it.bit2;
                const bool placed = pair == PAIR_ANY ||
                                    (pair >= 0 && (pair == code || (pair2 >= 0 && pair2 == code && it.pair_b)));
                ok = ok && !blocked[it.bit2] && in_set[it.bit2] && placed;
            }
            if (ok) {
                ++count;
                ++gates;
                if (out) out->push_back((int)i);
            } else {
                blocked[it.bit] = nd[it.bit] = 1;
                if (two) blocked[it.bit2] = nd[it.bit2] = 1;
                blocked_gate = true;
            }
        }
    }
    return count;
}

// Pending two-qubit gates with exactly one bit in the set: a tie-break that
// lets a greedy bit choice complete pairs (adding one bit alone enables none).
int half_pairs(const std::vector<ScanItem>& items, const std::vector<char>& done, const std::vector<char>& in_set) {
    int c = 0;
    for (size_t i = 0; i < items.size(); ++i)
        if (!done[i] && items[i].type == IT_GATE && items[i].bit2 >= 0 &&
            (in_set[items[i].bit] != in_set[items[i].bit2]))
            ++c;
    return c;
}

struct ScaleState {
    int h = 0;    // unnormalised Hadamards not yet compensated (each contributes sqrt 2)
    int sign = 1; // sign folded out of Inv
};

int64_t extract(int64_t x, const std::vector<int>& bits) {
    int64_t r = 0;
    for (size_t l = 0; l < bits.size(); ++l) r |= ((x >> bits[l]) & 1) << l;
    return r;
}

// Packs one stage's op list into fixed-slot sub-stages (see Stage).  Ops keep
// their order: each goes to the first free slot at or after the previous op's
// slot, and a new sub-stage (same layout, no exchange) starts when none fits.
// Hadamards collected in one mask act on distinct register bits and commute.
enum Slot {
    S_SEED = 0, S_FLIP_PRE, S_PHASE, S_MAT_PRE, S_H1, S_FLIP_MID, S_H2, S_MAT_POST, S_MAT4, S_MAT4B, S_D2B, S_D4B,
    S_SCALE, S_READ
};

Stage blank_sub(const HostStage& hs, int exchange) {
    Stage s{};
    int nrb = 0;
    for (int a = 0; a < kMaxRegBits; ++a) {
        s.rb[a] = hs.rb[a];
        if (hs.rb[a] >= 0) s.rbs[nrb++] = hs.rb[a];
    }
    std::sort(s.rbs, s.rbs + nrb);
    for (int a = nrb; a < kMaxRegBits; ++a) s.rbs[a] = -1;
    s.exchange = exchange;
    s.seed = s.flip_pre = s.flip_mid = s.read = -1;
    s.mat_pre_a = s.mat_post_a = s.d2b_a = -1;
    s.mat4 = s.mat4b = s.d4b_mat = -1;
    s.phase_first = s.phase_count = 0;
    for (int u = 0; u < kPhaseSlots; ++u) {
        s.phase_pm[u] = -1;
        s.phase_cnt[u] = 0;
        s.phase_ucnt[u] = 0;
        s.phase_tt[u] = s.phase_ut0[u] = s.phase_ut1[u] = -1;
        s.phase_ttm[u] = 0;
    }
    return s;
}

// Entries of the product table of `ops` over the label bits `mask`: entry ix is
// the product of the factors of the phases whose condition bits are all set in
// the pattern that deposits ix's bits at mask's positions.
template <typename Cond>
void tabulate(const std::vector<PhaseOp>& ops, uint64_t mask, Cond cond, std::vector<double>* twid) {
    int pos[64], m = 0;
    for (int b = 0; b < 64; ++b)
        if (mask >> b & 1) pos[m++] = b;
    for (uint64_t ix = 0; ix < (1ull << m); ++ix) {
        uint64_t pat = 0;
        for (int k = 0; k < m; ++k)
            if (ix >> k & 1) pat |= 1ull << pos[k];
        double c = 1.0, sn = 0.0;
        for (const PhaseOp& o : ops) {
            const uint64_t need = cond(o);
            if ((pat & need) != need) continue;
            const double fc = 1.0 + o.cm1, x = c;
            c = x * fc - sn * o.s;
            sn = x * o.s + sn * fc;
        }
        twid->push_back(c);
        twid->push_back(sn);
    }
}

// Finishes a sub-stage: its phases stored grouped by slot; in each slot the phases
// that go into product tables first (phase_ucnt), then the rest; then the mask of
// the steps.  The tile part of a slot (phases with no condition on the thread's
// label bits) is split into groups of phases tied by a shared tile-index bit, and
// the groups are packed, largest first, into at most two tables of at most
// kTwidBits index bits, each one of the pass's URefs while the pass has fewer
// than kMaxURefs; the thread part (no condition on the tile index) takes one
// table when its label bits fit.  A phase with no condition at all joins the
// tile part.  Phases of groups that fit no table stay in the kernel's loop.
void finish_sub(Stage& s, std::vector<PhaseOp>* table, std::vector<double>* twid, std::vector<URef>* urefs,
                size_t pass_urefs) {
    if (s.phase_count > 0) {
        auto b = table->begin() + s.phase_first, e = b + s.phase_count;
        std::stable_sort(b, e, [](const PhaseOp& x, const PhaseOp& y) { return x.slot < y.slot; });
        for (auto it = b; it != e; ++it) ++s.phase_cnt[it->slot];
        int32_t first = s.phase_first;
        for (int u = 0; u < kPhaseSlots; ++u) {
            const int cnt = s.phase_cnt[u];
            std::vector<PhaseOp> ops(table->begin() + first, table->begin() + first + cnt);
            // class of each phase: 0 / 1 the first / second tile table, 2 the thread
            // table, 3 the loop
            std::vector<int> cls(cnt, 3);
            // tile part: groups of phases joined by shared tile-index bits
            std::vector<int> tile_ix;
            for (int q = 0; q < cnt; ++q)
                if (ops[q].tmask == 0) tile_ix.push_back(q);
            std::vector<uint64_t> gmask;     // tile-index bits of each group
            std::vector<std::vector<int>> gmem;
            for (int q : tile_ix) {
                uint64_t m = (uint64_t)ops[q].fmask;
                std::vector<int> mem{q};
                for (size_t g = 0; g < gmask.size();) {
                    if (gmask[g] & m) {
                        m |= gmask[g];
                        mem.insert(mem.end(), gmem[g].begin(), gmem[g].end());
                        gmask.erase(gmask.begin() + g);
                        gmem.erase(gmem.begin() + g);
                    } else {
                        ++g;
                    }
                }
                gmask.push_back(m);
                gmem.push_back(mem);
            }
            std::vector<size_t> gorder(gmask.size());
            for (size_t g = 0; g < gorder.size(); ++g) gorder[g] = g;
            std::stable_sort(gorder.begin(), gorder.end(), [&](size_t x, size_t y) {
                return __builtin_popcountll(gmask[x]) > __builtin_popcountll(gmask[y]);
            });
            uint64_t umask[2] = {0, 0};
            bool used[2] = {false, false};
            const size_t room = (size_t)kMaxURefs - (urefs->size() - pass_urefs);
            for (size_t g : gorder) {
                for (int t = 0; t < 2 && (size_t)t < room; ++t) {
                    if (__builtin_popcountll(umask[t] | gmask[g]) > kTwidBits) continue;
                    umask[t] |= gmask[g];
                    used[t] = true;
                    for (int q : gmem[g]) cls[q] = t;
                    break;
                }
            }
            // thread part
            uint32_t tmask = 0;
            int nthr = 0;
            for (int q = 0; q < cnt; ++q)
                if (ops[q].fmask == 0 && ops[q].tmask != 0) {
                    tmask |= ops[q].tmask;
                    ++nthr;
                }
            if (nthr > 0 && __builtin_popcount(tmask) <= kTwidBits)
                for (int q = 0; q < cnt; ++q)
                    if (ops[q].fmask == 0 && ops[q].tmask != 0) cls[q] = 2;
            for (int t = 0; t < 2; ++t) {
                if (!used[t]) continue;
                std::vector<PhaseOp> part;
                for (int q = 0; q < cnt; ++q)
                    if (cls[q] == t) part.push_back(ops[q]);
                (t == 0 ? s.phase_ut0 : s.phase_ut1)[u] = (int32_t)(urefs->size() - pass_urefs);
                urefs->push_back({(int32_t)(twid->size() / 2), 0, (int64_t)umask[t]});
                tabulate(part, umask[t], [](const PhaseOp& o) { return (uint64_t)o.fmask; }, twid);
            }
            if (nthr > 0 && __builtin_popcount(tmask) <= kTwidBits) {
                std::vector<PhaseOp> part;
                for (int q = 0; q < cnt; ++q)
                    if (cls[q] == 2) part.push_back(ops[q]);
                s.phase_tt[u] = (int32_t)(twid->size() / 2);
                s.phase_ttm[u] = tmask;
                tabulate(part, tmask, [](const PhaseOp& o) { return (uint64_t)o.tmask; }, twid);
            }
            // tabulated phases first (any order), then the loop's
            int w = first;
            for (int pass = 0; pass < 2; ++pass)
                for (int q = 0; q < cnt; ++q)
                    if ((cls[q] < 3) == (pass == 0)) (*table)[w++] = ops[q];
            s.phase_ucnt[u] = 0;
            for (int q = 0; q < cnt; ++q) s.phase_ucnt[u] += cls[q] < 3;
            first += cnt;
        }
    }
    s.steps = (s.exchange ? ST_EXCHANGE : 0) | (s.seed >= 0 ? ST_SEED : 0) | (s.flip_pre >= 0 ? ST_FLIP_PRE : 0) |
              (s.phase_count > 0 ? ST_PHASE : 0) | (s.mat_pre_a >= 0 ? ST_MAT_PRE : 0) | (s.hmask1 ? ST_H1 : 0) |
              (s.flip_mid >= 0 ? ST_FLIP_MID : 0) | (s.hmask2 ? ST_H2 : 0) | (s.mat_post_a >= 0 ? ST_MAT_POST : 0) |
              (s.mat4 >= 0 ? ST_MAT4 : 0) | (s.d2b_a >= 0 ? ST_D2B : 0) | (s.d4b_mat >= 0 ? ST_D4B : 0) |
              (s.scale ? ST_SCALE : 0) | (s.read >= 0 ? ST_READ : 0) | (s.mat4b >= 0 ? ST_MAT4B : 0);
}

// A phase joins the accumulator slot of its register bits (the register bits of
// its qubits in this layout), or opens a new one; its other local bits become
// conditions on the thread's part of the label.
int place_phase(Stage& s, int cursor, const HostPhase& h, const HostStage& hs, std::vector<PhaseOp>* table) {
    if (cursor > S_PHASE) return -1;
    int pm = 0;
    uint32_t tmask = 0;
    for (int l : {h.la, h.lb}) {
        if (l < 0) continue;
        int a = -1;
        for (int q = 0; q < kMaxRegBits; ++q)
            if (hs.rb[q] == l) a = q;
        if (a >= 0)
            pm |= 1 << a;
        else
            tmask |= 1u << l;
    }
    int slot = -1;
    for (int u = 0; u < kPhaseSlots && slot < 0; ++u)
        if (s.phase_pm[u] == pm) slot = u;
    for (int u = 0; u < kPhaseSlots && slot < 0; ++u)
        if (s.phase_pm[u] < 0) {
            s.phase_pm[u] = pm;
            slot = u;
        }
    if (slot < 0) return -1;
    if (s.phase_count == 0) s.phase_first = (int32_t)table->size();
    table->push_back({slot, tmask, h.fmask, h.c - 1.0, h.s});
    ++s.phase_count;
    return S_PHASE;
}

int place(Stage& s, int cursor, const Op& o) {
    switch (o.kind) {
    case OP_SEED:
        if (cursor <= S_SEED && s.seed < 0) { s.seed = o.arg; return S_SEED; }
        return -1;
    case OP_FLIP:
        if (cursor <= S_FLIP_PRE && s.flip_pre < 0) { s.flip_pre = o.arg; return S_FLIP_PRE; }
        if (cursor <= S_FLIP_MID && s.flip_mid < 0) { s.flip_mid = o.arg; return S_FLIP_MID; }
        return -1;
    case OP_MAT:
        if (cursor <= S_MAT_PRE && s.mat_pre_a < 0) { s.mat_pre_a = o.a; s.mat_pre = o.arg; return S_MAT_PRE; }
        if (cursor <= S_MAT_POST && s.mat_post_a < 0) { s.mat_post_a = o.a; s.mat_post = o.arg; return S_MAT_POST; }
        return -1;
    case OP_H:
        if (cursor <= S_H1 && !(s.hmask1 >> o.a & 1)) { s.hmask1 |= 1 << o.a; return S_H1; }
        if (cursor <= S_H2 && !(s.hmask2 >> o.a & 1)) { s.hmask2 |= 1 << o.a; return S_H2; }
        return -1;
    case OP_D2BWD:
        if (cursor <= S_D2B && s.d2b_a < 0) {
            s.d2b_a = o.a; s.d2b_mat = o.arg; s.d2b_gslot = o.gslot; s.d2b_gscale = o.gscale;
            return S_D2B;
        }
        return -1;
    case OP_MAT4:
        if (o.a == 0 && cursor <= S_MAT4 && s.mat4 < 0) { s.mat4 = o.arg; return S_MAT4; }
        if (o.a == 2 && cursor <= S_MAT4B && s.mat4b < 0) { s.mat4b = o.arg; return S_MAT4B; }
        return -1;
    case OP_D4BWD:
        if (cursor <= S_D4B && s.d4b_mat < 0) {
            s.d4b_mat = o.arg; s.d4b_gslot = o.gslot; s.d4b_gscale = o.gscale;
            return S_D4B;
        }
        return -1;
    case OP_SCALE:
        if (cursor <= S_SCALE && !s.scale) { s.scale = 1; return S_SCALE; }
        return -1;
    case OP_READ:
        if (cursor <= S_READ && s.read < 0) { s.read = o.arg; return S_READ; }
        return -1;
    default:
        return -1;
    }
}

// LDS lane map of a layout that moves through LDS only (neither the first nor the
// last of its pass).  The slot swizzle XORs each 2^W-slot group of a label into
// its low W bits, so local bit p lands on swizzle bit p mod W; lanes that share
// one LDS access cycle differ in the thread's low bits, and they hit distinct
// banks when thread bit i sits on a local bit of residue i (W = 4 for 16-byte,
// 5 for 8-byte amplitudes).  The ascending map already does that for most
// layouts; one whose register bits take the bit of residue i that the ascending
// map would use gets, per residue, the lowest free local bit of that residue.
// Returns false (ascending map kept) when that holds already or a residue has no
// free bit.
bool choose_lanes(const HostStage& hs, int k, int W, int32_t* nlanes, uint32_t* lanes, uint32_t* rest) {
    uint32_t reg = 0;
    for (int a = 0; a < kMaxRegBits; ++a)
        if (hs.rb[a] >= 0) reg |= 1u << hs.rb[a];
    std::vector<int> fr;
    for (int l = 0; l < k; ++l)
        if (!(reg >> l & 1)) fr.push_back(l);
    if ((int)fr.size() < W) return false;
    bool ordered = true;
    for (int i = 0; i < W; ++i) ordered = ordered && fr[i] % W == i;
    if (ordered) return false;
    uint32_t pk = 0, used = 0;
    for (int i = 0; i < W; ++i) {
        int pick = -1;
        for (int l : fr)
            if (l % W == i && !(used >> l & 1)) {
                pick = l;
                break;
            }
        if (pick < 0) return false;
        used |= 1u << pick;
        pk |= (uint32_t)pick << (4 * i);
    }
    uint32_t r = 0;
    for (int l : fr)
        if (!(used >> l & 1)) r |= 1u << l;
    *nlanes = W;
    *lanes = pk;
    *rest = r;
    return true;
}

std::vector<Stage> pack_stage(const HostStage& hs, const std::vector<HostPhase>& phases, std::vector<PhaseOp>* table,
                              std::vector<double>* twid, std::vector<URef>* urefs, size_t pass_urefs) {
    std::vector<Stage> subs;
    Stage cur = blank_sub(hs, 1);
    int cursor = 0;
    auto put = [&](const Op& o) {
        return o.kind == OP_PHASE ? place_phase(cur, cursor, phases[o.arg], hs, table) : place(cur, cursor, o);
    };
    for (const Op& o : hs.ops) {
        int slot = put(o);
        if (slot < 0) {
            finish_sub(cur, table, twid, urefs, pass_urefs);
            subs.push_back(cur);
            cur = blank_sub(hs, 0);
            cursor = 0;
            slot = put(o);
        }
        cursor = slot;
    }
    finish_sub(cur, table, twid, urefs, pass_urefs);
    subs.push_back(cur);
    return subs;
}

// A pass's items on local tile bits.  A SWAP whose qubits are both non-carrier
// tile bits moves no data: from its position on, the two local bits stand for
// each other's qubits, and the tile is written back with the two state bits
// exchanged (Pass::stpos).  Such SWAPs leave the item list; every other item
// keeps the local bits and the read->state map in effect at its position.
struct LocalPass {
    std::vector<ScanItem> items;
    std::vector<int> src;                // index into the pass's selection of each item
    std::vector<int> map_id;             // entry of `maps` in effect at each item
    std::vector<std::vector<int>> maps;  // local bit -> state bit; maps[0] when read, back() when written
};

struct Compiler {
    Plan* plan;
    Instance* in;
    bool backward;
    int k, C, RB;
    int RBITS;  // register bits of the kernel instance (RB may be smaller for tiny tiles)
    // cut decisions depend only on the structure (nq, tiling, item kinds and bits,
    // what is done); instances of a batch often share it
    std::map<std::string, std::vector<int>>* cut_cache = nullptr;
    // the large-stride tile-bit preference of this compile (Tiling::page_cap, or 0
    // where that preference would cost passes)
    int pcap = 0;

    std::vector<int> free_bits(const std::vector<int>& tbits) const {
        std::vector<char> used(in->nq, 0);
        for (int b : tbits) used[b] = 1;
        std::vector<int> f;
        for (int b = 0; b < in->nq; ++b)
            if (!used[b]) f.push_back(b);
        return f;
    }

    int add_flip(const std::vector<int>& tbits, int64_t x, int slot) {
        Flip f;
        f.j = (int32_t)extract(x, tbits);
        f.tile = extract(x, free_bits(tbits));
        f.slot = slot;
        plan->flips.push_back(f);
        return (int)plan->flips.size() - 1;
    }

    // Stage planning inside one pass.  `items` are the pass's primitives in
    // scheduled order with bits given as local tile bits.  A stage holds at most
    // two disjoint ordered pairs of two-qubit gate bits, on register bits 0 and 1
    // and on register bits 2 and 3.
    std::vector<std::pair<std::vector<int>, std::vector<int>>> plan_stages(
        const std::vector<ScanItem>& items) const {
        const int n = (int)items.size();
        std::vector<char> done(n, 0);
        int left = n;
        auto io_ok = [&](int lb) { return (k - C >= RB) ? lb >= C : true; };
        std::vector<std::pair<std::vector<int>, std::vector<int>>> stages;
        bool first = true;
        while (left > 0) {
            std::vector<int> pairs;  // ordered pairs of the pending two-qubit gates
            std::set<int> need;
            for (int i = 0; i < n; ++i) {
                if (done[i] || items[i].type != IT_GATE) continue;
                need.insert(items[i].bit);
                if (items[i].bit2 >= 0) {
                    need.insert(items[i].bit2);
                    const int pr = (items[i].bit << 8) | items[i].bit2;
                    if (std::find(pairs.begin(), pairs.end(), pr) == pairs.end()) pairs.push_back(pr);
                }
            }
            // which pending pairs the second register pair may take (every pending
            // gate on it has a kernel step for register bits 2 and 3)
            std::vector<char> pb(pairs.size(), 1);
            for (int i = 0; i < n; ++i) {
                if (done[i] || items[i].type != IT_GATE || items[i].bit2 < 0) continue;
                const int pr = (items[i].bit << 8) | items[i].bit2;
                const size_t q = std::find(pairs.begin(), pairs.end(), pr) - pairs.begin();
                pb[q] = pb[q] && items[i].pair_b;
            }
            auto disjoint = [](int x, int y) {
                return (x >> 8) != (y >> 8) && (x >> 8) != (y & 255) && (x & 255) != (y >> 8) &&
                       (x & 255) != (y & 255);
            };
            // Does everything left fit in one stage that can also store?
            bool fits = (int)need.size() <= RB &&
                        (pairs.size() <= 1 ||
                         (pairs.size() == 2 && RB >= 4 && disjoint(pairs[0], pairs[1]) && (pb[0] || pb[1])));
            for (int b : need) fits = fits && io_ok(b);
            std::vector<int> rb;
            int pair = PAIR_NONE, pair2 = PAIR_NONE;
            if (fits) {
                if (pairs.size() == 2) {
                    pair = pb[1] ? pairs[0] : pairs[1];
                    pair2 = pb[1] ? pairs[1] : pairs[0];
                    rb = {pair >> 8, pair & 255, pair2 >> 8, pair2 & 255};
                } else if (!pairs.empty()) {
                    pair = pairs[0];
                    rb = {pair >> 8, pair & 255};
                }
                for (int b : need)
                    if (std::find(rb.begin(), rb.end(), b) == rb.end()) rb.push_back(b);
                for (int b = k - 1; b >= 0 && (int)rb.size() < RB; --b)
                    if (io_ok(b) && std::find(rb.begin(), rb.end(), b) == rb.end()) rb.push_back(b);
            } else {
                // options: no two-qubit gate, one of the first few pending pairs, or two
                // disjoint ones (the first on register bits 0 and 1, the second on 2 and 3)
                std::vector<std::pair<int, int>> options = {{PAIR_NONE, PAIR_NONE}};
                const size_t nopt = std::min<size_t>(pairs.size(), 4);
                for (size_t q = 0; q < nopt; ++q) options.push_back({pairs[q], PAIR_NONE});
                if (RB >= 4)
                    for (size_t q0 = 0; q0 < nopt; ++q0)
                        for (size_t q1 = q0 + 1; q1 < nopt; ++q1)
                            if (disjoint(pairs[q0], pairs[q1]) && (pb[q0] || pb[q1]))
                                options.push_back(pb[q1] ? std::make_pair(pairs[q0], pairs[q1])
                                                         : std::make_pair(pairs[q1], pairs[q0]));
                int best_gain = -1;
                for (const auto& opt : options) {
                    std::vector<int> r;
                    bool usable = true;
                    for (int pr : {opt.first, opt.second}) {
                        if (pr < 0) continue;
                        const int b1 = pr >> 8, b2 = pr & 255;
                        if (first && (!io_ok(b1) || !io_ok(b2))) usable = false;
                        r.push_back(b1);
                        r.push_back(b2);
                    }
                    if (!usable) continue;
                    while ((int)r.size() < RB) {
                        int best = -1, bg = -1, best_pref = -1;
                        for (int b = 0; b < k; ++b) {
                            if (std::find(r.begin(), r.end(), b) != r.end()) continue;
                            if (first && !io_ok(b)) continue;
                            std::vector<char> in_set(k, 0);
                            for (int x : r) in_set[x] = 1;
                            in_set[b] = 1;
                            int g = scan(items, done, in_set, k, -1, nullptr, opt.first, opt.second);
                            // first stage: prefer high bits; later: bits that cannot be
                            // stored from (low carriers) first, then low bits
                            int pref = first ? b : ((!io_ok(b) ? 1000 : 0) + (k - b));
                            if (g > bg || (g == bg && pref > best_pref)) {
                                best = b;
                                bg = g;
                                best_pref = pref;
                            }
                        }
                        if (best < 0) break;
                        r.push_back(best);
                    }
                    std::vector<char> in_set(k, 0);
                    for (int x : r) in_set[x] = 1;
                    const int g = scan(items, done, in_set, k, -1, nullptr, opt.first, opt.second);
                    if (g > best_gain) {
                        best_gain = g;
                        rb = r;
                        pair = opt.first;
                        pair2 = opt.second;
                    }
                }
            }
            std::vector<char> in_set(k, 0);
            for (int r : rb) in_set[r] = 1;
            std::vector<int> sel;
            scan(items, done, in_set, k, -1, &sel, pair, pair2);
            for (int i : sel) done[i] = 1;
            left -= (int)sel.size();
            stages.push_back({rb, sel});
            first = false;
            if (fits) break;
        }
        bool last_ok = !stages.empty();
        if (last_ok)
            for (int r : stages.back().first) last_ok = last_ok && io_ok(r);
        if (!last_ok) {
            std::vector<int> rb;
            for (int b = k - 1; b >= 0 && (int)rb.size() < RB; --b)
                if (io_ok(b)) rb.push_back(b);
            stages.push_back({rb, {}});
        }
        return stages;
    }

    // Tile bits of the next pass: the carriers, then greedily the bits that let
    // the most pending primitives run; returns the primitives the pass takes.
    std::vector<int> choose_tile(const std::vector<ScanItem>& items, const std::vector<char>& done,
                                 std::vector<int>* sel) const {
        const int nq = in->nq;
        const int max_gates = plan->tiling.fuse ? -1 : 1;
        std::vector<char> in_t(nq, 0);
        std::vector<int> t;
        for (int b = 0; b < C; ++b) {
            in_t[b] = 1;
            t.push_back(b);
        }
        // Among bits of equal gain, take bits at byte strides of 2 MiB or more (each
        // doubles the pages a tile touches) first while the tile has fewer than
        // page_cap of them, so that no later pass is left with all of them.
        const int pbit = kPageByteBit - (plan->prec == PK_FP64 ? 4 : 3);
        while ((int)t.size() < k) {
            int best = -1, best_gain = -1;
            int npage = 0;
            for (int b : t) npage += b >= pbit;
            std::vector<int> cand;
            if (pcap > 0 && npage < pcap)
                for (int b = nq - 1; b >= pbit; --b) cand.push_back(b);
            for (int b = 0; b < nq; ++b)
                if (!(pcap > 0 && npage < pcap && b >= pbit)) cand.push_back(b);
            for (int b : cand) {
                if (in_t[b]) continue;
                in_t[b] = 1;
                int g = 2 * scan(items, done, in_t, nq, max_gates, nullptr) + half_pairs(items, done, in_t);
                in_t[b] = 0;
                if (g > best_gain) {
                    best = b;
                    best_gain = g;
                }
            }
            in_t[best] = 1;
            t.push_back(best);
        }
        std::sort(t.begin(), t.end());
        sel->clear();
        scan(items, done, in_t, nq, max_gates, sel);
        if (sel->empty()) {
            // the greedy choice enables nothing (the half-pair tie-break can lead it
            // away from the first pending two-qubit gate): build the tile around the
            // first pending gate instead, which nothing earlier can block
            int first = -1;
            for (size_t i = 0; i < items.size() && first < 0; ++i)
                if (!done[i] && items[i].type == IT_GATE) first = (int)i;
            std::fill(in_t.begin(), in_t.end(), 0);
            t.clear();
            for (int b = 0; b < C; ++b) {
                in_t[b] = 1;
                t.push_back(b);
            }
            if (first >= 0)
                for (int b : {items[first].bit, items[first].bit2})
                    if (b >= 0 && !in_t[b]) {
                        in_t[b] = 1;
                        t.push_back(b);
                    }
            for (int b = 0; b < nq && (int)t.size() < k; ++b)
                if (!in_t[b]) {
                    in_t[b] = 1;
                    t.push_back(b);
                }
            std::sort(t.begin(), t.end());
            scan(items, done, in_t, nq, max_gates, sel);
        }
        return t;
    }

    LocalPass local_pass(const std::vector<ScanItem>& items, const std::vector<int>& t,
                         const std::vector<int>& sel, size_t count) const {
        LocalPass lp;
        std::vector<int> local_of(in->nq, -1);
        for (int l = 0; l < (int)t.size(); ++l) local_of[t[l]] = l;
        lp.maps.push_back(t);
        for (size_t j = 0; j < count; ++j) {
            const ScanItem& it = items[sel[j]];
            const int l1 = it.bit >= 0 ? local_of[it.bit] : -1;
            const int l2 = it.bit2 >= 0 ? local_of[it.bit2] : -1;
            if (it.type == IT_GATE && it.swap && l1 >= C && l2 >= C) {
                std::swap(local_of[it.bit], local_of[it.bit2]);
                std::vector<int> m = lp.maps.back();
                std::swap(m[l1], m[l2]);
                lp.maps.push_back(m);
                continue;
            }
            ScanItem li{it.type, it.type == IT_DIAG ? -1 : l1, l2, it.swap, it.pair_b};
            lp.items.push_back(li);
            lp.src.push_back((int)j);
            lp.map_id.push_back((int)lp.maps.size() - 1);
        }
        return lp;
    }

    // Cost of finishing the schedule greedily from `done`: (passes, sum of
    // squared stage counts).  Used to compare cuts of the current pass.
    std::pair<int, int> greedy_rest(const std::vector<ScanItem>& items, std::vector<char> done, int left) const {
        int passes = 0, cost = 0;
        std::vector<int> sel;
        while (left > 0) {
            auto t = choose_tile(items, done, &sel);
            int ns = (int)plan_stages(local_pass(items, t, sel, sel.size()).items).size();
            for (int i : sel) done[i] = 1;
            left -= (int)sel.size();
            ++passes;
            cost += ns * ns;
        }
        return {passes, cost};
    }

    // The pass may leave gates on some of its tile bits to later passes: a scan
    // with those bits removed still respects every ordering constraint.  Bits
    // are dropped greedily while that lowers (pass count, sum of squared stage
    // counts) of the whole remaining schedule, so one pass does not take all
    // the stages its tile allows when a later pass can absorb them for free.
    std::vector<int> choose_cut(const std::vector<ScanItem>& items, const std::vector<char>& done, int left,
                                const std::vector<int>& t, const std::vector<int>& sel) const {
        if ((int)sel.size() == left || !plan->tiling.fuse) return sel;
        const int nq = in->nq;
        std::string key;
        if (cut_cache) {
            int32_t hdr[5] = {nq, k, C, RB, pcap};
            key.append((const char*)hdr, sizeof hdr);
            for (size_t i = 0; i < items.size(); ++i) {
                key.push_back((char)(items[i].type * 4 + (items[i].swap ? 2 : 0) + (items[i].pair_b ? 1 : 0)));
                key.push_back((char)items[i].bit);
                key.push_back((char)items[i].bit2);
            }
            key.append(done.begin(), done.end());
            auto it = cut_cache->find(key);
            if (it != cut_cache->end()) return it->second;
        }
        auto cost_of = [&](const std::vector<int>& s) {
            std::vector<char> d = done;
            for (int i : s) d[i] = 1;
            int ns = (int)plan_stages(local_pass(items, t, s, s.size()).items).size();
            auto rest = greedy_rest(items, d, left - (int)s.size());
            return std::pair<int, int>{1 + rest.first, ns * ns + rest.second};
        };
        std::vector<char> in_t(nq, 0);
        for (int b : t) in_t[b] = 1;
        std::vector<int> best = sel;
        auto best_cost = cost_of(sel);
        for (;;) {
            std::vector<int> round_best;
            auto round_cost = best_cost;
            int drop = -1;
            for (int b : t) {
                if (!in_t[b]) continue;
                bool used = false;
                for (int i : best)
                    used = used || (items[i].type == IT_GATE && (items[i].bit == b || items[i].bit2 == b));
                if (!used) continue;
                in_t[b] = 0;
                std::vector<int> s;
                scan(items, done, in_t, nq, -1, &s);
                in_t[b] = 1;
                if (s.empty()) continue;
                auto c = cost_of(s);
                if (c < round_cost) {
                    round_cost = c;
                    round_best = s;
                    drop = b;
                }
            }
            if (drop < 0) break;
            in_t[drop] = 0;
            best = round_best;
            best_cost = round_cost;
        }
        if (cut_cache) (*cut_cache)[key] = best;
        return best;
    }

    // Local numbering of the tile bits.  The carriers stay local bits 0..C-1;
    // the rest are ordered so that the lowest non-carrier local bits -- the ones
    // the lanes of a wave cover next to the carriers when the first and last
    // stage read and write HBM -- are state bits whose byte stride is below
    // 4 KiB or at least 4 MiB.  Measured on MI355X: a wave-wide load whose lane
    // groups lie 4 KiB..2 MiB apart streams up to a third slower.  The order
    // only relabels local bits, so the state computed is the same.
    void order_lanes(std::vector<int>* t) const {
        const int ebits = plan->prec == PK_FP64 ? 4 : 3;  // log2 bytes per amplitude
        auto good = [&](int b) { return b + ebits < 12 || b + ebits >= 22; };
        std::stable_sort(t->begin() + C, t->end(), [&](int x, int y) {
            if (good(x) != good(y)) return good(x);
            return x < y;
        });
    }

    // Passes the tile and cut choices make for `items` with large-stride preference p.
    int count_passes(const std::vector<ScanItem>& items, int p) {
        const int saved = pcap;
        pcap = p;
        std::vector<char> done(items.size(), 0);
        int left = (int)items.size(), passes = 0;
        while (left > 0) {
            std::vector<int> sel;
            std::vector<int> t = choose_tile(items, done, &sel);
            sel = choose_cut(items, done, left, t, sel);
            for (int i : sel) done[i] = 1;
            left -= (int)sel.size();
            ++passes;
        }
        pcap = saved;
        return passes;
    }

    void compile(const std::vector<Prim>& prims, std::vector<HostPass>* out) {
        const int nq = in->nq;
        const int n = (int)prims.size();
        std::vector<ScanItem> items(n);
        for (int i = 0; i < n; ++i) {
            const Prim& p = prims[i];
            if (p.kind != Prim::GATE)
                items[i] = {IT_DIAG, -1, -1};
            else
                items[i] = {p.gk == Prim::GPHASE ? IT_PHASE : IT_GATE, p.bit, p.bit2, p.gk == Prim::GSWAP,
                            !(backward && p.gk == Prim::GD4)};
        }
        // The large-stride preference only breaks ties between equally useful tile
        // bits; where it nevertheless costs passes (two-qubit gates on neighbouring
        // qubits, whose single bits are all "half useful"), this compile drops it.
        pcap = plan->tiling.page_cap;
        if (pcap > 0 && n > 0 && count_passes(items, 0) < count_passes(items, pcap)) pcap = 0;
        std::vector<char> done(n, 0);
        int left = n;
        ScaleState sc;
        int pass_no = 0;
        do {
            std::vector<int> sel;
            std::vector<int> t = choose_tile(items, done, &sel);
            sel = choose_cut(items, done, left, t, sel);
            if (plan->tiling.lane_order == 1) order_lanes(&t);
            for (int i : sel) done[i] = 1;
            left -= (int)sel.size();
            const bool last = (left == 0);

            // --- local items and stages
            const LocalPass lp = local_pass(items, t, sel, sel.size());
            auto st = plan_stages(lp.items);
            if (lp.maps.size() > 1 && st.size() == 1) {
                // The tile is written with another map than it was read with, so
                // amplitudes change threads: in place, every thread's loads must
                // complete before any thread stores.  The barrier of an LDS
                // exchange guarantees that; a one-stage pass has none, so it gets
                // a second stage in a store layout.
                std::vector<int> rb;
                for (int b = k - 1; b >= 0 && (int)rb.size() < RB; --b)
                    if (k - C < RB || b >= C) rb.push_back(b);
                st.push_back({rb, {}});
            }
            std::vector<int> fpos(nq, -1);  // position of each bit outside the tile in the tile index
            {
                std::vector<char> in_t(nq, 0);
                for (int b : t) in_t[b] = 1;
                int f = 0;
                for (int b = 0; b < nq; ++b)
                    if (!in_t[b]) fpos[b] = f++;
            }

            HostPass hp;
            hp.k = k;
            hp.tbits = t;
            hp.sbits = lp.maps.back();
            hp.ntiles = (int64_t)1 << (nq - k);
            hp.rbits = RBITS;
            hp.kmax = std::max(k, RBITS + kWaveBits);
            if (pass_no == 0) hp.flags |= PASS_FIRST | (backward ? PASS_SEED_V1 : 0);
            if (last) hp.flags |= PASS_LAST | (backward ? PASS_SKIP_V0 : 0);
            for (size_t s = 0; s < st.size(); ++s) {
                HostStage hs;
                for (int a = 0; a < kMaxRegBits; ++a) hs.rb[a] = a < (int)st[s].first.size() ? st[s].first[a] : -1;
                auto reg_of = [&](int lb) {
                    for (int a = 0; a < kMaxRegBits; ++a)
                        if (hs.rb[a] == lb) return a;
                    return -1;
                };
                if (s == 0 && pass_no == 0 && backward) {
                    for (size_t m = 0; m < in->marked.size(); ++m) {
                        Op o{};
                        o.kind = OP_SEED;
                        o.arg = add_flip(t, in->marked[m], (int)(in - plan->inst.data()));
                        hs.ops.push_back(o);
                    }
                }
                for (int li : st[s].second) {
                    const Prim& p = prims[sel[lp.src[li]]];
                    const ScanItem& it = lp.items[li];
                    const std::vector<int>& map = lp.maps[lp.map_id[li]];
                    if (p.kind == Prim::ORACLE) {
                        for (int64_t x : in->marked) {
                            Op o{};
                            o.kind = OP_FLIP;
                            o.arg = add_flip(map, x, 0);
                            hs.ops.push_back(o);
                        }
                    } else if (p.kind == Prim::INV) {
                        sc.sign = -sc.sign;
                        Op o{};
                        o.kind = OP_FLIP;
                        o.arg = add_flip(map, 0, 0);
                        hs.ops.push_back(o);
                    } else if (p.gk == Prim::GPHASE) {
                        // the adjoint of a phase is its conjugate
                        HostPhase h{it.bit, it.bit2, 0, -1, -1, p.pc, backward ? -p.ps : p.ps};
                        if (it.bit < 0) h.fmask |= (int64_t)1 << fpos[p.bit];
                        if (it.bit2 < 0) h.fmask |= (int64_t)1 << fpos[p.bit2];
                        h.b1 = it.bit >= 0 ? t[it.bit] : p.bit;
                        h.b2 = it.bit2 >= 0 ? t[it.bit2] : p.bit2;
                        Op o{};
                        o.kind = OP_PHASE;
                        o.arg = (int32_t)hp.phases.size();
                        hp.phases.push_back(h);
                        hs.ops.push_back(o);
                    } else {
                        Op o{};
                        o.a = reg_of(it.bit);
                        if (p.gk == Prim::GH) {
                            o.kind = OP_H;
                            ++sc.h;
                        } else if (p.gk == Prim::GMAT) {
                            o.kind = OP_MAT;
                            o.arg = 2 * p.idx + (backward ? 1 : 0);
                        } else if (p.gk == Prim::GMAT4 || p.gk == Prim::GD4 || p.gk == Prim::GSWAP) {
                            // the stage holds the pair on register bits 0 (is1) and 1 (is2),
                            // or, as its second pair, on bits 2 and 3
                            const int r2 = reg_of(it.bit2);
                            if (!((o.a == 0 && r2 == 1) || (o.a == 2 && r2 == 3)))
                                throw std::logic_error("two-qubit register pair");
                            if (backward && p.gk == Prim::GD4 && o.a != 0)
                                throw std::logic_error("backward D4 on the second register pair");
                            if (p.gk == Prim::GMAT4 || p.gk == Prim::GSWAP) {
                                o.kind = OP_MAT4;
                                o.arg = 2 * p.idx + (backward ? 1 : 0);
                            } else if (!backward) {
                                o.kind = OP_MAT4;
                                o.arg = 2 * plan->n_static4 + 5 * p.idx;
                            } else {
                                o.kind = OP_D4BWD;
                                o.arg = 2 * plan->n_static4 + 5 * p.idx;  // D, D^H and the three derivatives
                                o.gscale = (float)std::ldexp(1.0, -sc.h);
                                o.gslot = (int32_t)plan->n_gpart;
                                plan->d2_grad.push_back({p.param, plan->n_gpart, hp.ntiles});
                                plan->n_gpart += 3 * hp.ntiles;
                            }
                        } else if (!backward) {
                            o.kind = OP_MAT;
                            o.arg = 2 * plan->n_static + 5 * p.idx;
                        } else {
                            o.kind = OP_D2BWD;
                            o.arg = 2 * plan->n_static + 5 * p.idx;  // D, D^H, dD/dalpha, dD/dbeta, dD/dgamma
                            o.gscale = (float)std::ldexp(1.0, -sc.h);
                            o.gslot = (int32_t)plan->n_gpart;
                            plan->d2_grad.push_back({p.param, plan->n_gpart, hp.ntiles});
                            plan->n_gpart += 3 * hp.ntiles;
                        }
                        hs.ops.push_back(o);
                    }
                }
                hp.stages.push_back(hs);
            }
            // --- deferred scaling: powers of two each pass, the rest at the end
            HostStage& fin = hp.stages.back();
            if (last) {
                double s = std::ldexp((double)sc.sign, -(sc.h / 2));
                if (sc.h % 2) s *= std::sqrt(0.5);
                if (backward) s *= 2.0;  // grad psi_in = 2 lambda_0
                hp.scale = s;
                sc = ScaleState{};
            } else {
                int e = sc.h / 2;
                hp.scale = std::ldexp(1.0, -e);
                sc.h -= 2 * e;
            }
            if (hp.scale != 1.0) {
                Op o{};
                o.kind = OP_SCALE;
                fin.ops.push_back(o);
            }
            if (last && !backward) {
                for (size_t m = 0; m < in->marked.size(); ++m) {
                    Op o{};
                    o.kind = OP_READ;
                    o.arg = add_flip(lp.maps.back(), in->marked[m], in->read_base + (int)m);
                    fin.ops.push_back(o);
                }
            }
            hp.uref_begin = (int)plan->urefs.size();
            const int lane_w = plan->prec == PK_FP64 ? 4 : 5;
            for (size_t si = 0; si < hp.stages.size(); ++si) {
                const HostStage& hs = hp.stages[si];
                std::vector<Stage> sub =
                    pack_stage(hs, hp.phases, &plan->phases, &plan->twid, &plan->urefs, (size_t)hp.uref_begin);
                int32_t nl = 0;
                uint32_t ln = 0, lr = 0;
                if (plan->lane_maps && si > 0 && si + 1 < hp.stages.size() &&
                    choose_lanes(hs, hp.k, lane_w, &nl, &ln, &lr))
                    for (Stage& st : sub) {
                        st.nlanes = nl;
                        st.lanes = ln;
                        st.lanes_rest = lr;
                    }
                hp.subs.insert(hp.subs.end(), sub.begin(), sub.end());
            }
            hp.nuref = (int)plan->urefs.size() - hp.uref_begin;
            out->push_back(hp);
            ++pass_no;
        } while (left > 0);
    }
};

// CPHASE (k = 0: theta = pi, Sec. 4.2) or CPHASEK (theta = 2 pi / 2^k, Eq. cphasek):
// diag(1, 1, 1, e^{i theta}) on qubits is1, is2, a phase on the amplitudes whose
// two qubits are 1, with the exact factors at theta = pi and pi/2.
Prim phase_prim(int nq, int is1, int is2, int k) {
    double c = -1.0, sn = 0.0;
    if (k == 2) {
        c = 0.0;
        sn = 1.0;
    } else if (k > 2) {
        const double ph = 2.0 * M_PI * std::ldexp(1.0, -k);
        c = std::cos(ph);
        sn = std::sin(ph);
    }
    Prim pr{Prim::GATE, nq - is1, Prim::GPHASE, 0};
    pr.bit2 = nq - is2;
    pr.pc = c;
    pr.ps = sn;
    return pr;
}

// A fixed 4x4 operator in the basis |q_is1 q_is2> (Eq. resmat2), row-major
// (re, im); the plan keeps it and its adjoint.
Prim mat4_prim(Plan* plan, int nq, int is1, int is2, const double* m, Prim::GKind gk) {
    Prim pr{Prim::GATE, nq - is1, gk, plan->n_static4};
    pr.bit2 = nq - is2;
    for (int e = 0; e < 32; ++e) plan->static_mats4.push_back(m[e]);
    for (int a = 0; a < 4; ++a)  // adjoint
        for (int b = 0; b < 4; ++b) {
            plan->static_mats4.push_back(m[2 * (4 * b + a)]);
            plan->static_mats4.push_back(-m[2 * (4 * b + a) + 1]);
        }
    ++plan->n_static4;
    return pr;
}

const double kSwap4[32] = {1, 0, 0, 0, 0, 0, 0, 0,  0, 0, 0, 0, 1, 0, 0, 0,
                           0, 0, 1, 0, 0, 0, 0, 0,  0, 0, 0, 0, 0, 0, 1, 0};

std::string fmt(const char* f, long long a = 0, long long b = 0) {
    char buf[256];
    std::snprintf(buf, sizeof buf, f, a, b);
    return buf;
}

}  // namespace

int compile_plan(Plan* plan, const pk_problem* probs, int n_inst, int prec, std::string* err) {
    if (prec != PK_FP64 && prec != PK_FP32) {
        *err = "prec must be PK_FP64 or PK_FP32";
        return PK_EINVAL;
    }
    if (n_inst < 1 || !probs) {
        *err = "need at least one problem";
        return PK_EINVAL;
    }
    plan->prec = prec;
    plan->tiling = Tiling{default_tile_bits(prec), 4, 1, 0, default_reg_bits(prec), 1, default_page_cap(prec)};
    const int nq_max = prec == PK_FP64 ? 30 : 31;
    int64_t off = 0;
    int d2 = 0;
    for (int i = 0; i < n_inst; ++i) {
        const pk_problem& p = probs[i];
        Instance in;
        if (p.nq < 1 || p.nq > nq_max) {
            *err = fmt("instance %lld: nq=%lld out of range", i, p.nq);
            return PK_EINVAL;
        }
        in.nq = p.nq;
        in.off = off;
        off += (int64_t)1 << p.nq;
        if (p.n_gates < 0 || (p.n_gates > 0 && !p.gates)) {
            *err = fmt("instance %lld: bad gate array", i);
            return PK_EINVAL;
        }
        if (p.n_marked < 0 || p.n_marked > 64 || (p.n_marked > 0 && !p.marked)) {
            *err = fmt("instance %lld: marked set must hold 0..64 labels", i);
            return PK_EINVAL;
        }
        std::set<int64_t> seen;
        for (int64_t m = 0; m < p.n_marked; ++m) {
            int64_t x = p.marked[m];
            if (x < 0 || x >= ((int64_t)1 << p.nq)) {
                *err = fmt("instance %lld: marked label %lld out of range", i, x);
                return PK_EINVAL;
            }
            if (!seen.insert(x).second) {
                *err = fmt("instance %lld: duplicate marked label %lld", i, x);
                return PK_EINVAL;
            }
            in.marked.push_back(x);
        }
        in.d2_base = d2;
        for (int g = 0; g < p.n_gates; ++g) {
            const pk_gate& gt = p.gates[g];
            const bool two = gt.kind == PK_GATE_TWOOP || gt.kind == PK_GATE_CNOT || gt.kind == PK_GATE_CPHASE ||
                             gt.kind == PK_GATE_CPHASEK || gt.kind == PK_GATE_SWAP || gt.kind == PK_GATE_D4;
            if (gt.kind == PK_GATE_QFT || gt.kind == PK_GATE_QFT_NOSWAP) {
                if (gt.is2 != 0 || gt.k < 1 || gt.is1 < 1 || gt.is1 + gt.k - 1 > p.nq) {
                    *err = fmt("instance %lld gate %lld: QFT needs qubits is1 .. is1+k-1 within 1..nq and is2 = 0", i, g);
                    return PK_EINVAL;
                }
            } else if (!two && (gt.is2 != 0 || gt.k != 0)) {
                *err = fmt("instance %lld gate %lld: two-qubit fields must be 0", i, g);
                return PK_EINVAL;
            }
            if (two && (gt.is2 < 1 || gt.is2 > p.nq || gt.is2 == gt.is1)) {
                *err = fmt("instance %lld gate %lld: second qubit label out of 1..nq or equal to the first", i, g);
                return PK_EINVAL;
            }
            if (two && gt.kind != PK_GATE_CPHASEK && gt.k != 0) {
                *err = fmt("instance %lld gate %lld: k is only for CPHASEK", i, g);
                return PK_EINVAL;
            }
            if (gt.kind == PK_GATE_CPHASEK && (gt.k < 1 || gt.k > 62)) {
                *err = fmt("instance %lld gate %lld: CPHASEK needs k in 1..62", i, g);
                return PK_EINVAL;
            }
            bool needs_qubit = gt.kind == PK_GATE_ONEOP || gt.kind == PK_GATE_H || gt.kind == PK_GATE_D2 || two;
            if (needs_qubit && (gt.is1 < 1 || gt.is1 > p.nq)) {
                *err = fmt("instance %lld gate %lld: qubit label out of 1..nq", i, g);
                return PK_EINVAL;
            }
            Prim pr{};
            switch (gt.kind) {
            case PK_GATE_ONEOP:
                if (!finite8(gt.op, 8)) {
                    *err = fmt("instance %lld gate %lld: non-finite operator", i, g);
                    return PK_EINVAL;
                }
                if (!is_unitary(gt.op)) plan->backward_ok = false;
                pr = {Prim::GATE, p.nq - gt.is1, Prim::GMAT, plan->n_static};
                for (int e = 0; e < 8; ++e) plan->static_mats.push_back(gt.op[e]);
                // adjoint: (M^H)[a][b] = conj(M[b][a])
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        plan->static_mats.push_back(gt.op[2 * (2 * b + a)]);
                        plan->static_mats.push_back(-gt.op[2 * (2 * b + a) + 1]);
                    }
                ++plan->n_static;
                in.prims.push_back(pr);
                break;
            case PK_GATE_H:
                in.prims.push_back({Prim::GATE, p.nq - gt.is1, Prim::GH, 0});
                break;
            case PK_GATE_HALL:
                for (int q = 1; q <= p.nq; ++q) in.prims.push_back({Prim::GATE, p.nq - q, Prim::GH, 0});
                break;
            case PK_GATE_ORACLE:
                in.prims.push_back({Prim::ORACLE, 0, Prim::GH, 0});
                break;
            case PK_GATE_INV:
                in.prims.push_back({Prim::INV, 0, Prim::GH, 0});
                break;
            case PK_GATE_D2:
                if (!finite8(gt.angle, 3)) {
                    *err = fmt("instance %lld gate %lld: non-finite angle", i, g);
                    return PK_EINVAL;
                }
                pr = {Prim::GATE, p.nq - gt.is1, Prim::GD2, d2};
                pr.param = (int)plan->params.size();
                in.prims.push_back(pr);
                plan->params.push_back({0, d2});
                for (int e = 0; e < 3; ++e) plan->default_angles.push_back(gt.angle[e]);
                ++d2;
                break;
            case PK_GATE_TWOOP:
            case PK_GATE_CNOT:
            case PK_GATE_CPHASE:
            case PK_GATE_CPHASEK:
            case PK_GATE_SWAP: {
                // fixed 4x4 operator in the basis |q_is1 q_is2> (Eq. resmat2), row-major (re, im)
                double m[32] = {0};
                auto set = [&](int r, int c, double re, double im) {
                    m[2 * (4 * r + c)] = re;
                    m[2 * (4 * r + c) + 1] = im;
                };
                if (gt.kind == PK_GATE_TWOOP) {
                    if (!finite8(gt.op, 32)) {
                        *err = fmt("instance %lld gate %lld: non-finite operator", i, g);
                        return PK_EINVAL;
                    }
                    for (int e = 0; e < 32; ++e) m[e] = gt.op[e];
                    if (!is_unitary4(m)) plan->backward_ok = false;
                } else if (gt.kind == PK_GATE_CNOT) {  // control is1, target is2 (Sec. 4.2)
                    set(0, 0, 1, 0); set(1, 1, 1, 0); set(2, 3, 1, 0); set(3, 2, 1, 0);
                } else if (gt.kind == PK_GATE_CPHASE || gt.kind == PK_GATE_CPHASEK) {
                    in.prims.push_back(phase_prim(p.nq, gt.is1, gt.is2, gt.kind == PK_GATE_CPHASE ? 0 : gt.k));
                    break;
                } else {  // SWAP: |ab> -> |ba>
                    for (int e = 0; e < 32; ++e) m[e] = kSwap4[e];
                }
                in.prims.push_back(mat4_prim(plan, p.nq, gt.is1, gt.is2, m,
                                             gt.kind == PK_GATE_SWAP ? Prim::GSWAP : Prim::GMAT4));
                break;
            }
            case PK_GATE_QFT:
            case PK_GATE_QFT_NOSWAP: {
                // Eq. QFT1 on the register held by state bits lo .. lo+k-1 (value bit t
                // on state bit lo + t, the register's first qubit on the top bit).  In
                // 2 pi n n' / 2^k = 2 pi sum_(i,j) b_i c_j 2^(i+j-k) (input bits b, output
                // bits c) only the terms i + j < k are not multiples of 2 pi.  A Hadamard
                // on value bit t turns b_t into c_(k-1-t), so the output is bit-reversed,
                // and supplies the term i + j = k - 1; the term of b_t with the output
                // bit on a higher, already transformed bit u is the controlled phase
                // e^(2 pi i / 2^(u - t + 1)).  From the top bit down: the phases of bit t
                // with every higher bit, then its Hadamard (App. A draws the same circuit).
                // Swapping bits t and k-1-t restores standard order; the labelled
                // variant leaves the register bit-reversed.
                const int top = p.nq - gt.is1, kq = gt.k, lo = top - kq + 1;
                auto qubit_of = [&](int bit) { return p.nq - bit; };
                for (int t = kq - 1; t >= 0; --t) {
                    for (int u = t + 1; u < kq; ++u)
                        in.prims.push_back(phase_prim(p.nq, qubit_of(lo + u), qubit_of(lo + t), u - t + 1));
                    in.prims.push_back({Prim::GATE, lo + t, Prim::GH, 0});
                }
                if (gt.kind == PK_GATE_QFT)
                    for (int t = 0; t < kq - 1 - t; ++t)
                        in.prims.push_back(
                            mat4_prim(plan, p.nq, qubit_of(lo + t), qubit_of(lo + kq - 1 - t), kSwap4, Prim::GSWAP));
                break;
            }
            case PK_GATE_D4:
                if (!finite8(gt.angle, 3)) {
                    *err = fmt("instance %lld gate %lld: non-finite angle", i, g);
                    return PK_EINVAL;
                }
                pr = {Prim::GATE, p.nq - gt.is1, Prim::GD4, plan->n_d4};
                pr.bit2 = p.nq - gt.is2;
                pr.param = (int)plan->params.size();
                in.prims.push_back(pr);
                plan->params.push_back({1, plan->n_d4});
                for (int e = 0; e < 3; ++e) plan->default_angles.push_back(gt.angle[e]);
                ++plan->n_d4;
                break;
            default:
                *err = fmt("instance %lld gate %lld: unknown kind", i, g);
                return PK_EINVAL;
            }
        }
        in.n_d2 = d2 - in.d2_base;
        plan->max_nq = std::max(plan->max_nq, p.nq);
        plan->inst.push_back(std::move(in));
    }
    plan->n_d2 = d2;
    plan->total_elems = off;
    return recompile(plan, err);
}

int recompile(Plan* plan, std::string* err) {
    (void)err;
    plan->passes.clear();
    plan->stages.clear();
    plan->flips.clear();
    plan->phases.clear();
    plan->twid.assign({1.0, 0.0});
    plan->urefs.clear();
    plan->idesc.clear();
    plan->order.clear();
    plan->d2_grad.clear();
    plan->n_partials = 0;
    plan->n_reads = 0;
    plan->n_gpart = 0;
    int read_base = 0;
    for (auto& in : plan->inst) {
        in.read_base = read_base;
        read_base += (int)in.marked.size();
    }
    plan->n_reads = read_base;

    for (int dir = 0; dir < 2; ++dir) {
        std::map<std::string, std::vector<int>> cut_cache;
        for (auto& in : plan->inst) {
            Compiler c;
            c.cut_cache = &cut_cache;
            c.plan = plan;
            c.in = &in;
            c.backward = dir == 1;
            // two state vectors per tile in the backward pass: cap the tile at 2^12
            // amplitudes so that both fit in registers without spilling
            const int kcap = c.backward ? std::min(plan->tiling.tile_bits, kBackwardMaxBits) : plan->tiling.tile_bits;
            c.k = std::min(kcap, in.nq);
            c.C = std::min(plan->tiling.carrier_bits, c.k);
            c.RBITS = c.backward ? 4 : plan->tiling.reg_bits;
            c.RB = std::min(c.RBITS, c.k);
            bool has_two = false;
            for (const Prim& pr : in.prims) has_two = has_two || (pr.bit2 >= 0 && pr.gk != Prim::GPHASE);
            if (has_two && c.k < in.nq && c.k - c.C < 2) {
                *err = "two-qubit gates need at least two non-carrier tile bits (tile_bits >= carrier_bits + 2)";
                return PK_EINVAL;
            }
            std::vector<Prim> prims = in.prims;
            if (c.backward) std::reverse(prims.begin(), prims.end());
            auto& dst = c.backward ? in.bwd : in.fwd;
            dst.clear();
            if (c.backward) in.gpart_base = (int)plan->n_gpart;
            c.compile(prims, &dst);
            if (!c.backward) {
                dst.back().part_base = (int)plan->n_partials;
                plan->n_partials += dst.back().ntiles;
            }
        }
    }
    // flatten: all forward passes (instance order), then all backward passes
    auto emit = [&](Instance& in, int idx, HostPass& hp) {
        Pass p{};
        p.k = hp.k;
        p.stage_begin = (int)plan->stages.size();
        p.ntiles = hp.ntiles;
        p.state_off = in.off;
        p.flags = hp.flags;
        p.scale = hp.scale;
        p.part_base = hp.part_base;
        p.uref_begin = hp.uref_begin;
        p.nuref = hp.nuref;
        p.kmax = hp.kmax;
        p.rbits = hp.rbits;
        for (int l = 0; l < 16; ++l) {
            p.tpos[l] = l < hp.k ? hp.tbits[l] : -1;
            p.stpos[l] = l < hp.k ? hp.sbits[l] : -1;
        }
        std::vector<char> used(in.nq, 0);
        for (int b : hp.tbits) used[b] = 1;
        std::vector<int> fbits;
        for (int b = 0; b < in.nq; ++b)
            if (!used[b]) fbits.push_back(b);
        // runs of consecutive positions: (source bit, length, destination bit)
        auto runs = [](const std::vector<int>& pos, Run* out) {
            int n = 0;
            for (size_t i = 0; i < pos.size();) {
                size_t j = i + 1;
                while (j < pos.size() && pos[j] == pos[j - 1] + 1) ++j;
                out[n].src = (int32_t)i;
                out[n].len = (int32_t)(j - i);
                out[n].dst = pos[i];
                out[n].pad = 0;
                ++n;
                i = j;
            }
            return n;
        };
        p.ntrun = runs(hp.tbits, p.trun);
        p.nstrun = runs(hp.sbits, p.strun);
        p.nfrun = runs(fbits, p.frun);
        // byte offsets of a thread inside a tile in the load / store layouts
        const int esz = plan->prec == PK_FP64 ? 16 : 8;
        for (int which = 0; which < 2; ++which) {
            const HostStage& hs = which == 0 ? hp.stages.front() : hp.stages.back();
            const std::vector<int>& pos = which == 0 ? hp.tbits : hp.sbits;
            uint64_t maxoff = 0;
            for (int l = 0; l < hp.k; ++l) {
                bool reg = false;
                for (int a = 0; a < kMaxRegBits; ++a) reg = reg || hs.rb[a] == l;
                if (!reg) maxoff += (uint64_t)1 << pos[l];
            }
            if (maxoff * (uint64_t)esz >= ((uint64_t)1 << 32)) p.flags |= PASS_WIDE;
        }
        p.nstages = (int)hp.subs.size();
        for (const Stage& st : hp.subs) plan->stages.push_back(st);
        plan->passes.push_back(p);
    };
    for (size_t i = 0; i < plan->inst.size(); ++i)
        for (size_t p = 0; p < plan->inst[i].fwd.size(); ++p) {
            HostPass& hp = plan->inst[i].fwd[p];
            const int64_t bytes = ((int64_t)1 << plan->inst[i].nq) * (plan->prec == PK_FP64 ? 16 : 8);
            if (plan->prec == PK_FP64 && (hp.flags & PASS_LAST) && bytes >= kStreamBytes && hp.sbits == hp.tbits)
                hp.flags |= PASS_STREAM;
            emit(plan->inst[i], (int)i, hp);
            if (i == 0 && plan->inst.size() == 1 && p < plan->walk.size()) plan->passes.back().walk = plan->walk[p];
            if (i == 0 && plan->inst.size() == 1 && p < plan->overlap.size())
                plan->passes.back().overlap = plan->overlap[p];
        }
    plan->n_fwd_passes = (int)plan->passes.size();
    for (size_t i = 0; i < plan->inst.size(); ++i)
        for (size_t p = 0; p < plan->inst[i].bwd.size(); ++p) {
            emit(plan->inst[i], (int)i, plan->inst[i].bwd[p]);
            const size_t nf = plan->inst[i].fwd.size();
            if (i == 0 && plan->inst.size() == 1 && plan->walk.size() == nf + plan->inst[i].bwd.size())
                plan->passes.back().walk = plan->walk[nf + p];
        }

    // batched launch tables
    int first = 0;
    for (size_t i = 0; i < plan->inst.size(); ++i) {
        const Instance& in = plan->inst[i];
        InstDesc d{};
        d.first_pass = first;
        d.npass = (int)in.fwd.size();
        d.read_base = in.read_base;
        d.nmarked = (int)in.marked.size();
        d.part_base = in.fwd.back().part_base;
        d.ntiles_last = in.fwd.back().ntiles;
        first += d.npass;
        plan->idesc.push_back(d);
        plan->order.push_back((int)i);
    }
    std::stable_sort(plan->order.begin(), plan->order.end(),
                     [&](int a, int b) { return plan->inst[a].nq > plan->inst[b].nq; });
    return PK_OK;
}

TeamSchedule team_schedule(const Plan* plan, int64_t grid, int n_xcd) {
    TeamSchedule ts;
    const int S = plan->batch.team_size;
    if (n_xcd < 1 || grid % n_xcd != 0) n_xcd = 1;
    ts.n_xcd = n_xcd;
    ts.team_size = S;
    const int64_t per_xcd = grid / n_xcd;
    if (S > 0 && per_xcd >= S) ts.n_teams = (int)std::min<int64_t>((per_xcd / S) * n_xcd, kMaxTeams);
    // a team index must name whole groups of S workgroups of one XCD
    ts.n_teams -= ts.n_teams % n_xcd;
    std::vector<std::vector<int32_t>> lists(ts.n_teams);
    std::vector<double> load(ts.n_teams, 0.0);
    for (int32_t i : plan->order) {
        const Instance& in = plan->inst[i];
        const bool large = ts.n_teams > 0 && in.fwd.front().ntiles >= (int64_t)plan->batch.min_team_tiles * S;
        if (!large) {
            ts.solo.push_back(i);
            continue;
        }
        int best = 0;
        for (int t = 1; t < ts.n_teams; ++t)
            if (load[t] < load[best]) best = t;
        lists[best].push_back(i);
        load[best] += (double)in.fwd.size() * (double)((int64_t)1 << in.nq);
    }
    ts.team_off.push_back(0);
    for (auto& l : lists) {
        ts.team_list.insert(ts.team_list.end(), l.begin(), l.end());
        ts.team_off.push_back((int32_t)ts.team_list.size());
    }
    return ts;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

TableLayout table_layout(const Plan* plan) {
    TableLayout t{};
    size_t o = 0;
    t.passes = o;
    o = align256(o + plan->passes.size() * sizeof(Pass));
    t.stages = o;
    o = align256(o + plan->stages.size() * sizeof(Stage));
    t.flips = o;
    o = align256(o + plan->flips.size() * sizeof(Flip));
    t.phases = o;
    o = align256(o + plan->phases.size() * sizeof(PhaseOp));
    t.twid = o;
    o = align256(o + plan->twid.size() * sizeof(double));
    t.urefs = o;
    o = align256(o + plan->urefs.size() * sizeof(URef));
    t.mats = o;  // static matrices followed by the default angles
    o = align256(o + (plan->static_mats.size() + plan->default_angles.size()) * sizeof(double));
    t.mats4 = o;  // static two-qubit matrices
    o = align256(o + plan->static_mats4.size() * sizeof(double));
    t.params = o;
    o = align256(o + plan->params.size() * sizeof(ParamRef));
    t.idesc = o;
    o = align256(o + plan->idesc.size() * sizeof(InstDesc));
    t.order = o;  // the queue order of the batched launch (instances left to single workgroups)
    o = align256(o + plan->inst.size() * sizeof(int32_t));
    t.team_off = o;
    o = align256(o + (kMaxTeams + 1) * sizeof(int32_t));
    t.team_list = o;
    o = align256(o + plan->inst.size() * sizeof(int32_t));
    t.red = o;  // evaluation reductions, then backward reductions
    o = align256(o + (2 * plan->inst.size() + 3 * plan->d2_grad.size()) * sizeof(Reduction));
    t.total = std::max<size_t>(o, 256);
    return t;
}

WsLayout workspace_layout(const Plan* plan, int op) {
    WsLayout w{};
    size_t o = 0;
    w.mats = o;
    o = align256(o + (size_t)(2 * plan->n_static + 5 * plan->n_d2) * 8 * sizeof(double));
    w.mats4 = o;
    o = align256(o + (size_t)(2 * plan->n_static4 + 5 * plan->n_d4) * 32 * sizeof(double));
    w.partials = o;
    o = align256(o + (size_t)plan->n_partials * sizeof(double));
    w.reads = o;
    o = align256(o + (size_t)plan->n_reads * sizeof(double));
    w.gpart = o;
    if (op == PK_OP_BACKWARD) o = align256(o + (size_t)plan->n_gpart * sizeof(double));
    w.counters = o;  // batched queue, barrier time-out flag, one barrier counter per team
    o = align256(o + (plan->inst.size() + 8 + kMaxTeams) * sizeof(int64_t));
    w.state = o;
    if (op == PK_OP_BACKWARD) {
        size_t esz = plan->prec == PK_FP64 ? 16 : 8;
        int64_t maxn = 0;
        for (auto& in : plan->inst) maxn = std::max<int64_t>(maxn, (int64_t)1 << in.nq);
        o = align256(o + (size_t)maxn * esz);
    }
    w.total = std::max<size_t>(o, 256);
    return w;
}

std::vector<Reduction> eval_reductions(const Plan* plan) {
    WsLayout w = workspace_layout(plan, PK_OP_EVAL);
    std::vector<Reduction> r;
    for (size_t i = 0; i < plan->inst.size(); ++i) {
        const InstDesc& d = plan->idesc[i];
        r.push_back({0, (int)i, (int64_t)(w.reads / 8) + d.read_base, d.nmarked});
        r.push_back({1, (int)i, (int64_t)(w.partials / 8) + d.part_base, d.ntiles_last});
    }
    return r;
}

std::vector<Reduction> backward_reductions(const Plan* plan) {
    WsLayout w = workspace_layout(plan, PK_OP_BACKWARD);
    std::vector<Reduction> r;
    for (const auto& g : plan->d2_grad)
        for (int t = 0; t < 3; ++t)
            r.push_back({2, 3 * g.d + t, (int64_t)(w.gpart / 8) + g.gslot + t * g.nt, g.nt});
    return r;
}

std::string describe(const Plan* plan) {
    std::string s = "{\"prec\":";
    s += plan->prec == PK_FP64 ? "\"fp64\"" : "\"fp32\"";
    s += ",\"tile_bits\":" + std::to_string(plan->tiling.tile_bits);
    s += ",\"carrier_bits\":" + std::to_string(plan->tiling.carrier_bits);
    s += ",\"fuse\":" + std::to_string(plan->tiling.fuse);
    s += ",\"n_static\":" + std::to_string(plan->n_static);
    s += ",\"n_d2\":" + std::to_string(plan->n_d2);
    s += ",\"n_static4\":" + std::to_string(plan->n_static4);
    s += ",\"n_d4\":" + std::to_string(plan->n_d4);
    s += ",\"params\":[";
    for (size_t q = 0; q < plan->params.size(); ++q)
        s += (q ? "," : "") + std::string("[") + std::to_string(plan->params[q].kind) + "," +
             std::to_string(plan->params[q].slot) + "]";
    s += "]";
    s += ",\"instances\":[";
    const char* kinds[] = {"H", "MAT", "FLIP", "SCALE", "READ", "SEED", "D2BWD", "MAT4", "D4BWD", "PHASE"};
    for (size_t i = 0; i < plan->inst.size(); ++i) {
        const Instance& in = plan->inst[i];
        if (i) s += ",";
        s += "{\"nq\":" + std::to_string(in.nq) + ",\"offset\":" + std::to_string(in.off);
        for (int dir = 0; dir < 2; ++dir) {
            s += dir == 0 ? ",\"forward\":[" : ",\"backward\":[";
            const auto& ps = dir == 0 ? in.fwd : in.bwd;
            for (size_t p = 0; p < ps.size(); ++p) {
                const HostPass& hp = ps[p];
                if (p) s += ",";
                s += "{\"k\":" + std::to_string(hp.k) + ",\"rbits\":" + std::to_string(hp.rbits) +
                     ",\"flags\":" + std::to_string(hp.flags) + ",\"walk\":" +
                     std::to_string(plan->inst.size() != 1 ? 0
                                    : dir == 0 ? (p < plan->walk.size() ? plan->walk[p] : 0)
                                    : (plan->walk.size() == in.fwd.size() + in.bwd.size() ? plan->walk[in.fwd.size() + p] : 0));
                s += ",\"overlap\":" + std::to_string(plan->inst.size() == 1 && dir == 0 && p < plan->overlap.size()
                                                           ? plan->overlap[p]
                                                           : 0);
                s += ",\"urefs\":[";
                for (int r = 0; r < hp.nuref; ++r) {
                    const URef& ur = plan->urefs[hp.uref_begin + r];
                    if (r) s += ",";
                    s += "[" + std::to_string(ur.base) + "," + std::to_string((long long)ur.mask) + "]";
                }
                s += "]";
                char buf[64];
                std::snprintf(buf, sizeof buf, "%.17g", hp.scale);
                s += ",\"scale\":";
                s += buf;
                s += ",\"tile_bits\":[";
                for (size_t l = 0; l < hp.tbits.size(); ++l) s += (l ? "," : "") + std::to_string(hp.tbits[l]);
                s += "],\"store_bits\":[";
                for (size_t l = 0; l < hp.sbits.size(); ++l) s += (l ? "," : "") + std::to_string(hp.sbits[l]);
                s += "],\"stages\":[";
                for (size_t st = 0; st < hp.stages.size(); ++st) {
                    const HostStage& hs = hp.stages[st];
                    if (st) s += ",";
                    s += "{\"rb\":[";
                    for (int a = 0; a < kMaxRegBits; ++a) s += (a ? "," : "") + std::to_string(hs.rb[a]);
                    s += "],\"ops\":[";
                    for (size_t o = 0; o < hs.ops.size(); ++o) {
                        const Op& op = hs.ops[o];
                        if (o) s += ",";
                        s += "{\"kind\":\"";
                        s += kinds[op.kind];
                        s += "\",\"a\":" + std::to_string(op.a) + ",\"arg\":" + std::to_string(op.arg);
                        if (op.kind == OP_FLIP || op.kind == OP_READ || op.kind == OP_SEED) {
                            const Flip& f = plan->flips[op.arg];
                            s += ",\"tile\":" + std::to_string(f.tile) + ",\"j\":" + std::to_string(f.j) +
                                 ",\"slot\":" + std::to_string(f.slot);
                        }
                        if (op.kind == OP_PHASE) {
                            const HostPhase& h = hp.phases[op.arg];
                            s += ",\"b1\":" + std::to_string(h.b1) + ",\"b2\":" + std::to_string(h.b2);
                            std::snprintf(buf, sizeof buf, ",\"c\":%.17g,\"s\":%.17g", h.c, h.s);
                            s += buf;
                        }
                        if (op.kind == OP_D2BWD || op.kind == OP_D4BWD) {
                            std::snprintf(buf, sizeof buf, "%.17g", (double)op.gscale);
                            s += ",\"gscale\":";
                            s += buf;
                        }
                        s += "}";
                    }
                    s += "]}";
                }
                s += "],\"subs\":[";
                for (size_t q = 0; q < hp.subs.size(); ++q) {
                    const Stage& u = hp.subs[q];
                    if (q) s += ",";
                    std::snprintf(buf, sizeof buf, "%.17g", (double)u.d2b_gscale);
                    s += "{\"steps\":" + std::to_string(u.steps) + ",\"rb\":[";
                    for (int a = 0; a < kMaxRegBits; ++a) s += (a ? "," : "") + std::to_string(u.rb[a]);
                    s += "],\"exchange\":" + std::to_string(u.exchange) + ",\"seed\":" + std::to_string(u.seed) +
                         ",\"flip_pre\":" + std::to_string(u.flip_pre) + ",\"phase_first\":" +
                         std::to_string(u.phase_first) + ",\"phase_count\":" + std::to_string(u.phase_count) +
                         ",\"phase_pm\":[" + std::to_string(u.phase_pm[0]) + "," + std::to_string(u.phase_pm[1]) +
                         "," + std::to_string(u.phase_pm[2]) + "," + std::to_string(u.phase_pm[3]) + "]" +
                         ",\"phase_cnt\":[" + std::to_string(u.phase_cnt[0]) + "," + std::to_string(u.phase_cnt[1]) +
                         "," + std::to_string(u.phase_cnt[2]) + "," + std::to_string(u.phase_cnt[3]) + "]" +
                         ",\"phase_ucnt\":[" + std::to_string(u.phase_ucnt[0]) + "," + std::to_string(u.phase_ucnt[1]) +
                         "," + std::to_string(u.phase_ucnt[2]) + "," + std::to_string(u.phase_ucnt[3]) + "]" +
                         ",\"phase_tt\":[" + std::to_string(u.phase_tt[0]) + "," + std::to_string(u.phase_tt[1]) +
                         "," + std::to_string(u.phase_tt[2]) + "," + std::to_string(u.phase_tt[3]) + "]" +
                         ",\"phase_ttm\":[" + std::to_string(u.phase_ttm[0]) + "," + std::to_string(u.phase_ttm[1]) +
                         "," + std::to_string(u.phase_ttm[2]) + "," + std::to_string(u.phase_ttm[3]) + "]" +
                         ",\"phase_ut0\":[" + std::to_string(u.phase_ut0[0]) + "," + std::to_string(u.phase_ut0[1]) +
                         "," + std::to_string(u.phase_ut0[2]) + "," + std::to_string(u.phase_ut0[3]) + "]" +
                         ",\"phase_ut1\":[" + std::to_string(u.phase_ut1[0]) + "," + std::to_string(u.phase_ut1[1]) +
                         "," + std::to_string(u.phase_ut1[2]) + "," + std::to_string(u.phase_ut1[3]) + "]" +
                         ",\"mat_pre_a\":" +
                         std::to_string(u.mat_pre_a) + ",\"mat_pre\":" + std::to_string(u.mat_pre) +
                         ",\"hmask1\":" + std::to_string(u.hmask1) + ",\"flip_mid\":" +
                         std::to_string(u.flip_mid) + ",\"hmask2\":" + std::to_string(u.hmask2) +
                         ",\"mat_post_a\":" + std::to_string(u.mat_post_a) + ",\"mat_post\":" +
                         std::to_string(u.mat_post) + ",\"d2b_a\":" + std::to_string(u.d2b_a) +
                         ",\"d2b_mat\":" + std::to_string(u.d2b_mat) + ",\"d2b_gscale\":" + buf +
                         ",\"mat4\":" + std::to_string(u.mat4) + ",\"mat4b\":" + std::to_string(u.mat4b) +
                         ",\"d4b_mat\":" + std::to_string(u.d4b_mat);
                    std::snprintf(buf, sizeof buf, "%.17g", (double)u.d4b_gscale);
                    s += ",\"d4b_gscale\":";
                    s += buf;
                    s += ",\"scale\":" + std::to_string(u.scale) + ",\"read\":" + std::to_string(u.read) +
                         ",\"nlanes\":" + std::to_string(u.nlanes) + ",\"lanes\":[";
                    for (int i = 0; i < u.nlanes; ++i) s += (i ? "," : "") + std::to_string((u.lanes >> (4 * i)) & 15u);
                    s += "],\"lanes_rest\":" + std::to_string(u.lanes_rest) + "}";
                }
                s += "]}";
            }
            s += "]";
        }
        s += "}";
    }
    s += "],\"phases\":[";
    for (size_t q = 0; q < plan->phases.size(); ++q) {
        const PhaseOp& ph = plan->phases[q];
        char buf[160];
        std::snprintf(buf, sizeof buf, "%s[%d,%u,%lld,%.17g,%.17g]", q ? "," : "", ph.slot, ph.tmask,
                      (long long)ph.fmask, ph.cm1, ph.s);
        s += buf;
    }
    // the product tables only while they are small (the emulated sizes): at full
    // size they run to megabytes
    s += "],\"twid_entries\":" + std::to_string(plan->twid.size() / 2) + ",\"twid\":";
    if (plan->twid.size() <= (size_t)1 << 17) {
        s += "[";
        for (size_t q = 0; q < plan->twid.size(); ++q) {
            char buf[40];
            std::snprintf(buf, sizeof buf, "%s%.17g", q ? "," : "", plan->twid[q]);
            s += buf;
        }
        s += "]";
    } else {
        s += "null";
    }
    s += ",\"flips\":[";
    for (size_t f = 0; f < plan->flips.size(); ++f) {
        const Flip& fl = plan->flips[f];
        if (f) s += ",";
        s += "[" + std::to_string(fl.tile) + "," + std::to_string(fl.j) + "," + std::to_string(fl.slot) + "]";
    }
    s += "]}";
    return s;
}

}  // namespace pk
