// sv_api.hip -- the C ABI of libsv (include/sv.h): validation, gate
// classification and dispatch, measurements, circuits and the adjoint sweep.
//
// Gate classification follows Sec. 2 of the paper: only a gate's non-zero
// matrix elements are used, so each named gate maps to the cheapest kernel
// class that realises it exactly:
//   permutation  X / CNOT / Toffoli / SWAP (any controls)  -> k_pair (moves)
//   subset phase Z, S, T, PHASE and their controlled forms -> k_one on the
//                |1..1> subspace of controls + target
//   diagonal     RZ (any controls)                          -> k_pair, one
//                phase per member (no partner exchange)
//   butterfly    H, RY (real), RX, Y, U2 (any controls)     -> k_pair
//   two-target   U4 (any controls)                          -> k_quad
// (targets below bit 6 take the wavefront form k_wpair of the paired
// kernel; gates with a qubit whose runs span under 1 KiB take the
// LDS-staged k_lds_gate where that keeps accesses on whole lines.)
// A control never adds work: it is a fixed 1-bit inserted into the group
// index, so the kernel visits only the controlled subspace.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <cstdlib>
#include <cstdio>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "sv_core.h"
#include "sv_dense.h"
#include "sv_phase.h"

namespace svk {

static thread_local std::string g_last_error;

sv_status set_error(sv_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

}  // namespace svk

using namespace svk;

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
struct sv_state_s {
    int n;
    int dtype;
    void* data;
    bool owned;
    hipStream_t stream;
    double* work;        // stage-1 partials + results
    size_t work_doubles;
    void* dense_dev;     // real form of the last dense block (device), allocated on first use
    void* dense_host;    // pinned staging of that real form
    hipEvent_t dense_ev; // the staging copy has been read once this completes
};

struct OpRec {
    int gate;
    int nc, nt;
    int q[SV_OP_MAX_QUBITS];
    int pidx;
    double value;
    std::vector<double> matrix;
};

struct sv_circuit_s {
    int n;
    int n_params;
    std::vector<OpRec> ops;
    // adjoint workspace (device)
    int n_slots;
    int seg;
    double* d_partials;
    double* d_slot_val;
    double* d_slot_scale;
    int* d_slot_param;
    double* d_grad;
    double* d_misc;  // [0] = E, then inner-product partials
    size_t misc_doubles;
};

// Handles are not addresses.  A handle packs a slot of the table below, the
// kind of object (state, circuit, batch) and the slot's generation, which
// advances when the object is freed: a handle kept after its free, or a
// handle of another kind, is rejected even when the allocator has since
// handed the freed object's address to a new one.
namespace {
struct HandleSlot {
    void* obj;
    uint32_t gen;
    int kind;
};
std::mutex g_mu;
std::vector<HandleSlot> g_slots;
std::vector<uint32_t> g_free_slots;
constexpr int kKindBits = 4;

uint64_t handle_encode(uint32_t slot, uint32_t gen, int kind)
{
    return ((uint64_t)gen << 32) | ((uint64_t)(slot + 1) << kKindBits) | (uint64_t)kind;
}

HandleSlot* handle_slot(const void* h, int kind)
{
    const uint64_t v = (uint64_t)(uintptr_t)h;
    const uint64_t slot1 = (v & 0xffffffffull) >> kKindBits;
    if (!v || (int)(v & ((1u << kKindBits) - 1u)) != kind || slot1 == 0 || slot1 > g_slots.size()) return nullptr;
    HandleSlot& e = g_slots[slot1 - 1];
    if (!e.obj || e.kind != kind || e.gen != (uint32_t)(v >> 32)) return nullptr;
    return &e;
}
}  // namespace

void* svk::handle_put(void* obj, int kind)
{
    std::lock_guard<std::mutex> lk(g_mu);
    uint32_t slot;
    if (!g_free_slots.empty()) {
        slot = g_free_slots.back();
        g_free_slots.pop_back();
    } else {
        slot = (uint32_t)g_slots.size();
        g_slots.push_back(HandleSlot{nullptr, 0, 0});
    }
    HandleSlot& e = g_slots[slot];
    e.obj = obj;
    e.kind = kind;
    if (++e.gen == 0) e.gen = 1;  // generation 0 is never handed out
    return (void*)(uintptr_t)handle_encode(slot, e.gen, kind);
}

void* svk::handle_get(const void* h, int kind)
{
    std::lock_guard<std::mutex> lk(g_mu);
    HandleSlot* e = handle_slot(h, kind);
    return e ? e->obj : nullptr;
}

void* svk::handle_drop(const void* h, int kind)
{
    std::lock_guard<std::mutex> lk(g_mu);
    HandleSlot* e = handle_slot(h, kind);
    if (!e) return nullptr;
    void* obj = e->obj;
    e->obj = nullptr;
    ++e->gen;  // every copy of the old handle is now stale
    g_free_slots.push_back((uint32_t)(e - g_slots.data()));
    return obj;
}

// Entry points take handles named <x>_h and resolve them to `x` here.
#define SV_STATE(st)                                                                   \
    sv_state_s* const st = (sv_state_s*)handle_get(st##_h, HK_STATE);                   \
    if (!st) return set_error(SV_ERR_HANDLE, "invalid state handle")

static sv_status hip_status(hipError_t e, const char* where)
{
    if (e == hipSuccess) return SV_OK;
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    return set_error(SV_ERR_HIP, buf);
}

static size_t elem_bytes(int dtype) { return dtype == SV_C128 ? 16 : 8; }

// ---------------------------------------------------------------------------
// launch-shape table (filled by defaults, overridable by the autotuner)
// ---------------------------------------------------------------------------
// Class 2 (an element-wise diagonal kernel) is retired: RZ runs as a paired
// update with one phase per member.  Its number stays reserved.
enum KClass {
    KC_PAIR = 0, KC_ONE = 1, KC_RETIRED = 2, KC_QUAD = 3, KC_GENERAL = 4, KC_WAVE = 5, KC_LDS = 6, KC_COUNT = 7
};
// Tier of a launch: bytes spanned by one run of consecutive touched
// amplitudes, 2^(lowest touched qubit) * element size: < 64 B, < 1 KiB, larger.
constexpr int kTiers = 3;
static Launch g_tune[KC_COUNT][2][kTiers];
static bool g_tune_init = false;

static void tune_defaults()
{
    // Measured on MI355X with 30-qubit states: small blocks; enough groups per
    // thread to keep two or more 16-byte loads in flight per lane (a complex64
    // amplitude is 8 bytes, so it needs twice the groups); non-temporal
    // accesses only once runs span >= 64 bytes.  The wavefront form reads
    // whole runs, so it streams non-temporally in every tier.
    for (int c = 0; c < KC_COUNT; ++c)
        for (int d = 0; d < 2; ++d) {
            const bool c128 = d == 1;
            const bool one_amp = c == KC_ONE || c == KC_WAVE;
            const int u = one_amp ? (c128 ? 2 : 4) : ((c == KC_PAIR && !c128) ? 2 : 1);
            const int nt0 = c == KC_WAVE || c == KC_ONE ? 1 : 0;
            g_tune[c][d][0] = Launch{128, u, nt0};
            g_tune[c][d][1] = Launch{128, u, 1};
            g_tune[c][d][2] = Launch{64, u, 1};
            if (c == KC_LDS)  // staged chunks are whole lines in every tier; block caps lds_block
                for (int t = 0; t < kTiers; ++t) g_tune[c][d][t] = Launch{512, 1, 1};
        }
    g_tune_init = true;
}

static int tier_of(int dtype, int low_qubit)
{
    const uint64_t span = low_qubit >= 40 ? (1ull << 40) : (elem_bytes(dtype) << low_qubit);
    return span < 64 ? 0 : (span < 1024 ? 1 : 2);
}

// Tier whose launch shape a gate takes: its own, or the one SV_FORCE_TIER
// (0, 1 or 2 in the environment, read at the first launch) names for every
// gate.  Forcing changes launch shapes only, never the kernel a gate runs.
static int shape_tier(int dtype, int low_qubit)
{
    static const int forced = [] {
        const char* e = getenv("SV_FORCE_TIER");
        if (!e || !*e) return -1;
        const int t = atoi(e);
        return t >= 0 && t < kTiers ? t : -1;
    }();
    return forced >= 0 ? forced : tier_of(dtype, low_qubit);
}

static Launch tune_get(int kc, int dtype, int low_qubit)
{
    if (!g_tune_init) tune_defaults();
    return g_tune[kc][dtype == SV_C128 ? 1 : 0][shape_tier(dtype, low_qubit)];
}

// Workgroup walk order of the group kernels (GroupSpec::order, block_slot).
// Measured on MI355X at 30 qubits (per-target medians of the gate sweep), a
// complex128 gate whose member offset is 32..128 MiB (target 21..23) runs
// 5-8% slower in launch order than at neighbouring targets, and the XCD
// spread brings it back in line; at 256 MiB and beyond, and at every
// complex64 target, the spread is 2-8% slower, so it is taken only in that
// band.  (Target 20, 16 MiB, is 8% slow under both orders.)  SV_BLOCK_ORDER=0
// or 1 in the environment (read at the first launch) or sv_set_block_order
// forces one order for every launch.
static int g_block_order = -2;  // -2: not yet read from the environment; -1: per launch

static int block_order_override()
{
    if (g_block_order == -2) {
        const char* e = getenv("SV_BLOCK_ORDER");
        g_block_order = (!e || !*e) ? -1 : (atoi(e) ? 1 : 0);
    }
    return g_block_order;
}

static int block_order(int dtype, uint64_t offsets)
{
    const int forced = block_order_override();
    if (forced >= 0) return forced;
    if (dtype != SV_C128) return 0;
    for (int t = 0; t < 64; ++t) {
        if (!((offsets >> t) & 1ull)) continue;
        const uint64_t bytes = elem_bytes(dtype) << t;
        if (bytes >= (32ull << 20) && bytes <= (128ull << 20)) return 1;
    }
    return 0;
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
static sv_status check_qubits(int n, const int* ctrl, int nc, const int* tgt, int nt)
{
    if (nc < 0 || nc > SV_MAX_CONTROLS) return set_error(SV_ERR_ARG, "number of controls out of range");
    if (nt < 0) return set_error(SV_ERR_ARG, "negative number of targets");
    if ((nc > 0 && !ctrl) || (nt > 0 && !tgt)) return set_error(SV_ERR_ARG, "null qubit array");
    uint64_t seen = 0;
    for (int j = 0; j < nc + nt; ++j) {
        const int q = j < nc ? ctrl[j] : tgt[j - nc];
        if (q < 0 || q >= n) return set_error(SV_ERR_QUBIT, "qubit index " + std::to_string(q) + " out of range");
        if (seen & (1ull << q)) return set_error(SV_ERR_QUBIT, "qubit index " + std::to_string(q) + " repeated");
        seen |= 1ull << q;
    }
    return SV_OK;
}

static int gate_targets(int gate)
{
    switch (gate) {
    case SV_SWAP:
    case SV_U4: return 2;
    default: return 1;
    }
}

static bool gate_has_param(int gate)
{
    return gate == SV_RX || gate == SV_RY || gate == SV_RZ || gate == SV_PHASE;
}

// ---------------------------------------------------------------------------
// plans: a gate classified into a kernel class with its index spec
// ---------------------------------------------------------------------------
enum PlanKind { PK_NOP = 0, PK_PAIR, PK_ONE, PK_QUAD, PK_WPAIR, PK_LDS };

struct Plan {
    int kind;
    int kc;
    int low;  // lowest inserted qubit (launch-shape tier); 64 = none
    GroupSpec gs;
    uint64_t off[4];
    int op;
    int wt;  // target of the wavefront form
    double m[128];
    LdsSpec ls;  // PK_LDS
    int lk;      // PK_LDS: gate qubits
};

// Bits whose runs of consecutive amplitudes span fewer bytes than this are
// predicated inside the kernel instead of inserted into the group index, so
// wavefront accesses stay on whole 128-byte lines.
constexpr uint64_t kPredBytes = 128;

// Build the group index spec: `ins` are inserted (fixed) bits, `fixed_one`
// the inserted bits that are 1 in every group, `pmask` the predicated bits.
static GroupSpec make_groups(int n, const int* ins, int nins, uint64_t set_mask, uint64_t pmask = 0)
{
    GroupSpec gs{};
    int p[kMaxIns];
    for (int i = 0; i < nins; ++i) p[i] = ins[i];
    std::sort(p, p + nins);
    gs.nins = nins;
    for (int i = 0; i < nins; ++i) gs.pos[i] = p[i];
    gs.n_groups = 1ull << (n - nins);
    gs.set_mask = set_mask;
    gs.pmask = pmask;
    return gs;
}

// Split `bits` (bits that must be 1 for the gate to act) into inserted and
// predicated ones; a bit is predicated if its run span is under kPredBytes or
// if it is below `min_insert` (the wavefront form keeps bits 0..5 in-lane).
struct BitSplit {
    int ins[kMaxIns];
    int nins;
    uint64_t set_mask;
    uint64_t pmask;
    int low;
};

static void split_bits(const int* q, int nq, int dtype, int min_insert, BitSplit* b)
{
    b->nins = 0;
    b->set_mask = 0;
    b->pmask = 0;
    b->low = 64;
    for (int j = 0; j < nq; ++j) {
        const bool pred = (elem_bytes(dtype) << q[j]) < kPredBytes || q[j] < min_insert;
        if (pred) {
            b->pmask |= 1ull << q[j];
        } else {
            b->ins[b->nins++] = q[j];
            b->set_mask |= 1ull << q[j];
            b->low = std::min(b->low, q[j]);
        }
    }
}

static void conj_transpose2(double* m)
{
    double t[8];
    // (r, c) -> conj of (c, r)
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            t[2 * (2 * r + c)] = m[2 * (2 * c + r)];
            t[2 * (2 * r + c) + 1] = -m[2 * (2 * c + r) + 1];
        }
    memcpy(m, t, sizeof t);
}

// Gates whose lowest qubit has runs under 1 KiB go through the LDS-staged
// kernel (k_lds_gate) when the state has room for a stage.
static bool lds_eligible(int n, int dtype, const int* q, int k)
{
    int lo = 64, h = 0;
    for (int j = 0; j < k; ++j) {
        lo = std::min(lo, q[j]);
        if (q[j] >= kLdsChunkBits) ++h;
    }
    return tier_of(dtype, lo) <= 1 && n >= kLdsChunkBits + h;
}

static void build_lds(int n, const int* q, int k, const int* ctrl, int nc, Plan* pl)
{
    constexpr int C = kLdsChunkBits;
    LdsSpec& ls = pl->ls;
    memset(&ls, 0, sizeof ls);
    ls.k = k;
    int hq[3], h = 0;
    for (int j = 0; j < k; ++j)
        if (q[j] >= C) hq[h++] = q[j];
    std::sort(hq, hq + h);
    ls.h = h;
    for (int j = 0; j < h; ++j) ls.hq[j] = hq[j];
    for (int j = 0; j < k; ++j) {
        int lp = q[j];
        if (q[j] >= C)
            for (int i = 0; i < h; ++i)
                if (hq[i] == q[j]) lp = C + i;
        ls.lpos[j] = lp;
        ls.lsort[j] = lp;
    }
    std::sort(ls.lsort, ls.lsort + k);
    int ins[kMaxIns], nins = 0;
    for (int j = 0; j < h; ++j) ins[nins++] = hq[j] - C;
    for (int j = 0; j < nc; ++j) {
        if (ctrl[j] < C) {
            ls.pmask |= 1u << ctrl[j];
        } else {
            ls.cmask |= 1ull << ctrl[j];
            ins[nins++] = ctrl[j] - C;
        }
    }
    pl->gs = make_groups(n - C, ins, nins, 0, 0);
    pl->kind = PK_LDS;
    pl->kc = KC_LDS;
    pl->lk = k;
    pl->low = 64;
    for (int j = 0; j < k; ++j) pl->low = std::min(pl->low, q[j]);
}

// Row a1 of the method: classify a gate into a kernel class with its index
// spec (group insertion, predicate, member offsets) and coefficients.
static sv_status build_plan(int n, int dtype, int gate, const int* ctrl, int nc, const int* tgt, int nt,
                            const double* params, const double* matrix, int adjoint, Plan* pl)
{
    if (gate < SV_I || gate > SV_U4) return set_error(SV_ERR_ARG, "unknown gate");
    if (nt != gate_targets(gate)) return set_error(SV_ERR_ARG, "wrong number of targets for gate");
    sv_status st = check_qubits(n, ctrl, nc, tgt, nt);
    if (st) return st;
    if (gate_has_param(gate) && !params) return set_error(SV_ERR_ARG, "gate needs params[0]");
    if ((gate == SV_U2 || gate == SV_U4) && !matrix) return set_error(SV_ERR_ARG, "gate needs a matrix");
    if (nc + nt > kMaxIns) return set_error(SV_ERR_ARG, "too many qubits");

    memset(pl, 0, sizeof *pl);
    const int t = tgt[0];
    const double sgn = adjoint ? -1.0 : 1.0;
    BitSplit bs;

    switch (gate) {
    case SV_I: pl->kind = PK_NOP; return SV_OK;
    case SV_X:
    case SV_Y:
    case SV_H:
    case SV_RX:
    case SV_RY:
    case SV_RZ:
    case SV_U2: {
        if (gate == SV_X) {
            pl->op = PAIR_SWAP;
        } else if (gate == SV_Y) {
            pl->op = PAIR_Y;
        } else if (gate == SV_H) {
            const double r = M_SQRT1_2;  // correctly rounded 2^(-1/2)
            pl->op = PAIR_REAL;
            double m[8] = {r, 0, r, 0, r, 0, -r, 0};
            memcpy(pl->m, m, sizeof m);
        } else if (gate == SV_RY) {
            const double c = cos(params[0] / 2), s = sgn * sin(params[0] / 2);
            pl->op = PAIR_REAL;
            double m[8] = {c, 0, -s, 0, s, 0, c, 0};
            memcpy(pl->m, m, sizeof m);
        } else if (gate == SV_RX) {
            const double c = cos(params[0] / 2), s = sgn * sin(params[0] / 2);
            pl->op = PAIR_RX;
            double m[8] = {c, 0, 0, -s, 0, -s, c, 0};
            memcpy(pl->m, m, sizeof m);
        } else if (gate == SV_RZ) {
            // diag(e^{-i th/2}, e^{i th/2}): every amplitude of the control
            // subspace changes, each by the phase of its own target bit
            const double c = cos(params[0] / 2), s = sgn * sin(params[0] / 2);
            pl->op = PAIR_DIAG;
            double m[8] = {c, -s, 0, 0, 0, 0, c, s};
            memcpy(pl->m, m, sizeof m);
        } else {
            pl->op = PAIR_DENSE;
            memcpy(pl->m, matrix, 8 * sizeof(double));
            if (adjoint) conj_transpose2(pl->m);
        }
        if (t < 6) {
            // wavefront form: lanes own contiguous amplitudes; controls below
            // bit 6 are predicated, higher ones inserted
            split_bits(ctrl, nc, dtype, 6, &bs);
            pl->kind = PK_WPAIR;
            pl->kc = KC_WAVE;
            pl->wt = t;
            pl->gs = make_groups(n, bs.ins, bs.nins, bs.set_mask, bs.pmask);
            pl->low = bs.low;
        } else {
            split_bits(ctrl, nc, dtype, 0, &bs);
            bs.ins[bs.nins++] = t;
            pl->kind = PK_PAIR;
            pl->kc = KC_PAIR;
            pl->gs = make_groups(n, bs.ins, bs.nins, bs.set_mask, bs.pmask);
            pl->off[0] = 0;
            pl->off[1] = 1ull << t;
            pl->low = std::min(bs.low, t);
        }
        return SV_OK;
    }
    case SV_SWAP: {
        // Half of the amplitudes move.  With both qubits at or above the
        // 128-byte line bits a line holds only moving or only staying
        // amplitudes, so the paired kernel touches just the moving lines; a
        // lower qubit shares every line between the two kinds, and then the
        // LDS-staged form, which streams whole lines, is the cheaper one.
        const bool line_aligned = (elem_bytes(dtype) << std::min(tgt[0], tgt[1])) >= kPredBytes;
        if (!line_aligned && lds_eligible(n, dtype, tgt, 2)) {
            build_lds(n, tgt, 2, ctrl, nc, pl);
            pl->op = 1;
            return SV_OK;
        }
        split_bits(ctrl, nc, dtype, 0, &bs);
        bs.ins[bs.nins++] = tgt[0];
        bs.ins[bs.nins++] = tgt[1];
        pl->kind = PK_PAIR;
        pl->kc = KC_PAIR;
        pl->op = PAIR_SWAP;
        pl->gs = make_groups(n, bs.ins, bs.nins, bs.set_mask, bs.pmask);
        pl->off[0] = 1ull << tgt[0];
        pl->off[1] = 1ull << tgt[1];
        pl->low = std::min(bs.low, std::min(tgt[0], tgt[1]));
        return SV_OK;
    }
    case SV_Z:
    case SV_S:
    case SV_T:
    case SV_PHASE: {
        // acts on the amplitudes whose control and target bits are all 1
        int bits[SV_MAX_CONTROLS + 1];
        for (int j = 0; j < nc; ++j) bits[j] = ctrl[j];
        bits[nc] = t;
        split_bits(bits, nc + 1, dtype, 0, &bs);
        pl->kind = PK_ONE;
        pl->kc = KC_ONE;
        pl->gs = make_groups(n, bs.ins, bs.nins, bs.set_mask, bs.pmask);
        pl->low = bs.low;
        if (gate == SV_Z) {
            pl->op = ONE_NEG;
        } else if (gate == SV_S) {
            pl->op = ONE_MULI;
            pl->m[0] = sgn;
        } else {
            const double ph = gate == SV_T ? M_PI / 4 : params[0];
            pl->op = ONE_MUL;
            pl->m[0] = cos(ph);
            pl->m[1] = sgn * sin(ph);
        }
        return SV_OK;
    }
    case SV_U4: {
        const int a = tgt[0], b = tgt[1];  // a = most significant matrix bit
        if (lds_eligible(n, dtype, tgt, 2)) {
            build_lds(n, tgt, 2, ctrl, nc, pl);
            pl->op = 0;
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c) {
                    const int src = adjoint ? (4 * c + r) : (4 * r + c);
                    pl->m[2 * (4 * r + c)] = matrix[2 * src];
                    pl->m[2 * (4 * r + c) + 1] = adjoint ? -matrix[2 * src + 1] : matrix[2 * src + 1];
                }
            return SV_OK;
        }
        split_bits(ctrl, nc, dtype, 0, &bs);
        bs.ins[bs.nins++] = a;
        bs.ins[bs.nins++] = b;
        pl->kind = PK_QUAD;
        pl->kc = KC_QUAD;
        pl->gs = make_groups(n, bs.ins, bs.nins, bs.set_mask, bs.pmask);
        pl->off[0] = 0;
        pl->off[1] = 1ull << b;
        pl->off[2] = 1ull << a;
        pl->off[3] = (1ull << a) | (1ull << b);
        pl->low = std::min(bs.low, std::min(a, b));
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) {
                const int src = adjoint ? (4 * c + r) : (4 * r + c);
                pl->m[2 * (4 * r + c)] = matrix[2 * src];
                pl->m[2 * (4 * r + c) + 1] = adjoint ? -matrix[2 * src + 1] : matrix[2 * src + 1];
            }
        return SV_OK;
    }
    }
    return set_error(SV_ERR_ARG, "unknown gate");
}

// The member offsets of a plan's groups (bits between the streams a group
// touches); the wavefront form's partners share a wavefront, the one-member
// form has none.
static uint64_t plan_offsets(const Plan& pl)
{
    switch (pl.kind) {
    case PK_PAIR: return pl.off[1];
    case PK_QUAD: return pl.off[3];
    case PK_LDS: {
        uint64_t m = 0;
        for (int j = 0; j < pl.ls.h; ++j) m |= 1ull << pl.ls.hq[j];
        return m;
    }
    default: return 0;
    }
}

template <typename T>
static hipError_t run_plan_t(const Plan& pl, void* psi, hipStream_t s, int dtype)
{
    const Launch lc = tune_get(pl.kc, dtype, pl.low);
    GroupSpec gs = pl.gs;
    gs.order = block_order(dtype, plan_offsets(pl));
    switch (pl.kind) {
    case PK_NOP: return hipSuccess;
    case PK_PAIR: {
        Coef2<T> c;
        for (int i = 0; i < 8; ++i) c.m[i] = (T)pl.m[i];
        return launch_pair<T>(psi, gs, pl.off[0], pl.off[1], pl.op, c, s, lc);
    }
    case PK_WPAIR: {
        Coef2<T> c;
        for (int i = 0; i < 8; ++i) c.m[i] = (T)pl.m[i];
        return launch_wpair<T>(psi, gs, pl.wt, pl.op, c, s, lc);
    }
    case PK_LDS: {
        T m[128];
        const int mm = 2 * (1 << pl.lk) * (1 << pl.lk);
        for (int i = 0; i < mm; ++i) m[i] = (T)pl.m[i];
        return launch_lds_gate<T>(psi, gs, pl.ls, pl.op, m, s, lc);
    }
    case PK_ONE: return launch_one<T>(psi, gs, pl.op, (T)pl.m[0], (T)pl.m[1], s, lc);
    case PK_QUAD: {
        Coef4<T> c;
        for (int i = 0; i < 32; ++i) c.m[i] = (T)pl.m[i];
        return launch_quad<T>(psi, gs, pl.off, c, s, lc);
    }
    }
    return hipErrorInvalidValue;
}

static sv_status run_plan(const Plan& pl, sv_state st, void* psi)
{
    const hipError_t e = st->dtype == SV_C128 ? run_plan_t<double>(pl, psi, st->stream, st->dtype)
                                              : run_plan_t<float>(pl, psi, st->stream, st->dtype);
    return hip_status(e, "gate launch");
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
// Workspace layout: doubles [0, 8) hold results, [8, ...) stage-1 partials.
constexpr size_t kWorkHead = 8;
static sv_status ensure_work(sv_state st, size_t partial_doubles)
{
    const size_t doubles = kWorkHead + partial_doubles;
    if (st->work_doubles >= doubles) return SV_OK;
    if (st->work) {
        (void)hipStreamSynchronize(st->stream);
        (void)hipFree(st->work);
        st->work = nullptr;
        st->work_doubles = 0;
    }
    if (hipMalloc((void**)&st->work, doubles * sizeof(double)) != hipSuccess) {
        st->work = nullptr;
        return set_error(SV_ERR_OOM, "workspace allocation failed");
    }
    st->work_doubles = doubles;
    return SV_OK;
}

// Entry points: sv.h declares each of them extern "C", so these definitions
// have C linkage.

// ---------------------------------------------------------------------------
// lifecycle
// ---------------------------------------------------------------------------
size_t sv_state_bytes(int n_qubits, sv_dtype dtype)
{
    if (n_qubits < 1 || n_qubits > SV_MAX_QUBITS) return 0;
    if (dtype != SV_C64 && dtype != SV_C128) return 0;
    return (size_t(1) << n_qubits) * elem_bytes(dtype);
}

static sv_status make_state(void* ptr, bool owned, int n, sv_dtype dtype, void* stream, sv_state* out)
{
    sv_state st = new sv_state_s{};
    st->n = n;
    st->dtype = dtype;
    st->data = ptr;
    st->owned = owned;
    st->stream = (hipStream_t)stream;
    st->work = nullptr;  // reduction workspace is allocated on first use
    st->work_doubles = 0;
    st->dense_dev = nullptr;
    st->dense_host = nullptr;
    st->dense_ev = nullptr;
    *out = (sv_state)handle_put(st, HK_STATE);
    return SV_OK;
}

sv_status sv_alloc(int n_qubits, sv_dtype dtype, void* stream, sv_state* out)
{
    if (!out) return set_error(SV_ERR_ARG, "null output handle");
    const size_t bytes = sv_state_bytes(n_qubits, dtype);
    if (!bytes) return set_error(SV_ERR_ARG, "n_qubits or dtype out of range");
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess || !p) {
        (void)hipGetLastError();
        return set_error(SV_ERR_OOM, "state allocation of " + std::to_string(bytes) + " bytes failed");
    }
    sv_status rc = make_state(p, true, n_qubits, dtype, stream, out);
    if (rc) {
        (void)hipFree(p);
        return rc;
    }
    return sv_set_basis(*out, 0);
}

sv_status sv_wrap(void* dev_ptr, int n_qubits, sv_dtype dtype, void* stream, sv_state* out)
{
    if (!out) return set_error(SV_ERR_ARG, "null output handle");
    if (!dev_ptr) return set_error(SV_ERR_ARG, "null device pointer");
    if (((uintptr_t)dev_ptr) % 16) return set_error(SV_ERR_ARG, "device pointer must be 16-byte aligned");
    if (!sv_state_bytes(n_qubits, dtype)) return set_error(SV_ERR_ARG, "n_qubits or dtype out of range");
    return make_state(dev_ptr, false, n_qubits, dtype, stream, out);
}

sv_status sv_free(sv_state st_h)
{
    sv_state_s* const st = (sv_state_s*)handle_drop(st_h, HK_STATE);
    if (!st) return set_error(SV_ERR_HANDLE, "invalid state handle");
    (void)hipStreamSynchronize(st->stream);
    if (st->work) (void)hipFree(st->work);
    if (st->dense_dev) (void)hipFree(st->dense_dev);
    if (st->dense_host) (void)hipHostFree(st->dense_host);
    if (st->dense_ev) (void)hipEventDestroy(st->dense_ev);
    if (st->owned && st->data) (void)hipFree(st->data);
    delete st;
    return SV_OK;
}

sv_status sv_set_stream(sv_state st_h, void* stream)
{
    SV_STATE(st);
    st->stream = (hipStream_t)stream;
    return SV_OK;
}

sv_status sv_get_info(sv_state st_h, int* n_qubits, int* dtype, void** dev_ptr)
{
    SV_STATE(st);
    if (n_qubits) *n_qubits = st->n;
    if (dtype) *dtype = st->dtype;
    if (dev_ptr) *dev_ptr = st->data;
    return SV_OK;
}

sv_status sv_set_basis(sv_state st_h, uint64_t index)
{
    SV_STATE(st);
    const uint64_t na = 1ull << st->n;
    if (index >= na) return set_error(SV_ERR_ARG, "basis index out of range");
    const hipError_t e = st->dtype == SV_C128 ? launch_set_basis<double>(st->data, na, index, st->stream)
                                              : launch_set_basis<float>(st->data, na, index, st->stream);
    return hip_status(e, "set_basis");
}

sv_status sv_copy_to_host(sv_state st_h, void* host, size_t bytes)
{
    SV_STATE(st);
    if (!host) return set_error(SV_ERR_ARG, "null host pointer");
    if (bytes != sv_state_bytes(st->n, (sv_dtype)st->dtype)) return set_error(SV_ERR_ARG, "byte count mismatch");
    hipError_t e = hipMemcpyAsync(host, st->data, bytes, hipMemcpyDeviceToHost, st->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
    return hip_status(e, "copy_to_host");
}

sv_status sv_copy_from_host(sv_state st_h, const void* host, size_t bytes)
{
    SV_STATE(st);
    if (!host) return set_error(SV_ERR_ARG, "null host pointer");
    if (bytes != sv_state_bytes(st->n, (sv_dtype)st->dtype)) return set_error(SV_ERR_ARG, "byte count mismatch");
    hipError_t e = hipMemcpyAsync(st->data, host, bytes, hipMemcpyHostToDevice, st->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
    return hip_status(e, "copy_from_host");
}

sv_status sv_copy_state(sv_state dst_h, sv_state src_h)
{
    SV_STATE(dst);
    SV_STATE(src);
    if (dst->n != src->n || dst->dtype != src->dtype) return set_error(SV_ERR_ARG, "state shape mismatch");
    if (dst == src) return SV_OK;
    const size_t bytes = sv_state_bytes(src->n, (sv_dtype)src->dtype);
    return hip_status(hipMemcpyAsync(dst->data, src->data, bytes, hipMemcpyDeviceToDevice, dst->stream),
                      "copy_state");
}

sv_status sv_synchronize(sv_state st_h)
{
    SV_STATE(st);
    return hip_status(hipStreamSynchronize(st->stream), "synchronize");
}

// ---------------------------------------------------------------------------
// gates
// ---------------------------------------------------------------------------
sv_status sv_apply_controlled(sv_state st_h, sv_gate gate, const int* controls, int nc, const int* targets, int nt,
                              const double* params, const double* matrix, int adjoint)
{
    SV_STATE(st);
    Plan pl;
    sv_status rc = build_plan(st->n, st->dtype, gate, controls, nc, targets, nt, params, matrix, adjoint, &pl);
    if (rc) return rc;
    return run_plan(pl, st, st->data);
}

sv_status sv_apply_gate(sv_state st, sv_gate gate, const int* targets, int nt, const double* params,
                        const double* matrix, int adjoint)
{
    return sv_apply_controlled(st, gate, nullptr, 0, targets, nt, params, matrix, adjoint);
}

sv_status sv_apply_general(sv_state st_h, const int* qubits, int k, const double* matrix)
{
    SV_STATE(st);
    if (k < 1 || k > SV_MAX_GENERAL_K) return set_error(SV_ERR_ARG, "general gate needs 1 <= k <= 3");
    if (!matrix) return set_error(SV_ERR_ARG, "null matrix");
    sv_status rc = check_qubits(st->n, nullptr, 0, qubits, k);
    if (rc) return rc;
    GroupSpec gs = make_groups(st->n, qubits, k, 0);
    const int M = 1 << k;
    uint64_t off[8];
    int low = 64;
    for (int r = 0; r < M; ++r) {
        uint64_t o = 0;
        for (int j = 0; j < k; ++j)
            if ((r >> (k - 1 - j)) & 1) o |= 1ull << qubits[j];
        off[r] = o;
    }
    for (int j = 0; j < k; ++j) low = std::min(low, qubits[j]);
    gs.order = block_order(st->dtype, off[M - 1]);
    if (k == 1 && qubits[0] < 6) {
        // the same dense 2x2, with the partner amplitude fetched across lanes
        Plan pl;
        memset(&pl, 0, sizeof pl);
        pl.kind = PK_WPAIR;
        pl.kc = KC_WAVE;
        pl.wt = qubits[0];
        pl.op = PAIR_DENSE;
        pl.low = 64;
        pl.gs = make_groups(st->n, nullptr, 0, 0, 0);
        memcpy(pl.m, matrix, 8 * sizeof(double));
        return run_plan(pl, st, st->data);
    }
    if (lds_eligible(st->n, st->dtype, qubits, k)) {
        Plan pl;
        memset(&pl, 0, sizeof pl);
        build_lds(st->n, qubits, k, nullptr, 0, &pl);
        pl.op = 0;
        memcpy(pl.m, matrix, sizeof(double) * 2 * M * M);
        return run_plan(pl, st, st->data);
    }
    const Launch lc = tune_get(KC_GENERAL, st->dtype, low);
    hipError_t e;
    if (st->dtype == SV_C128) {
        e = launch_general<double>(st->data, gs, k, off, matrix, st->stream, lc);
    } else {
        float mf[128];
        for (int i = 0; i < 2 * M * M; ++i) mf[i] = (float)matrix[i];
        e = launch_general<float>(st->data, gs, k, off, mf, st->stream, lc);
    }
    return hip_status(e, "general launch");
}

static sv_status apply_dense(sv_state_s* st, const int* qubits, int k, const double* matrix)
{
    if (k < kDenseMinK || k > kDenseMaxK) return set_error(SV_ERR_ARG, "dense block needs 4 <= k <= 6");
    if (!matrix) return set_error(SV_ERR_ARG, "null matrix");
    sv_status rc = check_qubits(st->n, nullptr, 0, qubits, k);
    if (rc) return rc;
    DenseSpec sp;
    memset(&sp, 0, sizeof sp);
    sp.k = k;
    for (int j = 0; j < k; ++j) sp.qs_sorted[j] = qubits[j];
    std::sort(sp.qs_sorted, sp.qs_sorted + k);
    for (int c = 0; c < (1 << k); ++c)
        for (int j = 0; j < k; ++j)
            if ((c >> (k - 1 - j)) & 1) sp.dep[c] |= 1ull << qubits[j];
    sp.groups = (int64_t)1 << (st->n - k);
    sp.order = block_order(st->dtype, sp.dep[(1 << k) - 1]);
    // A group's 2^k amplitudes sit in up to 2^k pages when the targets are
    // high, and the UTCL1 misses on a grid-stride walk, whose next block is
    // far away (measured at 30 qubits: 13-18% of complex64 translations miss
    // at the top placement against under 0.01% at the bottom).  A contiguous
    // run per workgroup (team of 1) keeps its pages for k <= 5 (4-10% faster
    // off the bottom, equal on it); at k = 6 its 64 pages per wavefront
    // thrash more than the grid-stride walk (a team as large as the grid),
    // 1.3-1.8x slower at the top.  Teams of 8 to 2048 workgroups sharing a
    // run measured no better for any placement.
    sp.team = k <= 5 ? 1 : (1 << 30);
    // one buffer of the largest real form (k = kDenseMaxK) serves every call
    const size_t cap = dense_lds_bytes(kDenseMaxK, SV_C128);
    if (!st->dense_dev) {
        if (hipMalloc(&st->dense_dev, cap) != hipSuccess || hipHostMalloc(&st->dense_host, cap) != hipSuccess ||
            hipEventCreateWithFlags(&st->dense_ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            if (st->dense_dev) (void)hipFree(st->dense_dev);
            if (st->dense_host) (void)hipHostFree(st->dense_host);
            st->dense_dev = st->dense_host = nullptr;
            st->dense_ev = nullptr;
            return set_error(SV_ERR_OOM, "dense block buffers");
        }
    } else {
        // the previous call's upload must have read the staging buffer
        const hipError_t e = hipEventSynchronize(st->dense_ev);
        if (e != hipSuccess) return hip_status(e, "dense staging");
    }
    const int n2 = 2 << k;
    std::vector<double> B((size_t)n2 * n2);
    dense_real_form(matrix, k, B.data());
    const size_t bytes = dense_lds_bytes(k, st->dtype);
    if (st->dtype == SV_C128) memcpy(st->dense_host, B.data(), bytes);
    else
        for (size_t i = 0; i < B.size(); ++i) ((float*)st->dense_host)[i] = (float)B[i];
    hipError_t e = hipMemcpyAsync(st->dense_dev, st->dense_host, bytes, hipMemcpyHostToDevice, st->stream);
    if (e == hipSuccess) e = hipEventRecord(st->dense_ev, st->stream);
    if (e == hipSuccess) e = launch_dense(st->data, st->dtype, st->dense_dev, sp, st->stream);
    return hip_status(e, "dense block launch");
}

sv_status sv_apply_dense(sv_state st_h, const int* qubits, int k, const double* matrix)
{
    SV_STATE(st);
    return apply_dense(st, qubits, k, matrix);
}

// ---------------------------------------------------------------------------
// measurement
// ---------------------------------------------------------------------------
static sv_status finish_scalar(sv_state st, const double* dres, double* out)
{
    hipError_t e = hipMemcpyAsync(out, dres, sizeof(double), hipMemcpyDeviceToHost, st->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
    return hip_status(e, "result copy");
}

sv_status sv_norm2(sv_state st_h, double* out)
{
    SV_STATE(st);
    if (!out) return set_error(SV_ERR_ARG, "null output");
    const uint64_t na = 1ull << st->n;
    sv_status rw = ensure_work(st, kReduceBlocks);
    if (rw) return rw;
    double* partials = st->work + kWorkHead;
    double* res = st->work;
    hipError_t e = st->dtype == SV_C128 ? launch_norm_partial<double>(st->data, na, partials, st->stream)
                                        : launch_norm_partial<float>(st->data, na, partials, st->stream);
    if (e == hipSuccess) e = launch_sum_partials(partials, reduce_blocks_for(na), res, st->stream);
    sv_status rc = hip_status(e, "norm");
    if (rc) return rc;
    return finish_scalar(st, res, out);
}

// An observable split into diagonal terms (xmask = 0: one pass evaluates up
// to kDiagTermsPerPass of them, or the closed forms sum Z_i / sum Z_i Z_i+1
// in one) and off-diagonal terms (one pass each).  The term lists are
// std::vector here and fixed-capacity arrays in the allocation-free plan.
template <typename T, int N>
struct FixedVec {
    T v[N];
    int n = 0;
    size_t size() const { return (size_t)n; }
    bool empty() const { return n == 0; }
    T& operator[](size_t i) { return v[i]; }
    const T& operator[](size_t i) const { return v[i]; }
};
template <typename T>
static bool add_term(std::vector<T>& v, const T& x)
{
    v.push_back(x);
    return true;
}
template <typename T, int N>
static bool add_term(FixedVec<T, N>& v, const T& x)
{
    if (v.n >= N) return false;
    v.v[v.n++] = x;
    return true;
}

struct ObsPlan {
    int diag_kind;  // -1 none, 0 generic, 1 sum Z, 2 sum ZZ
    double diag_coeff;
    std::vector<double> dc;
    std::vector<uint64_t> dz;
    std::vector<double> oc;
    std::vector<uint64_t> ox, oz;
    std::vector<int> oy;
};

// Term capacity of the allocation-free plan: at most kNoAllocPasses
// reduction passes, each a pass of up to kDiagTermsPerPass diagonal terms or
// one off-diagonal term.
constexpr int kNoAllocPasses = 64;
struct ObsPlanFixed {
    int diag_kind;
    double diag_coeff;
    FixedVec<double, kNoAllocPasses * kDiagTermsPerPass> dc;
    FixedVec<uint64_t, kNoAllocPasses * kDiagTermsPerPass> dz;
    FixedVec<double, kNoAllocPasses> oc;
    FixedVec<uint64_t, kNoAllocPasses> ox, oz;
    FixedVec<int, kNoAllocPasses> oy;
};

// Closed forms among the diagonal terms: one common coefficient and the z
// masks exactly {2^i : i < n} (sum Z_i, kind 1) or {3 * 2^i : i < n - 1}
// (sum Z_i Z_i+1, kind 2), in any order; else 0 (generic list).
template <typename V, typename W>
static int closed_form(int n, const V& dc, const W& dz)
{
    for (size_t k = 1; k < dc.size(); ++k)
        if (dc[k] != dc[0]) return 0;
    const size_t m = dz.size();
    uint64_t seen = 0;
    bool single = m == (size_t)n, pairs = n > 1 && m == (size_t)(n - 1);
    for (size_t k = 0; k < m && (single || pairs); ++k) {
        const uint64_t z = dz[k];
        const int i = z ? __builtin_ctzll(z) : 64;
        if (i >= 64 || (seen >> i) & 1ull) return 0;
        seen |= 1ull << i;
        if (z != (1ull << i) || i >= n) single = false;
        if (z != (3ull << i) || i + 1 >= n) pairs = false;
    }
    return single ? 1 : (pairs ? 2 : 0);
}

template <typename P>
static sv_status plan_obs(int n, const sv_obs* obs, P* op)
{
    if (!obs) return set_error(SV_ERR_ARG, "null observable");
    if (obs->n_terms < 0) return set_error(SV_ERR_ARG, "negative term count");
    if (obs->n_terms > 0 && (!obs->coeffs || !obs->xmask || !obs->zmask))
        return set_error(SV_ERR_ARG, "null observable arrays");
    const uint64_t all = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
    op->diag_kind = -1;
    for (int k = 0; k < obs->n_terms; ++k) {
        const uint64_t x = obs->xmask[k], z = obs->zmask[k];
        if ((x | z) & ~all) return set_error(SV_ERR_QUBIT, "observable term acts outside the state");
        bool ok;
        if (x == 0) {
            ok = add_term(op->dc, obs->coeffs[k]) && add_term(op->dz, z);
        } else {
            ok = add_term(op->oc, obs->coeffs[k]) && add_term(op->ox, x) && add_term(op->oz, z) &&
                 add_term(op->oy, (int)__builtin_popcountll(x & z));
        }
        if (!ok)  // only the fixed-capacity plan can run out of room
            return set_error(SV_ERR_ARG, "observable needs more reduction passes than this entry point holds (" +
                                             std::to_string(kNoAllocPasses) + ")");
    }
    if (!op->dc.empty()) {
        op->diag_kind = closed_form(n, op->dc, op->dz);
        if (op->diag_kind > 0) op->diag_coeff = op->dc[0];
    }
    return SV_OK;
}

// Reduction passes of a plan (each writes one stage-1 grid of partials).
template <typename P>
static int obs_pass_count(const P& op)
{
    const int diag = op.diag_kind > 0 ? 1 : (int)((op.dc.size() + kDiagTermsPerPass - 1) / kDiagTermsPerPass);
    return diag + (int)op.oc.size();
}

template <typename T, typename P>
static hipError_t obs_passes(sv_state st, const P& op, double* partials, int* count)
{
    int off = 0;
    hipError_t e = hipSuccess;
    const int n = st->n;
    if (op.diag_kind > 0) {
        e = launch_diag_obs_partial<T>(st->data, n, op.diag_kind, op.diag_coeff, nullptr, nullptr, 0, partials + off,
                                       st->stream);
        off += reduce_blocks_for(1ull << n);
    } else if (op.diag_kind == 0) {
        for (size_t k0 = 0; k0 < op.dc.size() && e == hipSuccess; k0 += kDiagTermsPerPass) {
            const int nt = (int)std::min<size_t>(kDiagTermsPerPass, op.dc.size() - k0);
            e = launch_diag_obs_partial<T>(st->data, n, 0, 1.0, &op.dc[k0], &op.dz[k0], nt, partials + off,
                                           st->stream);
            off += reduce_blocks_for(1ull << n);
        }
    }
    for (size_t k = 0; k < op.oc.size() && e == hipSuccess; ++k) {
        e = launch_pauli_partial<T>(st->data, n, op.ox[k], op.oz[k], op.oy[k], op.oc[k], partials + off, st->stream);
        off += reduce_blocks_for(1ull << (n - 1));
    }
    *count = off;
    return e;
}

// Partials needed by the passes of an observable (worst case: one full
// stage-1 grid per pass).
static size_t obs_partials(const ObsPlan& op)
{
    return ((op.dc.size() + kDiagTermsPerPass - 1) / kDiagTermsPerPass + op.oc.size() + 1) * kReduceBlocks;
}

// The caller has reserved obs_partials(op) doubles of workspace; out_dev may
// point into the workspace head, so nothing here may reallocate it.
static sv_status expval_to_dev(sv_state st, const ObsPlan& op, double* out_dev)
{
    int count = 0;
    double* partials = st->work + kWorkHead;
    hipError_t e = st->dtype == SV_C128 ? obs_passes<double>(st, op, partials, &count)
                                        : obs_passes<float>(st, op, partials, &count);
    // an empty observable sums zero partials: the kernel still writes 0.0
    if (e == hipSuccess) e = launch_sum_partials(partials, count, out_dev, st->stream);
    return hip_status(e, "expval");
}

sv_status sv_expval_obs_dev(sv_state st_h, const sv_obs* obs, double* out_dev)
{
    SV_STATE(st);
    if (!out_dev) return set_error(SV_ERR_ARG, "null output");
    ObsPlan op;
    sv_status rc = plan_obs(st->n, obs, &op);
    if (rc) return rc;
    rc = ensure_work(st, obs_partials(op));
    if (rc) return rc;
    return expval_to_dev(st, op, out_dev);
}

// ---------------------------------------------------------------------------
// expectation value into device memory without any allocation
// ---------------------------------------------------------------------------
// The reduction partials of sv_expval_obs_dev_noalloc live in this file-scope
// device array, one copy per GPU, held until the process ends (512 KiB).
// Host code never passes its name to a kernel: the name is a host-side
// stand-in, so each device's address is looked up once, with that device
// current, and kept in scratch_dev.
static __device__ __align__(256) double scratch[kNoAllocPasses * kReduceBlocks];

constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[kScratchDevices];

// The current device's address of `scratch`.
static sv_status scratch_dev(double** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "current device");
    if (dev < 0 || dev >= kScratchDevices) return set_error(SV_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_status(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
        g_scratch_dev[dev] = (double*)p;
    }
    *out = g_scratch_dev[dev];
    return SV_OK;
}

sv_status sv_expval_obs_dev_noalloc(sv_state st_h, const sv_obs* obs, double* out_dev)
{
    SV_STATE(st);
    if (!out_dev) return set_error(SV_ERR_ARG, "null output");
    ObsPlanFixed op;  // fixed-capacity term lists: no heap
    sv_status rc = plan_obs(st->n, obs, &op);
    if (rc) return rc;
    if (obs_pass_count(op) > kNoAllocPasses)
        return set_error(SV_ERR_ARG, "observable needs " + std::to_string(obs_pass_count(op)) +
                                         " reduction passes; this entry point holds at most " +
                                         std::to_string(kNoAllocPasses));
    double* partials = nullptr;
    rc = scratch_dev(&partials);
    if (rc) return rc;
    // every partial the final sum reads is written first by this call's own
    // stage-1 kernels on the same stream, so nothing needs clearing
    int count = 0;
    hipError_t e = st->dtype == SV_C128 ? obs_passes<double>(st, op, partials, &count)
                                        : obs_passes<float>(st, op, partials, &count);
    if (e == hipSuccess) e = launch_sum_partials(partials, count, out_dev, st->stream);
    return hip_status(e, "expval");
}

sv_status sv_expval_obs(sv_state st_h, const sv_obs* obs, double* out)
{
    SV_STATE(st);
    if (!out) return set_error(SV_ERR_ARG, "null output");
    ObsPlan op;
    sv_status rc = plan_obs(st->n, obs, &op);
    if (rc) return rc;
    rc = ensure_work(st, obs_partials(op));
    if (rc) return rc;
    rc = expval_to_dev(st, op, st->work);
    if (rc) return rc;
    return finish_scalar(st, st->work, out);
}

// One Pauli string as bit masks: X and Y positions in *x, Z and Y in *z.
static sv_status pauli_masks(int n_state, const char* paulis, const int* qubits, int n, uint64_t* x, uint64_t* z)
{
    if (n < 0 || (n > 0 && (!paulis || !qubits))) return set_error(SV_ERR_ARG, "bad arguments");
    sv_status rc = check_qubits(n_state, nullptr, 0, qubits, n);
    if (rc) return rc;
    *x = *z = 0;
    for (int j = 0; j < n; ++j) {
        const uint64_t b = 1ull << qubits[j];
        switch (paulis[j]) {
        case 'I': break;
        case 'X': *x |= b; break;
        case 'Y': *x |= b; *z |= b; break;
        case 'Z': *z |= b; break;
        default: return set_error(SV_ERR_ARG, "pauli letters must be I, X, Y or Z");
        }
    }
    return SV_OK;
}

// <psi|P|psi> of one Pauli string into device memory out_dev (may be the
// workspace head).
static sv_status expval_pauli_to_dev(sv_state_s* st, const char* paulis, const int* qubits, int n, double* out_dev,
                                     bool out_in_work)
{
    uint64_t x, z;
    sv_status rc = pauli_masks(st->n, paulis, qubits, n, &x, &z);
    if (rc) return rc;
    const double c = 1.0;
    sv_obs o{1, &c, &x, &z};
    ObsPlan op;
    rc = plan_obs(st->n, &o, &op);
    if (rc) return rc;
    rc = ensure_work(st, obs_partials(op));
    if (rc) return rc;
    return expval_to_dev(st, op, out_in_work ? st->work : out_dev);
}

sv_status sv_expval_pauli(sv_state st_h, const char* paulis, const int* qubits, int n, double* out)
{
    SV_STATE(st);
    if (!out) return set_error(SV_ERR_ARG, "bad arguments");
    sv_status rc = expval_pauli_to_dev(st, paulis, qubits, n, nullptr, true);
    if (rc) return rc;
    return finish_scalar(st, st->work, out);
}

sv_status sv_expval_pauli_dev(sv_state st_h, const char* paulis, const int* qubits, int n, double* out_dev)
{
    SV_STATE(st);
    if (!out_dev) return set_error(SV_ERR_ARG, "null output");
    return expval_pauli_to_dev(st, paulis, qubits, n, out_dev, false);
}

// ---------------------------------------------------------------------------
// circuits
// ---------------------------------------------------------------------------
#define SV_CIRC(c)                                                                     \
    sv_circuit_s* const c = (sv_circuit_s*)handle_get(c##_h, HK_CIRCUIT);               \
    if (!c) return set_error(SV_ERR_HANDLE, "invalid circuit handle")

static sv_status op_plan(const sv_circuit_s* c, int dtype, const OpRec& o, const double* params, int adjoint,
                         Plan* pl)
{
    double th = o.value;
    if (o.pidx >= 0) th = params[o.pidx];
    return build_plan(c->n, dtype, o.gate, o.q, o.nc, o.q + o.nc, o.nt, &th, o.matrix.empty() ? nullptr : o.matrix.data(),
                      adjoint, pl);
}

sv_status sv_circuit_create(int n_qubits, const sv_op* ops, int n_ops, int n_params, sv_circuit* out)
{
    if (!out) return set_error(SV_ERR_ARG, "null output handle");
    if (n_qubits < 1 || n_qubits > SV_MAX_QUBITS) return set_error(SV_ERR_ARG, "n_qubits out of range");
    if (n_ops < 0 || (n_ops > 0 && !ops) || n_params < 0) return set_error(SV_ERR_ARG, "bad op list");
    auto* c = new sv_circuit_s{};
    c->n = n_qubits;
    c->n_params = n_params;
    int slots = 0;
    for (int i = 0; i < n_ops; ++i) {
        const sv_op& s = ops[i];
        OpRec o;
        o.gate = s.gate;
        o.nc = s.n_controls;
        o.nt = s.n_targets;
        o.pidx = s.param_index;
        o.value = s.value;
        if (o.nc < 0 || o.nt < 0 || o.nc + o.nt > SV_OP_MAX_QUBITS) {
            delete c;
            return set_error(SV_ERR_ARG, "op " + std::to_string(i) + ": bad qubit counts");
        }
        for (int j = 0; j < o.nc + o.nt; ++j) o.q[j] = s.qubits[j];
        if (o.pidx >= n_params || o.pidx < -1) {
            delete c;
            return set_error(SV_ERR_ARG, "op " + std::to_string(i) + ": parameter index out of range");
        }
        if (o.pidx >= 0 && !gate_has_param(o.gate)) {
            delete c;
            return set_error(SV_ERR_ARG, "op " + std::to_string(i) + ": gate takes no parameter");
        }
        if (s.gate == SV_U2 || s.gate == SV_U4) {
            const int m = s.gate == SV_U2 ? 8 : 32;
            if (!s.matrix) {
                delete c;
                return set_error(SV_ERR_ARG, "op " + std::to_string(i) + ": missing matrix");
            }
            o.matrix.assign(s.matrix, s.matrix + m);
        }
        // validate by planning once with a zero angle
        Plan pl;
        const double zero = 0.0;
        sv_status rc = build_plan(n_qubits, SV_C128, o.gate, o.q, o.nc, o.q + o.nc, o.nt, &zero,
                                  o.matrix.empty() ? nullptr : o.matrix.data(), 0, &pl);
        if (rc) {
            delete c;
            return set_error(rc, "op " + std::to_string(i) + ": " + g_last_error);
        }
        if (o.pidx >= 0) ++slots;
        c->ops.push_back(o);
    }
    c->n_slots = slots;
    c->seg = reduce_blocks_for(1ull << (n_qubits - 1));
    c->misc_doubles = 8 + (size_t)kReduceBlocks;
    // device workspace
    bool ok = hipMalloc((void**)&c->d_partials, sizeof(double) * std::max<size_t>(1, (size_t)slots * c->seg)) ==
                  hipSuccess &&
              hipMalloc((void**)&c->d_slot_val, sizeof(double) * std::max(1, slots)) == hipSuccess &&
              hipMalloc((void**)&c->d_slot_scale, sizeof(double) * std::max(1, slots)) == hipSuccess &&
              hipMalloc((void**)&c->d_slot_param, sizeof(int) * std::max(1, slots)) == hipSuccess &&
              hipMalloc((void**)&c->d_grad, sizeof(double) * std::max(1, n_params)) == hipSuccess &&
              hipMalloc((void**)&c->d_misc, sizeof(double) * c->misc_doubles) == hipSuccess;
    if (!ok) {
        (void)hipFree(c->d_partials);
        (void)hipFree(c->d_slot_val);
        (void)hipFree(c->d_slot_scale);
        (void)hipFree(c->d_slot_param);
        (void)hipFree(c->d_grad);
        (void)hipFree(c->d_misc);
        delete c;
        return set_error(SV_ERR_OOM, "circuit workspace allocation failed");
    }
    std::vector<double> scale(std::max(1, slots));
    std::vector<int> sparam(std::max(1, slots));
    int s = 0;
    for (const OpRec& o : c->ops) {
        if (o.pidx < 0) continue;
        sparam[s] = o.pidx;
        scale[s] = o.gate == SV_PHASE ? -2.0 : 1.0;
        ++s;
    }
    (void)hipMemcpy(c->d_slot_scale, scale.data(), sizeof(double) * scale.size(), hipMemcpyHostToDevice);
    (void)hipMemcpy(c->d_slot_param, sparam.data(), sizeof(int) * sparam.size(), hipMemcpyHostToDevice);
    *out = (sv_circuit)handle_put(c, HK_CIRCUIT);
    return SV_OK;
}

sv_status sv_circuit_free(sv_circuit c_h)
{
    sv_circuit_s* const c = (sv_circuit_s*)handle_drop(c_h, HK_CIRCUIT);
    if (!c) return set_error(SV_ERR_HANDLE, "invalid circuit handle");
    (void)hipDeviceSynchronize();
    (void)hipFree(c->d_partials);
    (void)hipFree(c->d_slot_val);
    (void)hipFree(c->d_slot_scale);
    (void)hipFree(c->d_slot_param);
    (void)hipFree(c->d_grad);
    (void)hipFree(c->d_misc);
    delete c;
    return SV_OK;
}

static sv_status circuit_forward(sv_circuit c, sv_state st, const double* params)
{
    for (const OpRec& o : c->ops) {
        Plan pl;
        sv_status rc = op_plan(c, st->dtype, o, params, 0, &pl);
        if (rc) return rc;
        rc = run_plan(pl, st, st->data);
        if (rc) return rc;
    }
    return SV_OK;
}

// ---- runs of diagonal gates -------------------------------------------------

// Phase terms (mask, angle in half-turns) of a diagonal op: exp(i pi turns)
// on every amplitude whose index contains mask.  Returns false for other ops.
static bool diag_terms(const OpRec& o, const double* params, std::vector<uint64_t>& masks,
                       std::vector<double>& turns)
{
    if (o.nt != 1) return false;
    uint64_t cm = 0;
    for (int j = 0; j < o.nc; ++j) cm |= 1ull << o.q[j];
    const uint64_t tm = cm | (1ull << o.q[o.nc]);
    const double th = o.pidx >= 0 ? params[o.pidx] : o.value;
    switch (o.gate) {
    case SV_I: return true;
    case SV_Z: masks.push_back(tm); turns.push_back(1.0); return true;
    case SV_S: masks.push_back(tm); turns.push_back(0.5); return true;
    case SV_T: masks.push_back(tm); turns.push_back(0.25); return true;
    case SV_PHASE: masks.push_back(tm); turns.push_back(th / M_PI); return true;
    case SV_RZ:  // exp(-i th/2) on the control subspace, exp(i th) more where the target is 1
        masks.push_back(cm);
        turns.push_back(-0.5 * th / M_PI);
        masks.push_back(tm);
        turns.push_back(th / M_PI);
        return true;
    default: return false;
    }
}

static sv_status run_phase_terms(sv_state st, const uint64_t* masks, const double* turns, int nt)
{
    PhaseRun pr;
    memset(&pr, 0, sizeof pr);
    uint64_t common = ~0ull;
    for (int t = 0; t < nt; ++t) {
        pr.mask[t] = masks[t];
        pr.turns[t] = turns[t];
        common &= masks[t];
    }
    pr.n_terms = nt;
    for (int q = 0; q < st->n; ++q)
        if ((common >> q) & 1) pr.common_pos[pr.n_common++] = q;
    pr.groups = (int64_t)1 << (st->n - pr.n_common);
    return hip_status(launch_phase_run(st->data, st->dtype, pr, st->stream), "phase run launch");
}

sv_status sv_apply_phases(sv_state st_h, int n_terms, const uint64_t* masks, const double* angles)
{
    SV_STATE(st);
    if (n_terms < 1 || n_terms > kMaxPhaseTerms || !masks || !angles)
        return set_error(SV_ERR_ARG, "phase run needs 1..64 terms and non-null arrays");
    std::vector<double> turns(n_terms);
    for (int t = 0; t < n_terms; ++t) {
        if (st->n < 64 && (masks[t] >> st->n)) return set_error(SV_ERR_QUBIT, "phase term mask beyond the state");
        turns[t] = angles[t] / M_PI;
    }
    return run_phase_terms(st, masks, turns.data(), n_terms);
}

static void op_target_matrix(const OpRec& o, const double* params, std::vector<std::complex<double>>& m);

// An uncontrolled one-target gate that is not diagonal: it can share a pass
// with the diagonal run that follows it.
static bool pair_fusable(const OpRec& o)
{
    if (o.nc != 0 || o.nt != 1) return false;
    switch (o.gate) {
    case SV_X:
    case SV_Y:
    case SV_H:
    case SV_RX:
    case SV_RY:
    case SV_U2: return true;
    default: return false;
    }
}

// The circuit with every run of two or more consecutive diagonal ops applied
// as one phase pass (a run longer than kMaxPhaseTerms terms takes several),
// consecutive uncontrolled one-target gates on one qubit composed into one
// 2x2, and such a gate followed by a diagonal run applied together with it
// in one pass.
static sv_status circuit_forward_fused(sv_circuit c, sv_state st, const double* params)
{
    std::vector<uint64_t> masks;
    std::vector<double> turns;
    size_t run_begin = 0, run_len = 0;
    int pending = -1;  // a pair gate waiting for the run after it
    std::vector<std::complex<double>> pend;  // its matrix, later same-qubit gates composed on
    int pend_ops = 0;                        // ops composed into pend
    auto run_op = [&](const OpRec& o) -> sv_status {
        Plan pl;
        sv_status rc = op_plan(c, st->dtype, o, params, 0, &pl);
        if (!rc) rc = run_plan(pl, st, st->data);
        return rc;
    };
    auto flush = [&]() -> sv_status {
        sv_status rc = SV_OK;
        if (pending >= 0) {
            if (masks.empty()) {
                if (pend_ops == 1) {
                    rc = run_op(c->ops[pending]);
                } else {  // the composed 2x2 as a U2 on the same qubit
                    OpRec u2 = c->ops[pending];
                    u2.gate = SV_U2;
                    u2.pidx = -1;
                    u2.matrix.resize(8);
                    for (int e = 0; e < 4; ++e) {
                        u2.matrix[2 * e] = pend[e].real();
                        u2.matrix[2 * e + 1] = pend[e].imag();
                    }
                    rc = run_op(u2);
                }
            } else {
                PairCoef u;
                for (int e = 0; e < 4; ++e) {
                    u.m[2 * e] = pend[e].real();
                    u.m[2 * e + 1] = pend[e].imag();
                }
                const uint64_t tb = 1ull << c->ops[pending].q[0];
                // every term holds the gate's qubit and at most one more bit: a
                // phase linear in the bits, tabulated per byte by the kernel
                bool linear = true;
                for (uint64_t m2 : masks) linear &= (m2 & tb) && __builtin_popcountll(m2 & ~tb) <= 1;
                if (linear) {
                    LinearPhase lp;
                    memset(&lp, 0, sizeof lp);
                    int top = 0;
                    for (size_t t = 0; t < masks.size(); ++t) {
                        const uint64_t other = masks[t] & ~tb;
                        if (!other) {
                            lp.turns_const += turns[t];
                            continue;
                        }
                        const int b = __builtin_ctzll(other);
                        lp.turns_of_bit[b] += turns[t];
                        top = std::max(top, b);
                    }
                    lp.n_bytes = top / 8 + 1;
                    // the per-byte phase tables live in the state's workspace
                    rc = ensure_work(st, kLinearPhaseTableBytes / sizeof(double));
                    if (!rc)
                        rc = hip_status(launch_pair_linear_phase(st->data, st->dtype, c->ops[pending].q[0], u, lp,
                                                                 (int64_t)1 << (st->n - 1), st->work + kWorkHead,
                                                                 st->stream),
                                        "pair and linear phase launch");
                    masks.clear();
                    turns.clear();
                    run_len = 0;
                    pending = -1;
                    return rc;
                }
                // terms holding the gate's qubit first (they reach only its 1 side)
                PhaseRun pr;
                memset(&pr, 0, sizeof pr);
                int n_with = 0;
                for (int pass = 0; pass < 2; ++pass)
                    for (size_t t = 0; t < masks.size(); ++t)
                        if (((masks[t] & tb) != 0) == (pass == 0)) {
                            pr.mask[pr.n_terms] = masks[t];
                            pr.turns[pr.n_terms] = turns[t];
                            ++pr.n_terms;
                            n_with += pass == 0;
                        }
                pr.groups = (int64_t)1 << (st->n - 1);
                rc = hip_status(
                    launch_pair_phase_run(st->data, st->dtype, c->ops[pending].q[0], u, pr, n_with, st->stream),
                    "pair and phase run launch");
            }
        } else if (run_len == 1) {  // a lone diagonal op keeps its own kernel
            rc = run_op(c->ops[run_begin]);
        } else if (!masks.empty()) {
            rc = run_phase_terms(st, masks.data(), turns.data(), (int)masks.size());
        }
        masks.clear();
        turns.clear();
        run_len = 0;
        pending = -1;
        return rc;
    };
    for (size_t i = 0; i < c->ops.size(); ++i) {
        const OpRec& o = c->ops[i];
        std::vector<uint64_t> m;
        std::vector<double> tt;
        if (diag_terms(o, params, m, tt)) {
            if (masks.size() + m.size() > (size_t)kMaxPhaseTerms) {
                sv_status rc = flush();
                if (rc) return rc;
            }
            if (run_len == 0) run_begin = i;
            ++run_len;
            masks.insert(masks.end(), m.begin(), m.end());
            turns.insert(turns.end(), tt.begin(), tt.end());
            continue;
        }
        if (pair_fusable(o) && pending >= 0 && run_len == 0 && c->ops[pending].q[0] == o.q[0]) {
            // o after the pending gate on the same qubit: pend <- M(o) pend
            std::vector<std::complex<double>> m;
            op_target_matrix(o, params, m);
            const std::vector<std::complex<double>> a = pend;
            for (int r = 0; r < 2; ++r)
                for (int k = 0; k < 2; ++k) pend[2 * r + k] = m[2 * r] * a[k] + m[2 * r + 1] * a[2 + k];
            ++pend_ops;
            continue;
        }
        sv_status rc = flush();
        if (rc) return rc;
        if (pair_fusable(o)) {
            pending = (int)i;
            op_target_matrix(o, params, pend);
            pend_ops = 1;
            continue;
        }
        rc = run_op(o);
        if (rc) return rc;
    }
    return flush();
}

sv_status sv_circuit_apply_fused(sv_circuit c_h, sv_state st_h, const double* params)
{
    SV_CIRC(c);
    SV_STATE(st);
    if (st->n != c->n) return set_error(SV_ERR_ARG, "state size does not match the circuit");
    if (c->n_params > 0 && !params) return set_error(SV_ERR_ARG, "null params");
    return circuit_forward_fused(c, st, params);
}

// ---- circuits as dense blocks on the matrix cores ---------------------------

using cplx = std::complex<double>;

static uint64_t op_qubit_mask(const OpRec& o)
{
    uint64_t m = 0;
    for (int j = 0; j < o.nc + o.nt; ++j) m |= 1ull << o.q[j];
    return m;
}

// The op's matrix on its targets (2^nt square, row-major, first target the
// most significant bit), as the gate kernels apply it.
static void op_target_matrix(const OpRec& o, const double* params, std::vector<cplx>& m)
{
    const double th = o.pidx >= 0 ? params[o.pidx] : o.value;
    const double c = cos(th / 2), s = sin(th / 2), r = M_SQRT1_2;
    const cplx i1(0, 1);
    switch (o.gate) {
    case SV_X: m = {0, 1, 1, 0}; break;
    case SV_Y: m = {0, -i1, i1, 0}; break;
    case SV_Z: m = {1, 0, 0, -1}; break;
    case SV_H: m = {r, r, r, -r}; break;
    case SV_S: m = {1, 0, 0, i1}; break;
    case SV_T: m = {1, 0, 0, std::polar(1.0, M_PI / 4)}; break;
    case SV_RX: m = {c, -i1 * s, -i1 * s, c}; break;
    case SV_RY: m = {c, -s, s, c}; break;
    case SV_RZ: m = {std::polar(1.0, -th / 2), 0, 0, std::polar(1.0, th / 2)}; break;
    case SV_PHASE: m = {1, 0, 0, std::polar(1.0, th)}; break;
    case SV_SWAP: m = {1, 0, 0, 0, 0, 0, 1, 0, 0, 1, 0, 0, 0, 0, 0, 1}; break;
    case SV_U2:
    case SV_U4: {
        const size_t d = (size_t)1 << o.nt;
        m.resize(d * d);
        for (size_t i = 0; i < d * d; ++i) m[i] = cplx(o.matrix[2 * i], o.matrix[2 * i + 1]);
        break;
    }
    default: m = {1, 0, 0, 1}; break;  // identity
    }
}

// v (2^k amplitudes, local bit p of the index = block qubit of position p)
// <- the op on local target bits lt (lt[0] the matrix MSB), local controls lc.
static void apply_local(cplx* v, int k, const std::vector<cplx>& g, const int* lt, int nt, const int* lc, int nc)
{
    uint64_t tmask = 0, cmask = 0;
    for (int j = 0; j < nt; ++j) tmask |= 1ull << lt[j];
    for (int j = 0; j < nc; ++j) cmask |= 1ull << lc[j];
    const int d = 1 << nt;
    uint64_t idx[4];
    cplx w[4];
    for (uint64_t i = 0; i < (1ull << k); ++i) {
        if ((i & tmask) || (i & cmask) != cmask) continue;
        for (int r = 0; r < d; ++r) {
            uint64_t o = i;
            for (int j = 0; j < nt; ++j)
                if ((r >> (nt - 1 - j)) & 1) o |= 1ull << lt[j];
            idx[r] = o;
        }
        for (int r = 0; r < d; ++r) {
            cplx acc = 0;
            for (int c2 = 0; c2 < d; ++c2) acc += g[r * d + c2] * v[idx[c2]];
            w[r] = acc;
        }
        for (int r = 0; r < d; ++r) v[idx[r]] = w[r];
    }
}

struct BlockPlan {
    std::vector<std::vector<int>> blocks;  // op indices in application order
    std::vector<uint64_t> qubits;          // qubit mask of each block
};

// Greedy, commutation-aware packing: a block starts from the earliest
// unscheduled op and keeps absorbing a ready op (every earlier op sharing a
// qubit with it already placed) that grows its qubit set least, while the
// set stays within k qubits.  Ops on more than k qubits form blocks alone.
static void plan_blocks(int n, const std::vector<OpRec>& ops, int k, BlockPlan& bp)
{
    const int nops = (int)ops.size();
    std::vector<std::vector<int>> qops(n);
    std::vector<uint64_t> mask(nops);
    for (int i = 0; i < nops; ++i) {
        mask[i] = op_qubit_mask(ops[i]);
        for (int q = 0; q < n; ++q)
            if ((mask[i] >> q) & 1) qops[q].push_back(i);
    }
    std::vector<size_t> head(n, 0);
    std::vector<char> done(nops, 0);
    auto ready = [&](int i) {
        for (int q = 0; q < n; ++q)
            if (((mask[i] >> q) & 1) && qops[q][head[q]] != i) return false;
        return true;
    };
    auto place = [&](int i) {
        for (int q = 0; q < n; ++q)
            if ((mask[i] >> q) & 1) ++head[q];
        done[i] = 1;
    };
    int next = 0;
    while (true) {
        while (next < nops && done[next]) ++next;
        if (next == nops) break;
        std::vector<int> blk{next};
        uint64_t S = mask[next];
        place(next);
        if (__builtin_popcountll(S) <= k) {
            while (true) {
                int best = -1, best_growth = 64;
                for (int q = 0; q < n; ++q) {
                    if (head[q] >= qops[q].size()) continue;
                    const int i = qops[q][head[q]];
                    if (done[i] || !ready(i) || __builtin_popcountll(S | mask[i]) > k) continue;
                    const int growth = __builtin_popcountll(mask[i] & ~S);
                    if (growth < best_growth || (growth == best_growth && i < best)) {
                        best = i;
                        best_growth = growth;
                    }
                }
                if (best < 0) break;
                blk.push_back(best);
                S |= mask[best];
                place(best);
            }
        }
        bp.blocks.push_back(blk);
        bp.qubits.push_back(S);
    }
}

static sv_status circuit_forward_blocks(sv_circuit c, sv_state st, const double* params, int k, int* n_dense)
{
    BlockPlan bp;
    plan_blocks(c->n, c->ops, k, bp);
    int dense = 0;
    std::vector<cplx> g, M, col;
    for (size_t b = 0; b < bp.blocks.size(); ++b) {
        const std::vector<int>& blk = bp.blocks[b];
        uint64_t S = bp.qubits[b];
        if (blk.size() == 1) {  // a lone op keeps its own kernel
            Plan pl;
            sv_status rc = op_plan(c, st->dtype, c->ops[blk[0]], params, 0, &pl);
            if (!rc) rc = run_plan(pl, st, st->data);
            if (rc) return rc;
            continue;
        }
        // the matrix cores take 4..6 qubits: pad with the lowest qubits outside the block
        for (int q = 0; q < st->n && __builtin_popcountll(S) < kDenseMinK; ++q) S |= 1ull << q;
        std::vector<int> Q;  // block qubits, first = matrix MSB (descending)
        for (int q = st->n - 1; q >= 0; --q)
            if ((S >> q) & 1) Q.push_back(q);
        const int kb = (int)Q.size();
        int pos[64];  // qubit -> local bit of the matrix index
        for (int j = 0; j < kb; ++j) pos[Q[j]] = kb - 1 - j;
        const size_t d = (size_t)1 << kb;
        M.assign(d * d, 0);
        col.assign(d, 0);
        std::vector<std::vector<cplx>> mats(blk.size());
        for (size_t t = 0; t < blk.size(); ++t) op_target_matrix(c->ops[blk[t]], params, mats[t]);
        for (size_t cc = 0; cc < d; ++cc) {
            std::fill(col.begin(), col.end(), cplx(0));
            col[cc] = 1;
            for (size_t t = 0; t < blk.size(); ++t) {
                const OpRec& o = c->ops[blk[t]];
                int lt[2], lc[SV_OP_MAX_QUBITS];
                for (int j = 0; j < o.nc; ++j) lc[j] = pos[o.q[j]];
                for (int j = 0; j < o.nt; ++j) lt[j] = pos[o.q[o.nc + j]];
                apply_local(col.data(), kb, mats[t], lt, o.nt, lc, o.nc);
            }
            for (size_t r = 0; r < d; ++r) M[r * d + cc] = col[r];
        }
        sv_status rc = apply_dense(st, Q.data(), kb, (const double*)M.data());
        if (rc) return rc;
        ++dense;
    }
    if (n_dense) *n_dense = dense;
    return SV_OK;
}

sv_status sv_circuit_apply_blocks(sv_circuit c_h, sv_state st_h, const double* params, int k, int* n_dense_blocks)
{
    SV_CIRC(c);
    SV_STATE(st);
    if (st->n != c->n) return set_error(SV_ERR_ARG, "state size does not match the circuit");
    if (c->n_params > 0 && !params) return set_error(SV_ERR_ARG, "null params");
    if (k < kDenseMinK || k > kDenseMaxK) return set_error(SV_ERR_ARG, "block size must be 4..6 qubits");
    if (st->n < kDenseMinK) return set_error(SV_ERR_ARG, "dense blocks need a state of at least 4 qubits");
    return circuit_forward_blocks(c, st, params, k, n_dense_blocks);
}

sv_status sv_block_plan(int n_qubits, const sv_op* ops, int n_ops, int k, int64_t* info)
{
    if (!info) return set_error(SV_ERR_ARG, "null info");
    if (k < kDenseMinK || k > kDenseMaxK) return set_error(SV_ERR_ARG, "block size must be 4..6 qubits");
    if (n_qubits < 1 || n_qubits > SV_MAX_QUBITS) return set_error(SV_ERR_ARG, "n_qubits out of range");
    if (n_ops < 0 || (n_ops > 0 && !ops)) return set_error(SV_ERR_ARG, "bad op list");
    std::vector<OpRec> recs(n_ops);
    for (int i = 0; i < n_ops; ++i) {
        const sv_op& so = ops[i];
        OpRec& o = recs[i];
        o.gate = so.gate;
        o.nc = so.n_controls;
        o.nt = so.n_targets;
        if (o.nc < 0 || o.nt < 1 || o.nc + o.nt > SV_OP_MAX_QUBITS)
            return set_error(SV_ERR_ARG, "op " + std::to_string(i) + ": bad qubit counts");
        for (int j = 0; j < o.nc + o.nt; ++j) o.q[j] = so.qubits[j];
        sv_status rc = check_qubits(n_qubits, o.q, o.nc, o.q + o.nc, o.nt);
        if (rc) return rc;
    }
    BlockPlan bp;
    plan_blocks(n_qubits, recs, k, bp);
    int64_t dense = 0, single = 0, in_dense = 0, widest = 0;
    for (size_t b = 0; b < bp.blocks.size(); ++b) {
        if (bp.blocks[b].size() == 1) ++single;
        else {
            ++dense;
            in_dense += (int64_t)bp.blocks[b].size();
        }
        widest = std::max<int64_t>(widest, __builtin_popcountll(bp.qubits[b]));
    }
    info[0] = dense;
    info[1] = single;
    info[2] = in_dense;
    info[3] = widest;
    return SV_OK;
}

sv_status sv_circuit_apply(sv_circuit c_h, sv_state st_h, const double* params)
{
    SV_CIRC(c);
    SV_STATE(st);
    if (st->n != c->n) return set_error(SV_ERR_ARG, "state size does not match the circuit");
    if (c->n_params > 0 && !params) return set_error(SV_ERR_ARG, "null params");
    return circuit_forward(c, st, params);
}

template <typename T>
static hipError_t apply_obs_lambda(sv_state psi, sv_state lam, const ObsPlan& op)
{
    const int n = psi->n;
    hipStream_t s = psi->stream;
    hipError_t e;
    if (op.diag_kind > 0) {
        e = launch_obs_diag_apply<T>(psi->data, lam->data, n, op.diag_kind, op.diag_coeff, nullptr, nullptr, 0, 0, s);
    } else if (op.diag_kind == 0) {
        e = hipSuccess;
        for (size_t k0 = 0; k0 < op.dc.size() && e == hipSuccess; k0 += kDiagTermsPerPass) {
            const int nt = (int)std::min<size_t>(kDiagTermsPerPass, op.dc.size() - k0);
            e = launch_obs_diag_apply<T>(psi->data, lam->data, n, 0, 1.0, &op.dc[k0], &op.dz[k0], nt, k0 > 0, s);
        }
    } else {
        // lambda = 0 (no diagonal part): o(x) = 0 with an empty term list
        e = launch_obs_diag_apply<T>(psi->data, lam->data, n, 0, 1.0, nullptr, nullptr, 0, 0, s);
    }
    for (size_t k = 0; k < op.oc.size() && e == hipSuccess; ++k)
        e = launch_obs_pauli_apply<T>(psi->data, lam->data, n, op.ox[k], op.oz[k], op.oy[k], op.oc[k], s);
    return e;
}

static int gen_of(int gate)
{
    switch (gate) {
    case SV_RX: return GEN_X;
    case SV_RY: return GEN_Y;
    case SV_RZ: return GEN_Z;
    default: return GEN_P1;
    }
}

// U^dagger of a parameterised one-target op as a dense 2x2
static void rot_dagger(int gate, double th, double* m)
{
    const double c = cos(th / 2), s = sin(th / 2);
    double r[8] = {0};
    switch (gate) {
    case SV_RX: { double t[8] = {c, 0, 0, s, 0, s, c, 0}; memcpy(r, t, sizeof t); break; }
    case SV_RY: { double t[8] = {c, 0, s, 0, -s, 0, c, 0}; memcpy(r, t, sizeof t); break; }
    case SV_RZ: { double t[8] = {c, s, 0, 0, 0, 0, c, -s}; memcpy(r, t, sizeof t); break; }
    default: { double t[8] = {1, 0, 0, 0, 0, 0, cos(th), -sin(th)}; memcpy(r, t, sizeof t); break; }
    }
    memcpy(m, r, sizeof r);
}

template <typename T>
static sv_status adjoint_sweep(sv_circuit c, sv_state psi, sv_state lam, const double* params)
{
    hipStream_t s = psi->stream;
    int slot = c->n_slots - 1;
    for (int k = (int)c->ops.size() - 1; k >= 0; --k) {
        const OpRec& o = c->ops[k];
        if (o.pidx >= 0) {
            const double th = params[o.pidx];
            const int t = o.q[o.nc];
            int ins[kMaxIns];
            uint64_t cmask = 0;
            for (int j = 0; j < o.nc; ++j) {
                ins[j] = o.q[j];
                cmask |= 1ull << o.q[j];
            }
            ins[o.nc] = t;
            const GroupSpec gs = make_groups(c->n, ins, o.nc + 1, cmask);
            double md[8];
            rot_dagger(o.gate, th, md);
            Coef2<T> u;
            for (int i = 0; i < 8; ++i) u.m[i] = (T)md[i];
            hipError_t e = launch_adj_rot<T>(psi->data, lam->data, gs, 1ull << t, gen_of(o.gate), u,
                                             c->d_partials + (size_t)slot * c->seg, c->seg, s);
            if (e != hipSuccess) return hip_status(e, "adjoint step");
            --slot;
        } else {
            Plan pl;
            sv_status rc = op_plan(c, psi->dtype, o, params, 1, &pl);
            if (rc) return rc;
            rc = run_plan(pl, psi, psi->data);
            if (rc) return rc;
            rc = run_plan(pl, psi, lam->data);
            if (rc) return rc;
        }
    }
    return SV_OK;
}

sv_status sv_adjoint_grad(sv_circuit c_h, sv_state psi_h, sv_state lam_h, const double* params, const sv_obs* obs,
                          double* expval_out, double* grad_out)
{
    SV_CIRC(c);
    SV_STATE(psi);
    SV_STATE(lam);
    if (psi == lam) return set_error(SV_ERR_ARG, "psi and lam must be different states");
    if (psi->n != c->n || lam->n != c->n || psi->dtype != lam->dtype)
        return set_error(SV_ERR_ARG, "state sizes/dtypes do not match the circuit");
    if (c->n_params > 0 && (!params || !grad_out)) return set_error(SV_ERR_ARG, "null params or grad_out");
    ObsPlan op;
    sv_status rc = plan_obs(c->n, obs, &op);
    if (rc) return rc;
    if (psi->stream != lam->stream) {
        // keep all work on psi's stream: lam must be idle first
        (void)hipStreamSynchronize(lam->stream);
    }
    rc = circuit_forward(c, psi, params);
    if (rc) return rc;
    const bool d = psi->dtype == SV_C128;
    hipError_t e = d ? apply_obs_lambda<double>(psi, lam, op) : apply_obs_lambda<float>(psi, lam, op);
    const uint64_t na = 1ull << c->n;
    if (e == hipSuccess)
        e = d ? launch_inner_partial<double>(psi->data, lam->data, na, c->d_misc + 8, psi->stream)
              : launch_inner_partial<float>(psi->data, lam->data, na, c->d_misc + 8, psi->stream);
    if (e == hipSuccess) e = launch_sum_partials(c->d_misc + 8, reduce_blocks_for(na), c->d_misc, psi->stream);
    rc = hip_status(e, "adjoint setup");
    if (rc) return rc;
    rc = d ? adjoint_sweep<double>(c, psi, lam, params) : adjoint_sweep<float>(c, psi, lam, params);
    if (rc) return rc;
    e = launch_sum_segments(c->d_partials, c->seg, c->n_slots, nullptr, c->d_slot_val, psi->stream);
    if (e == hipSuccess)
        e = launch_scatter_grads(c->d_slot_val, c->d_slot_param, c->d_slot_scale, c->n_slots, c->d_grad, c->n_params,
                                 psi->stream);
    if (e == hipSuccess && expval_out)
        e = hipMemcpyAsync(expval_out, c->d_misc, sizeof(double), hipMemcpyDeviceToHost, psi->stream);
    if (e == hipSuccess && c->n_params > 0)
        e = hipMemcpyAsync(grad_out, c->d_grad, sizeof(double) * c->n_params, hipMemcpyDeviceToHost, psi->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(psi->stream);
    return hip_status(e, "adjoint gradient");
}

// ---------------------------------------------------------------------------
// tuning + diagnostics
// ---------------------------------------------------------------------------
sv_status sv_tune_set(int kernel_class, int dtype, int tier, int block, int unroll, int nt)
{
    if (!g_tune_init) tune_defaults();
    if (kernel_class < 0 || kernel_class >= KC_COUNT || kernel_class == KC_RETIRED ||
        (dtype != SV_C64 && dtype != SV_C128) || tier < 0 || tier >= kTiers)
        return set_error(SV_ERR_ARG, "bad tuning key");
    if (block < 64 || block > 1024 || (block & 63))
        return set_error(SV_ERR_ARG, "block must be a multiple of 64 in [64, 1024]");
    if (unroll != 1 && unroll != 2 && unroll != 4) return set_error(SV_ERR_ARG, "unroll must be 1, 2 or 4");
    if (nt != 0 && nt != 1) return set_error(SV_ERR_ARG, "nt must be 0 or 1");
    g_tune[kernel_class][dtype == SV_C128 ? 1 : 0][tier] = Launch{block, unroll, nt};
    return SV_OK;
}

sv_status sv_set_block_order(int order)
{
    if (order < -1 || order > 1) return set_error(SV_ERR_ARG, "block order must be -1, 0 or 1");
    g_block_order = order;
    return SV_OK;
}

sv_status sv_get_block_order(int* order)
{
    if (!order) return set_error(SV_ERR_ARG, "null output");
    *order = block_order_override();
    return SV_OK;
}

sv_status sv_tune_get(int kernel_class, int dtype, int tier, int* block, int* unroll, int* nt)
{
    if (!g_tune_init) tune_defaults();
    if (kernel_class < 0 || kernel_class >= KC_COUNT || (dtype != SV_C64 && dtype != SV_C128) || tier < 0 ||
        tier >= kTiers || !block || !unroll || !nt)
        return set_error(SV_ERR_ARG, "bad tuning key");
    const Launch l = g_tune[kernel_class][dtype == SV_C128 ? 1 : 0][tier];
    *block = l.block;
    *unroll = l.unroll;
    *nt = l.nt;
    return SV_OK;
}

sv_status sv_plan_info(int n_qubits, int dtype, int gate, const int* controls, int nc, const int* targets, int nt,
                       int* kernel_class, int* tier, int* op, int* block, int* unroll, int* nt_flag)
{
    if (n_qubits < 1 || n_qubits > SV_MAX_QUBITS || (dtype != SV_C64 && dtype != SV_C128))
        return set_error(SV_ERR_ARG, "n_qubits or dtype out of range");
    if (!kernel_class || !tier || !op || !block || !unroll || !nt_flag) return set_error(SV_ERR_ARG, "null output");
    int kc, low, opv = 0, lds_h = 0;
    if (gate == -1) {  // the general dense kernel on `targets`
        if (nt < 1 || nt > SV_MAX_GENERAL_K || nc != 0) return set_error(SV_ERR_ARG, "general gate needs 1..3 targets");
        sv_status rc = check_qubits(n_qubits, nullptr, 0, targets, nt);
        if (rc) return rc;
        kc = KC_GENERAL;
        low = 64;
        for (int j = 0; j < nt; ++j) low = std::min(low, targets[j]);
        opv = nt;
        if (nt == 1 && targets[0] < 6) {
            kc = KC_WAVE;
            opv = PAIR_DENSE;
            low = 64;
        } else if (lds_eligible(n_qubits, dtype, targets, nt)) {
            kc = KC_LDS;
            opv = nt << 4;
            for (int j = 0; j < nt; ++j) lds_h += targets[j] >= kLdsChunkBits;
        }
    } else {
        Plan pl;
        const double zero = 0.0;
        double mtx[32] = {0};
        sv_status rc = build_plan(n_qubits, dtype, gate, controls, nc, targets, nt, &zero, mtx, 0, &pl);
        if (rc) return rc;
        if (pl.kind == PK_NOP) return set_error(SV_ERR_ARG, "identity launches nothing");
        kc = pl.kc;
        low = pl.low;
        opv = pl.kind == PK_LDS ? ((pl.lk << 4) | pl.op) : pl.op;
        if (pl.kind == PK_LDS) lds_h = pl.ls.h;
    }
    const Launch l = tune_get(kc, dtype, low);
    *kernel_class = kc;
    *tier = shape_tier(dtype, low);
    *op = opv;
    *block = kc == KC_LDS ? lds_block(opv >> 4, lds_h, opv & 15, (int)elem_bytes(dtype), l.block) : l.block;
    *unroll = kc == KC_LDS ? lds_stage_depth(opv >> 4, l.unroll, (int)elem_bytes(dtype)) : l.unroll;
    *nt_flag = l.nt;
    return SV_OK;
}

const char* sv_last_error(void) { return g_last_error.c_str(); }

const char* sv_status_string(sv_status s)
{
    switch (s) {
    case SV_OK: return "SV_OK";
    case SV_ERR_ARG: return "SV_ERR_ARG";
    case SV_ERR_QUBIT: return "SV_ERR_QUBIT";
    case SV_ERR_OOM: return "SV_ERR_OOM";
    case SV_ERR_HIP: return "SV_ERR_HIP";
    case SV_ERR_UNSUPPORTED: return "SV_ERR_UNSUPPORTED";
    case SV_ERR_HANDLE: return "SV_ERR_HANDLE";
    }
    return "unknown";
}

int sv_version(void) { return 1; }

