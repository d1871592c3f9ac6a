// sv_pass.h -- tables shared by the fused pass engine (k_pass.hip) and its
// host-side compiler (sv_batch.hip).
#pragma once

#include "sv_core.h"

namespace svk {

constexpr int kMaxPassSlots = 64;  // parameterised ops per pass (LDS partial slots)
constexpr int kMaxTileQubits = 13;

enum FusedKind : int32_t { FK_PAIR = 0, FK_DIAG = 1, FK_PHASE = 2, FK_SWAP = 3, FK_QUAD = 4 };

// One op of a pass, in tile-local bit positions.
struct FOp {
    int32_t kind;
    int32_t a, b;   // local target bits (b: second target of SWAP / QUAD)
    uint32_t cm;    // local bits that must all be 1 (controls; for FK_PHASE also the target)
    int32_t coef;   // offset of the op's coefficients in the coefficient table (doubles)
    int32_t slot;   // gradient slot within the circuit, -1 if not parameterised
    int32_t gen;    // generator (GenKind) of a parameterised op
    int32_t pad;
};

struct FPass {
    int32_t q[16];  // tile qubits, ascending; local bit k <-> global qubit q[k]
    int32_t op_begin, op_end;
};

struct FCirc {
    void* psi;
    void* lam;
    int64_t g_part_begin;  // offset of this circuit's [slot][tile] gradient partials
    int32_t n, tq;
    int32_t n_tiles;       // 2^(n - tq)
    int32_t n_pass;        // forward passes (stages: passes, observable, reverse passes)
    int32_t pass_begin;
    int32_t obs_kind;      // 1 = sum_i Z_i, 2 = sum_i Z_i Z_{i+1}
    int32_t e_part_begin;
    int32_t cb;            // coalescing bits: every pass's tile holds global bits 0..cb-1 as local bits 0..cb-1
};

// Items [first, first + n_tiles) are the tiles of stage `stage` of `circ`;
// items are ordered level by level, so each stage level is a contiguous range.
struct FSeg {
    int64_t first;
    int32_t circ;
    int32_t stage;
    int32_t n_tiles;
    int32_t pad;
};

// Per-op coefficient recipe (evaluated on the device from the parameters).
struct FCoefSpec {
    int32_t gate;
    int32_t pidx;    // global parameter index, -1 = fixed angle `value`
    int32_t coef;    // destination offset
    int32_t nfixed;  // fixed coefficient count (non-rotation gates)
    double value;
    double fixed[32];
};

struct PassTables {
    const FCirc* circs;
    const FPass* passes;
    const FOp* ops;
    const FSeg* segs;
    const double* coef;
    double* e_part;
    double* g_part;
    int64_t n_items;
    int32_t n_segs;
    int32_t tq_max;
    int32_t with_grad;
    int32_t hi_entries;  // LDS address-map entries: max over circuits of 2^(tq - cb)
};

// Set the engine's dynamic LDS limit (once, outside any graph capture).
hipError_t pass_engine_prepare(int dtype, size_t lds_bytes);
// Items [item_begin, item_end) of one stage level, one workgroup per tile.
hipError_t launch_pass_level(const PassTables& tb, int dtype, int64_t item_begin, int64_t item_end, int threads,
                             size_t lds_bytes, hipStream_t s);
hipError_t launch_pass_coef(const FCoefSpec* spec, int n, const double* params, double* coef, hipStream_t s);
hipError_t launch_pass_segsum(const double* part, const int64_t* off, const int* cnt, const double* scale, double* out,
                              int n_seg, hipStream_t s);
hipError_t launch_pass_grad_csr(const double* slot_val, const int* rowptr, const int* cols, int n_params, double* grad,
                                hipStream_t s);
size_t pass_engine_lds_bytes(int tq_max, int hi_entries, int with_grad, int dtype);

}  // namespace svk
