// sv_pass.h -- tables shared by the fused pass engine (k_pass.hip) and its
// host-side compiler (sv_batch.hip).
#pragma once

#include "sv_core.h"

namespace svk {

constexpr int kMaxPassSlots = 64;  // parameterised ops per pass (LDS partial slots)
constexpr int kMaxTileQubits = 13;
// Register-tiled passes: each thread holds 2^rb amplitudes of the tile;
// a workgroup has at most kMaxPassThreads threads (2^(tq - rb)).
constexpr int kMinRegBits = 3, kMaxRegBits = 4;
constexpr int kMaxPassThreads = 512;
// LDS swizzle group: a tile-local index l is stored at l ^ fold(l), where
// fold XORs every higher group of kSwzBits bits into the lowest group, so
// lanes whose lowest kSwzBits lane bits sit at positions of distinct
// residues mod kSwzBits hit distinct banks.
constexpr int kSwzBits = 4;

// FK_PAIR: complex 2x2 on a target; FK_PAIRR: real 2x2 (H, RY); FK_PAIRX: the
// exchange of the pair (X).  All three keep the complex 2x2 in the coefficient
// table, so the LDS-sweep form treats them alike.  FK_PAIRC (forward lists
// only): a complex 2x2 on target a that depends on one selector bit b, the
// first matrix where bit b is 0 and the second where it is 1 (16 doubles): a
// run of one-target gates on a in which some gates are controlled by b, such
// as a rotation followed by a CNOT from b.  FK_PAIRT (forward lists only): a
// complex 2x2 on target a chosen per tile by the bits of b, a packed mask of
// qubits outside the tile (as below): a run of one-target gates on a whose
// controls all lie outside the tile, where each gate acts on the tiles holding
// its controls.  Its coefficients are 2^popcount(b) matrices of 8 doubles,
// entry e for the tiles whose bits under b, gathered in order, read e.
// FK_RFUSE (reverse lists only): two one-target gates A then B on one target
// with the same controls, un-applied as one complex 2x2 (coefficients: the
// product B A, then M = B G_A B^dagger for A's generator G_A); slot and gen
// are B's, b is A's slot (-1: none): the kernel takes B's gradient partial
// with B's generator and A's with M, both before the un-apply, which is the
// same as taking A's after un-applying B.
enum FusedKind : int32_t {
    FK_PAIR = 0, FK_DIAG = 1, FK_PHASE = 2, FK_SWAP = 3, FK_QUAD = 4, FK_LAYOUT = 5, FK_PAIRR = 6, FK_PAIRX = 7,
    FK_PAIRC = 8, FK_PAIRT = 9, FK_RFUSE = 10
};
// Largest packed mask of an FK_PAIRT (bits), so its table holds at most 32
// matrices.
constexpr int kMaxTileSelBits = 5;

// One op of a pass, in tile-local bit positions.  FK_LAYOUT (register-tiled
// passes only) re-distributes the tile: a = index of the layout that holds
// from here on, b = the layout that held before.
//
// Bits outside the tile are constant over a tile, so an op whose controls lie
// there acts on a tile only if the tile holds them all.  A one-target op
// (FK_PAIR, FK_PAIRR, FK_PAIRX, FK_DIAG) needs only its target in the tile;
// a subset phase (FK_PHASE: Z, S, T, PHASE with any controls) multiplies the
// amplitudes holding every bit of its mask, which makes it diagonal in all of
// them, so it needs just one of its bits in the tile (a).  Bits inside the
// tile are local bits in cm; for these kinds b holds the op's bits outside
// the tile, packed as a tile index is (bit i = the i-th lowest qubit outside
// the tile; 0: none), and the kernels test (tile & b) == b.  In forward lists
// an FK_PHASE's kb = 1 chains it to the next op, a subset phase on the same
// local mask whose phase the kernel multiplies in before applying the
// group's product once; kb = 2 makes it a member of a run on target a whose
// next op is a member too, kb = 3 the run's last member: each member's
// in-tile mask is a, or a and one lane bit, and the run's product (per lane:
// a member with a lane bit counts on the lanes holding it) is applied once
// to the amplitudes holding a (reverse sweeps ignore kb).
struct FOp {
    int32_t kind;
    int32_t a, b;   // local target bits (b: second target of SWAP / QUAD, selector of FK_PAIRC, packed mask
                    // of the out-of-tile bits of one-target kinds, FK_PHASE and FK_PAIRT)
    uint32_t cm;    // local bits that must all be 1 (controls; for FK_PHASE also the target)
    int32_t coef;   // offset of the op's coefficients in the coefficient table (doubles)
    int32_t slot;   // gradient slot within the circuit, -1 if not parameterised
    int8_t gen;     // generator (GenKind) of a parameterised op
    // Register-tiled passes, for the layout the op runs in: the register bits
    // holding a and b (-1 where the bit is a lane bit; b for SWAP, QUAD and
    // FK_PAIRC), and cm split into its
    // register bits (as register indices, cmk) and its lane bits (cml).
    int8_t ka, kb;
    uint8_t cmk;
    uint32_t cml;
};

// A distribution of a tile over the threads of a workgroup: lane bit i of
// the thread index is tile-local bit pos[i] (i < tq - rb), register bit r is
// tile-local bit pos[tq - rb + r].  A layout belongs to one pass, so the
// tile-local and global bit values are stored ready for use (zero past the
// lane bits).
struct FLayout {
    uint8_t pos[16];
    uint16_t lane_l[16];  // 1 << pos[i] for lane bit i
    uint16_t reg_l[4];    // 1 << pos[tq - rb + r]
    uint32_t pad_;
    uint64_t lane_g[16];  // global bit of lane bit i: 1 << q[pos[i]]
    uint64_t reg_g[4];    // global bit of register bit r
};

// A pass has two op lists over the same ops: the forward list (planned for
// the forward register width) and the list the reverse sweep walks backwards
// (planned for the reverse width; the same range when the widths agree).
struct FPass {
    int32_t q[16];  // tile qubits, ascending; local bit k <-> global qubit q[k]
    int32_t op_begin, op_end;
    int32_t lay_begin, lay_end;  // layouts a register-tiled forward pass loads in and ends in
    int32_t rop_begin, rop_end;
    int32_t rlay_begin, rlay_end;
    uint64_t free_mask;  // global bits outside the tile (the tile index is deposited into them)
    int32_t gated;       // 1 if a one-target op of the forward list has controls outside the tile
    int32_t pad_;
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
    int32_t reg;           // 1: forward passes are register-tiled (tq >= rb); 0: every op sweeps an LDS tile
    int32_t rreg;          // the same for reverse passes (tq >= reverse rb)
    int32_t pad_;
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
// A fused op (several one-target gates on the same target and controls in a
// row, forward passes only) has nfactor > 0: its coefficients are the
// product of the factor gates' 2x2 matrices, factors [factor_begin,
// factor_begin + nfactor) of the factor table in the order applied; each
// factor is an FCoefSpec whose fixed[0..7] holds the full 2x2 of a fixed gate.
// out_diag = 1 writes the product's diagonal only (d0, d1); 2 writes two
// products (FK_PAIRC: 16 values), each factor entering the first, the second
// or both as its `branch` says (1, 2, 3); 3 writes 2^popcount(branch)
// products (FK_PAIRT: the spec's branch is the op's packed mask), product e
// taking the factors whose own packed mask (their `branch`) lies within the
// bits that e selects; 4 (FK_RFUSE, two factors A then B) writes B A and,
// if the spec's branch is 1 + A's generator kind, B G_A B^dagger (16 values);
// 0 writes all 8 values.
struct FCoefSpec {
    int32_t gate;
    int32_t pidx;    // global parameter index, -1 = fixed angle `value`
    int32_t coef;    // destination offset
    int32_t nfixed;  // fixed coefficient count (non-rotation gates)
    double value;
    double fixed[32];
    int32_t nfactor, factor_begin;
    int32_t out_diag;
    int32_t branch;  // factor entries of an out_diag = 2 or 3 product; the op's mask of an out_diag = 3 spec
};

struct PassTables {
    const FCirc* circs;
    const FPass* passes;
    const FOp* ops;
    const FLayout* lays;
    const FSeg* segs;
    const double* coef;
    const float* coef_f;  // the same coefficients rounded to float (complex64 runs)
    double* e_part;
    double* g_part;
    int64_t n_items;
    int32_t n_segs;
    int32_t tq_max;
    int32_t with_grad;
    int32_t hi_entries;  // LDS address-map entries: max over circuits of 2^(tq - cb)
    int32_t reg_bits;    // rb of register-tiled forward passes
    int32_t rreg_bits;   // rb of register-tiled reverse passes
    int32_t lds_small;   // 1 if some circuit takes the LDS-sweep form (tq < rb)
};

enum PassMode : int { PM_FWD = 0, PM_OBS = 1, PM_REV = 2 };
// Raise the engine kernels' dynamic LDS limit to at least lds_bytes (outside
// any graph capture).
hipError_t pass_engine_prepare(size_t lds_bytes);
// Items [item_begin, item_end), all of stage kind `mode`, one workgroup per tile.
// gated: some forward pass among the items has FPass.gated set.
hipError_t launch_pass_items(const PassTables& tb, int dtype, int mode, int64_t item_begin, int64_t item_end,
                             int threads, size_t lds_bytes, hipStream_t s, bool gated = false);
hipError_t launch_pass_coef(const FCoefSpec* spec, int n, const FCoefSpec* factors, const double* params,
                            double* coef, float* coef_f, hipStream_t s);
hipError_t launch_pass_segsum(const double* part, const int64_t* off, const int* cnt, const double* scale, double* out,
                              int n_seg, hipStream_t s);
hipError_t launch_pass_grad_csr(const double* slot_val, const int* rowptr, const int* cols, int n_params, double* grad,
                                hipStream_t s);
// Dynamic LDS of a pass workgroup: tiles and address map, plus per-slot wave
// partials for slot_waves waves (reverse passes; 0 for forward ones).
size_t pass_engine_lds_bytes(int tq_max, int hi_entries, int with_grad, int dtype, int lds_small, int slot_waves);
// Workgroup size for register width rb: 2^(tq_max - rb), at least one wavefront.
int pass_engine_threads(int tq_max, int reg_bits);

}  // namespace svk
