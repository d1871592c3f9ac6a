// sv_core.h -- internal declarations of libsv (kernels <-> host dispatch).
//
// Index generation (Sec. 2: a gate acts on the groups of amplitudes that
// differ only in the gate's qubits; a control selects where it acts): group g
// in [0, 2^(N - nins)) maps to the base index obtained by inserting a zero bit
// at each position of `pos` (ascending) and OR-ing `set_mask` (control bits,
// plus target bits for gates that touch only the |1> subspace).  Members of a
// group are base + offset[r].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/sv.h"

namespace svk {

constexpr int kMaxIns = 12;  // controls + targets inserted into a group index

struct GroupSpec {
    uint64_t n_groups;
    uint64_t set_mask;
    // Predicate: the gate acts on a group iff (base & pmask) == pmask.  Control
    // (or target) bits whose runs would span under 128 bytes are predicated
    // instead of inserted, so every access stays on whole cache lines; groups
    // that fail the predicate are written back unchanged.
    uint64_t pmask;
    int32_t nins;
    // Order in which the workgroups walk the groups (block_slot): 0 = launch
    // order, 1 = one contiguous eighth of the grid per XCD.
    int32_t order;
    int32_t pos[kMaxIns];
};

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

// Operation kinds of the paired (two-member) kernel.
enum PairOp : int {
    PAIR_SWAP = 0,  // permutation: (a, b) -> (b, a)
    PAIR_Y = 1,     // (a, b) -> (-i b, i a)
    PAIR_REAL = 2,  // real 2x2 (H, RY)
    PAIR_RX = 3,    // [[c, -i s], [-i s, c]]
    PAIR_DENSE = 4, // complex 2x2 (U2 and anything else)
    PAIR_DIAG = 5   // diag(m00, m11): each member times its own phase (RZ); no partner needed
};

// Operation kinds of the single-member (subset-diagonal) kernel.
enum OneOp : int {
    ONE_NEG = 0,   // a -> -a (Z, CZ)
    ONE_MULI = 1,  // a -> s * i * a with s = +-1 (S, S^dagger)
    ONE_MUL = 2    // a -> z * a (T, PHASE, controlled phase)
};

template <typename T>
struct Coef2 {  // 2x2 complex, row-major interleaved: m00 m01 m10 m11
    T m[8];
};

template <typename T>
struct Coef4 {  // 4x4 complex
    T m[32];
};

template <typename T, int K>
struct GeneralSpec {  // dense 2^K x 2^K, all groups, no structure used
    uint64_t off[1 << K];
    T m[2 * (1 << K) * (1 << K)];
};

// Row a2 of the method on the device: group index -> base amplitude index.
__device__ __forceinline__ uint64_t group_base(uint64_t g, const GroupSpec& gs)
{
#pragma unroll
    for (int i = 0; i < kMaxIns; ++i) {
        if (i < gs.nins) {
            const int p = gs.pos[i];
            const uint64_t lo = g & ((1ull << p) - 1ull);
            g = ((g >> p) << (p + 1)) | lo;
        }
    }
    return g | gs.set_mask;
}

// The place of workgroup b (of G) in a walk over the groups.  The hardware
// deals consecutive workgroups to the 8 XCDs in turn.  order 0 keeps launch
// order, so at any moment the whole chip streams one narrow window of the
// state (plus the windows of the gate's partner offsets); order 1 gives XCD x
// (the workgroups b = x mod 8) the x-th contiguous eighth of the grid, so the
// chip streams 8 windows an eighth of the state apart, which measured faster
// on MI355X for complex128 gates with a member offset of 32-128 MiB (the host
// picks the order per launch).  Any G: XCD x owns floor(G/8) slots, plus one
// if x < G mod 8.
__device__ __forceinline__ uint64_t block_slot(uint32_t b, uint32_t G, int order)
{
    if (!order) return b;
    const uint32_t x = b & 7u, q = G >> 3, r = G & 7u;
    return (uint64_t)x * q + (x < r ? x : r) + (b >> 3);
}

// LDS-staged single gate: a block stages 2^(kLdsChunkBits + h) amplitudes --
// 2^h contiguous chunks of 2^kLdsChunkBits, one per combination of the h gate
// qubits at or above kLdsChunkBits -- applies the gate to every group inside
// the stage and streams the chunks back.
constexpr int kLdsChunkBits = 8;
// Lines a thread of the LDS-staged kernel moves per round trip between HBM
// and LDS for a k-qubit gate under a launch shape's unroll: the 3-qubit form
// stages `unroll`; the 2-qubit forms stage two in complex64 (8-byte
// amplitudes: a thread's single line leaves too few bytes in flight) and one
// in complex128, where more registers per thread cost more waves than the
// extra line brings.
inline int lds_stage_depth(int k, int unroll, int elem_bytes)
{
    if (k == 3) return unroll;
    return k == 2 && elem_bytes == 8 && unroll >= 2 ? 2 : 1;
}
// Workgroup size of the LDS-staged kernel for a stage of 2^(kLdsChunkBits + h)
// amplitudes: `a` amplitudes of the stage per thread -- 4 for complex128
// 2-qubit matrices, 2 for the complex128 SWAP move, 8 otherwise, the fastest
// counts measured on MI355X at 30 qubits over stages of 256 to 1024
// amplitudes (a workgroup of one wavefront on a 256-amplitude stage of a
// complex128 2-qubit matrix took 5.35 ms per gate against 5.82 with two) --
// at least one wavefront and at most `cap`, the launch shape's block.
inline int lds_block(int k, int h, int op, int elem_bytes, int cap)
{
    const int a = elem_bytes == 16 && k == 2 ? (op == 1 ? 2 : 4) : 8;
    const int want = (1 << (kLdsChunkBits + h)) / a;
    const int b = want < 64 ? 64 : want;
    return b < cap ? b : (cap < 64 ? 64 : cap);
}
struct LdsSpec {
    int32_t k;        // gate qubits (1..3)
    int32_t h;        // gate qubits >= kLdsChunkBits
    int32_t hq[3];    // those qubits, ascending (absolute positions)
    int32_t lpos[3];  // local bit of gate qubit j (j = 0 is the matrix MSB)
    int32_t lsort[3]; // lpos sorted ascending (group insertion order)
    uint32_t pmask;   // local bits (controls below kLdsChunkBits) that must be 1
    uint64_t cmask;   // absolute control bits at or above kLdsChunkBits (inserted, set to 1)
};

struct Launch {
    int block;   // threads per block
    int unroll;  // groups per thread (1, 2 or 4)
    int nt;      // 1: non-temporal loads and stores (streaming, no cache allocation)
};

// Global loads / stores of one complex amplitude, optionally non-temporal.
// The two scalar halves merge into one 16-byte (complex128) or 8-byte
// (complex64) access with the nt bit set.
template <bool NT, typename V>
__device__ __forceinline__ V ldg(const V* p)
{
    if constexpr (NT) {
        V r;
        r.x = __builtin_nontemporal_load(&p->x);
        r.y = __builtin_nontemporal_load(&p->y);
        return r;
    } else {
        return *p;
    }
}

template <bool NT, typename V>
__device__ __forceinline__ void stg(V* p, const V& v)
{
    if constexpr (NT) {
        __builtin_nontemporal_store(v.x, &p->x);
        __builtin_nontemporal_store(v.y, &p->y);
    } else {
        *p = v;
    }
}

// ---- launchers (k_gates.hip) --------------------------------------------
template <typename T>
hipError_t launch_pair(void* psi, const GroupSpec& gs, uint64_t o0, uint64_t o1, int op,
                       const Coef2<T>& c, hipStream_t s, Launch lc);
// Wavefront form of the paired update for a target t < 6: every lane owns one
// amplitude of a contiguous run (group_base over inserted bits >= 6 only), the
// partner amplitude x ^ 2^t sits in lane (lane ^ 2^t) of the same wavefront and
// is fetched with a cross-lane shuffle.
template <typename T>
hipError_t launch_wpair(void* psi, const GroupSpec& gs, int t, int op, const Coef2<T>& c, hipStream_t s,
                        Launch lc);
// op: 0 = dense 2^k x 2^k (m holds 2 * 4^k values), 1 = SWAP of the two
// gate qubits (k = 2; pure moves).  `tiles` enumerates stages: zero bits
// inserted at (p - kLdsChunkBits) for every inserted high position p, no set mask.
template <typename T>
hipError_t launch_lds_gate(void* psi, const GroupSpec& tiles, const LdsSpec& ls, int op, const T* m, hipStream_t s,
                           Launch lc);
template <typename T>
hipError_t launch_one(void* psi, const GroupSpec& gs, int op, T zr, T zi, hipStream_t s, Launch lc);
template <typename T>
hipError_t launch_quad(void* psi, const GroupSpec& gs, const uint64_t off[4], const Coef4<T>& c,
                       hipStream_t s, Launch lc);
template <typename T>
hipError_t launch_general(void* psi, const GroupSpec& gs, int k, const uint64_t* off, const T* m,
                          hipStream_t s, Launch lc);
template <typename T>
hipError_t launch_set_basis(void* psi, uint64_t n_amps, uint64_t index, hipStream_t s);

// ---- reductions (k_reduce.hip) -------------------------------------------
constexpr int kReduceBlocks = 1024;  // fixed stage-1 grid: results are order-stable
constexpr int kReduceThreads = 256;

template <typename T>
hipError_t launch_norm_partial(const void* psi, uint64_t n_amps, double* partials, hipStream_t s);
// One Pauli term: xmask == 0 -> sum |a|^2 (-1)^{pc(x&z)}; else paired form.
template <typename T>
hipError_t launch_pauli_partial(const void* psi, int n, uint64_t xmask, uint64_t zmask, int ny,
                                double coeff, double* partials, hipStream_t s);
// Diagonal observable sum_k c_k (-1)^{pc(x & z_k)}; kind 1 = sum Z, 2 = sum ZZ
// (closed forms, scaled by coeff), 0 = generic list of at most
// kDiagTermsPerPass host terms (passed by value in the kernel arguments).
constexpr int kDiagTermsPerPass = 32;
template <typename T>
hipError_t launch_diag_obs_partial(const void* psi, int n, int kind, double coeff,
                                   const double* hcoef, const uint64_t* hz, int nterms,
                                   double* partials, hipStream_t s);
// Number of stage-1 blocks (= partials written) for n_items work items.
int reduce_blocks_for(uint64_t n_items);
hipError_t launch_sum_partials(const double* partials, int count, double* out, hipStream_t s);
hipError_t launch_sum_segments(const double* partials, int seg_len, int n_seg, const double* scale,
                               double* out, hipStream_t s);

// ---- circuits / adjoint (k_adjoint.hip) -----------------------------------
// Generator kinds of parameterised ops: the gradient is
// scale * Im <lambda| G |phi> over the op's control subspace.
enum GenKind : int { GEN_X = 0, GEN_Y = 1, GEN_Z = 2, GEN_P1 = 3 };

// Fused reverse step of a parameterised one-target op: per group reads phi and
// lambda once, adds Im <lambda|G|phi> to a block partial, applies U^dagger to
// both and writes them back.  Exactly `nblocks` partials are written.
template <typename T>
hipError_t launch_adj_rot(void* phi, void* lam, const GroupSpec& gs, uint64_t off, int gen,
                          const Coef2<T>& udag, double* partials, int nblocks, hipStream_t s);
// lam = O psi for a diagonal observable (kind as launch_diag_obs_partial).
template <typename T>
hipError_t launch_obs_diag_apply(const void* psi, void* lam, int n, int kind, double coeff,
                                 const double* hcoef, const uint64_t* hz, int nterms, int accumulate,
                                 hipStream_t s);
// lam += coeff * P psi for one Pauli term with xmask != 0.
template <typename T>
hipError_t launch_obs_pauli_apply(const void* psi, void* lam, int n, uint64_t xmask, uint64_t zmask,
                                  int ny, double coeff, hipStream_t s);
// Re <a|b> block partials (fp64).
template <typename T>
hipError_t launch_inner_partial(const void* a, const void* b, uint64_t n_amps, double* partials,
                                hipStream_t s);
// grad[j] = sum over slots s with slot_param[s] == j of slot_scale[s] * slot_val[s],
// slots in ascending order (device arrays).
hipError_t launch_scatter_grads(const double* slot_val, const int* slot_param, const double* slot_scale,
                                int n_slots, double* grad, int n_params, hipStream_t s);

// ---- helpers ----------------------------------------------------------------
sv_status set_error(sv_status st, const std::string& msg);
// Handle table (states, circuits, batches): handle_put returns a new handle
// for obj; handle_get returns the object of a live handle of that kind, else
// nullptr; handle_drop does the same and invalidates every copy of the handle.
enum HandleKind : int { HK_STATE = 1, HK_CIRCUIT = 2, HK_BATCH = 3 };
void* handle_put(void* obj, int kind);
void* handle_get(const void* h, int kind);
void* handle_drop(const void* h, int kind);

}  // namespace svk
