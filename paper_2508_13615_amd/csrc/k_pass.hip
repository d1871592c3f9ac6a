// k_pass.hip -- fused pass engine: many circuits (or one large one), every
// stage of forward, measurement and adjoint sweep, one graph launch.
//
// A circuit's ops are grouped on the host into passes (sv_batch.hip): the
// ops of a pass touch only the qubits of a set Q with |Q| = tq, so the state
// splits into 2^(n - tq) independent tiles of 2^tq amplitudes (the amplitudes
// that differ only in Q's bits).  A work item is one tile of one stage:
//   forward pass p  load the tile into LDS (pass 0 builds |0...0> instead),
//                   apply the pass's ops in LDS, store it;
//   observable      lambda = O psi on a contiguous chunk and a partial of
//                   <psi|O|psi> (diagonal observables sum Z / sum ZZ);
//   reverse pass    load the phi and lambda tiles, walk the pass's ops
//                   backwards: a parameterised op first adds
//                   Im <lambda|G|phi> over the tile to a per-(op, tile)
//                   partial, then U^dagger is applied to both tiles; store.
// Each tile crosses HBM once per pass however many gates the pass holds
// (gate fusion), and the gates run against LDS.
//
// Scheduling: the items are ordered level by level (stage s of every circuit
// before stage s + 1), and each level is one kernel launch with one
// workgroup per tile.  Kernel boundaries order the stages and make every
// tile written by one level visible to the next on all XCDs; no workgroup
// ever waits on another.  All level launches of a run are captured once into
// a hipGraph and replayed.  (An earlier single persistent kernel synchronised
// stages with device-scope counters; on this multi-XCD part each acquire poll
// invalidates the L2, so waiting workgroups throttled the working ones.)
#include "sv_core.h"
#include "sv_pass.h"

namespace svk {

// The run's tables (segments, circuits, passes, layouts, ops, coefficients)
// are not written while a pass launch runs.  Reading them through the
// constant address space lets the compiler use scalar loads; through a
// generic pointer it must assume the state stores may alias them and
// fetch every uniform value with per-lane vector loads.
template <typename X>
using cptr = const __attribute__((address_space(4))) X*;

template <typename X>
__device__ __forceinline__ cptr<X> as_const(const X* p)
{
    return (cptr<X>)p;
}

// Copy of a table entry read through the constant address space.
template <typename X>
__device__ __forceinline__ X ld_const(cptr<X> p)
{
    static_assert(sizeof(X) % 4 == 0, "table entries are whole words");
    union {
        X x;
        uint32_t w[sizeof(X) / 4];
    } u;
    const cptr<uint32_t> q = (cptr<uint32_t>)p;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(X) / 4); ++i) u.w[i] = q[i];
    return u.x;
}

__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// (ar + i ai) a + (br + i bi) b.  In double precision as one multiply and
// three fused multiply-adds per component: those kernels are bound by vector
// instruction issue.  The float kernels are bound by dependency latency, and
// the shorter chains of two products summed suit them better.
template <typename V, typename T>
__device__ __forceinline__ V cmul_add2(T ar_, T ai_, V a, T br_, T bi_, V b)
{
    V r;
    if constexpr (sizeof(T) == 8) {
        r.x = fmadd(ar_, a.x, fmadd(-ai_, a.y, fmadd(br_, b.x, -bi_ * b.y)));
        r.y = fmadd(ar_, a.y, fmadd(ai_, a.x, fmadd(br_, b.y, bi_ * b.x)));
    } else {
        r.x = (ar_ * a.x - ai_ * a.y) + (br_ * b.x - bi_ * b.y);
        r.y = (ar_ * a.y + ai_ * a.x) + (br_ * b.y + bi_ * b.x);
    }
    return r;
}

__device__ __forceinline__ uint32_t ins0(uint32_t x, int p)
{
    const uint32_t lo = x & ((1u << p) - 1u);
    return ((x >> p) << (p + 1)) | lo;
}

// Coefficients of a 2x2 (row-major, interleaved) or its conjugate transpose.
template <typename T, typename P>
__device__ __forceinline__ void load2x2(P cf, bool dagger, T* u)
{
    if (!dagger) {
#pragma unroll
        for (int i = 0; i < 8; ++i) u[i] = (T)cf[i];
    } else {
        // (r, c) <- conj (c, r)
        u[0] = (T)cf[0]; u[1] = (T)-cf[1];
        u[2] = (T)cf[4]; u[3] = (T)-cf[5];
        u[4] = (T)cf[2]; u[5] = (T)-cf[3];
        u[6] = (T)cf[6]; u[7] = (T)-cf[7];
    }
}

// LDS address of tile-local index l in the register engine's exchange buffer.
__device__ __forceinline__ uint32_t swz(uint32_t l)
{
    // l < 2^16: fold bit groups [4, 8), [8, 12), [12, 16) into [0, 4)
    return l ^ (((l >> 4) ^ (l >> 8) ^ (l >> 12)) & ((1u << kSwzBits) - 1u));
}

// Apply one op (or its inverse) to an LDS tile of 2^tq amplitudes; with SWZ
// the tile is stored at swz(l) (the register engine's exchange layout).
template <typename T, bool SWZ = false, typename P = const double*>
__device__ void lds_apply(typename Vec2<T>::type* A0, const FOp op, P coef, bool dagger, int tq)
{
    using V = typename Vec2<T>::type;
    struct Tile {
        V* a;
        __device__ V& operator[](uint32_t i) const { return a[SWZ ? swz(i) : i]; }
    } A{A0};
    const int nthr = blockDim.x;
    const uint32_t cm = op.cm;
    const P cf = coef + op.coef;
    switch (op.kind) {
    case FK_PAIRX:
    case FK_PAIRR:
    case FK_PAIR: {
        T u[8];
        load2x2<T>(cf, dagger, u);
        const uint32_t np = 1u << (tq - 1);
        for (uint32_t p = threadIdx.x; p < np; p += nthr) {
            const uint32_t i0 = ins0(p, op.a);
            if ((i0 & cm) != cm) continue;
            const uint32_t i1 = i0 | (1u << op.a);
            const V v0 = A[i0], v1 = A[i1];
            A[i0] = cmul_add2<V, T>(u[0], u[1], v0, u[2], u[3], v1);
            A[i1] = cmul_add2<V, T>(u[4], u[5], v0, u[6], u[7], v1);
        }
        break;
    }
    case FK_DIAG: {  // element-wise d[bit a], entries cf[0..3] = d0 (re, im), d1 (re, im)
        const T d0r = (T)cf[0], d0i = (T)(dagger ? -cf[1] : cf[1]);
        const T d1r = (T)cf[2], d1i = (T)(dagger ? -cf[3] : cf[3]);
        const uint32_t na = 1u << tq;
        for (uint32_t i = threadIdx.x; i < na; i += nthr) {
            if ((i & cm) != cm) continue;
            const bool b = (i >> op.a) & 1u;
            const T zr = b ? d1r : d0r, zi = b ? d1i : d0i;
            const V v = A[i];
            V r;
            r.x = zr * v.x - zi * v.y;
            r.y = zr * v.y + zi * v.x;
            A[i] = r;
        }
        break;
    }
    case FK_PHASE: {  // z on the amplitudes whose bits cm are all 1 (cm includes the target)
        const T zr = (T)cf[0], zi = (T)(dagger ? -cf[1] : cf[1]);
        const uint32_t na = 1u << tq;
        for (uint32_t i = threadIdx.x; i < na; i += nthr) {
            if ((i & cm) != cm) continue;
            const V v = A[i];
            V r;
            r.x = zr * v.x - zi * v.y;
            r.y = zr * v.y + zi * v.x;
            A[i] = r;
        }
        break;
    }
    case FK_SWAP: {
        const int lo = op.a < op.b ? op.a : op.b, hi = op.a < op.b ? op.b : op.a;
        const uint32_t np = 1u << (tq - 2);
        for (uint32_t p = threadIdx.x; p < np; p += nthr) {
            const uint32_t base = ins0(ins0(p, lo), hi);
            if ((base & cm) != cm) continue;
            const uint32_t i = base | (1u << op.a), j = base | (1u << op.b);
            const V v = A[i];
            A[i] = A[j];
            A[j] = v;
        }
        break;
    }
    default: {  // FK_QUAD: 4x4 on local bits a (matrix MSB) and b
        const int lo = op.a < op.b ? op.a : op.b, hi = op.a < op.b ? op.b : op.a;
        const uint32_t np = 1u << (tq - 2);
        const uint32_t off[4] = {0u, 1u << op.b, 1u << op.a, (1u << op.a) | (1u << op.b)};
        for (uint32_t p = threadIdx.x; p < np; p += nthr) {
            const uint32_t base = ins0(ins0(p, lo), hi);
            if ((base & cm) != cm) continue;
            V v[4], r[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = A[base | off[k]];
#pragma unroll
            for (int row = 0; row < 4; ++row) {
                T sr = T(0), si = T(0);
#pragma unroll
                for (int col = 0; col < 4; ++col) {
                    const int e = dagger ? (4 * col + row) : (4 * row + col);
                    const T ur = (T)cf[2 * e], ui = (T)(dagger ? -cf[2 * e + 1] : cf[2 * e + 1]);
                    sr += ur * v[col].x - ui * v[col].y;
                    si += ur * v[col].y + ui * v[col].x;
                }
                r[row].x = sr;
                r[row].y = si;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) A[base | off[k]] = r[k];
        }
        break;
    }
    }
}

// FK_PAIRC on an LDS tile (forward passes of the LDS-sweep form): the 2x2
// cf[0..7] where bit b is 0, cf[8..15] where it is 1.  Kept out of lds_apply,
// which the register passes also inline with all their amplitudes live.
template <typename T>
__device__ void lds_pairc(typename Vec2<T>::type* A, const FOp op, const double* coef, int tq)
{
    using V = typename Vec2<T>::type;
    const double* cf = coef + op.coef;
    T u0[8], u1[8];
    load2x2<T>(cf, false, u0);
    load2x2<T>(cf + 8, false, u1);
    const uint32_t np = 1u << (tq - 1);
    for (uint32_t p = threadIdx.x; p < np; p += blockDim.x) {
        const uint32_t i0 = ins0(p, op.a);
        const uint32_t i1 = i0 | (1u << op.a);
        const T* u = ((i0 >> op.b) & 1u) ? u1 : u0;
        const V v0 = A[i0], v1 = A[i1];
        A[i0] = cmul_add2<V, T>(u[0], u[1], v0, u[2], u[3], v1);
        A[i1] = cmul_add2<V, T>(u[4], u[5], v0, u[6], u[7], v1);
    }
}

// Per-thread Im <lambda|G|phi> over the tile for a one-target generator on
// local bit a, restricted to the local control mask cm.
template <typename T>
__device__ double lds_gen_inner(const typename Vec2<T>::type* P, const typename Vec2<T>::type* L, const FOp& op,
                                int tq)
{
    double acc = 0.0;
    const uint32_t cm = op.cm & ~(1u << op.a);  // a subset-phase op lists its target in cm
    const uint32_t np = 1u << (tq - 1);
    for (uint32_t p = threadIdx.x; p < np; p += blockDim.x) {
        const uint32_t i0 = ins0(p, op.a);
        if ((i0 & cm) != cm) continue;
        const uint32_t i1 = i0 | (1u << op.a);
        const double a0r = P[i0].x, a0i = P[i0].y, a1r = P[i1].x, a1i = P[i1].y;
        const double l0r = L[i0].x, l0i = L[i0].y, l1r = L[i1].x, l1i = L[i1].y;
        // Im(conj(l) * g) = l.r g.i - l.i g.r
        switch (op.gen) {
        case GEN_X: acc += (l0r * a1i - l0i * a1r) + (l1r * a0i - l1i * a0r); break;
        case GEN_Y: acc += (l0r * (-a1r) - l0i * a1i) + (l1r * a0r - l1i * (-a0i)); break;
        case GEN_Z: acc += (l0r * a0i - l0i * a0r) - (l1r * a1i - l1i * a1r); break;
        default: acc += (l1r * a1i - l1i * a1r); break;
        }
    }
    return acc;
}

// v plus the value DPP control CTRL routes to each lane (rows outside ROWS add
// zero); a double moves as its two 32-bit halves.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_plus(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
    return v + __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront in a fixed order, returned to every
// lane (every lane must call it).  Within each row of 16 lanes: pairs
// (quad_perm 1,0,3,2), quads (2,3,0,1), half rows (row_half_mirror), rows
// (row_mirror); then row 0's sum into row 1 and row 2's into row 3
// (row_bcast:15), and lane 31's into rows 2 and 3 (row_bcast:31): lane 63
// holds the total.  Cross-lane moves through DPP take a few cycles each, where
// a shuffle through the LDS crossbar waits on a memory-like round trip.
__device__ __forceinline__ double wave_sum(double v)
{
    v = dpp_plus<0xB1, 0xf>(v);
    v = dpp_plus<0x4E, 0xf>(v);
    v = dpp_plus<0x141, 0xf>(v);
    v = dpp_plus<0x140, 0xf>(v);
    v = dpp_plus<0x142, 0xa>(v);
    v = dpp_plus<0x143, 0xc>(v);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Sum over the block of one value per thread, order fixed; result on thread 0.
__device__ double block_sum_fixed(double v, double* red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------------------
// Register-tiled passes.  The tile's 2^tq amplitudes are spread over
// 2^(tq - RB) threads, 2^RB per thread (the layout says which tile-local bits
// are lane bits and which are register bits).  An op whose targets are
// register bits runs entirely in registers: no LDS traffic and no barrier.
// Diagonal and subset-phase ops need no particular layout.  Between groups of
// ops the host inserts a layout change, the only step that goes through LDS
// (every thread writes its amplitudes, barrier, reads its new ones).
// ---------------------------------------------------------------------------


// Lane bits of the thread and register offsets of a layout.  The layout
// table holds the bit values, so nothing here waits on a dependent load.
// The table words are read whole and unconditionally (uniform scalar loads);
// each lane then keeps the values of its own set bits by a select.  (A load
// under the lane's bit test becomes a per-lane vector load, and the chain of
// them, one wait each, stalled every layout change.)  A workgroup has at most
// kMaxPassThreads threads, so only the lowest kPassLaneBits lane bits occur.
constexpr int kPassLaneBits = 9;
static_assert((1 << kPassLaneBits) == kMaxPassThreads, "lane bits cover the largest pass workgroup");

template <int RB>
__device__ __forceinline__ void frame_of(cptr<FLayout> L, uint32_t tid, uint32_t& tl, uint32_t* off)
{
    const cptr<uint32_t> w = (cptr<uint32_t>)L->lane_l;  // two 16-bit entries per word
    uint32_t t = 0;
#pragma unroll
    for (int i = 0; i < kPassLaneBits; ++i) {
        const uint32_t b = (w[i >> 1] >> (16 * (i & 1))) & 0xffffu;
        t |= ((tid >> i) & 1u) ? b : 0u;
    }
    tl = t;
    off[0] = 0;
#pragma unroll
    for (int j = 1; j < (1 << RB); ++j) off[j] = off[j & (j - 1)] | L->reg_l[__builtin_ctz(j)];
    // The offsets are uniform.  The exchanges that use them sit under the
    // active-thread test, and a table load moved into that branch becomes a
    // per-lane vector load with a wait; pinning the offsets to scalar
    // registers here keeps them scalar loads ahead of the branch.
#pragma unroll
    for (int j = 1; j < (1 << RB); ++j) asm volatile("" ::"s"(off[j]));
}

// Global element offsets of this thread's registers in a layout.
template <int RB>
__device__ __forceinline__ void global_frame(cptr<FLayout> L, uint32_t tid, uint64_t tile_base, uint64_t* g)
{
    uint64_t t = tile_base;
#pragma unroll
    for (int i = 0; i < kPassLaneBits; ++i) {
        const uint64_t b = L->lane_g[i];
        t |= ((tid >> i) & 1u) ? b : 0ull;
    }
    g[0] = t;
#pragma unroll
    for (int j = 1; j < (1 << RB); ++j) g[j] = g[j & (j - 1)] | L->reg_g[__builtin_ctz(j)];
}

template <typename V, int RB>
__device__ __forceinline__ void lds_put(V* __restrict__ lds, const V* v, uint32_t tl, const uint32_t* off)
{
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) lds[swz(tl | off[j])] = v[j];
}

template <typename V, int RB>
__device__ __forceinline__ void lds_get(const V* __restrict__ lds, V* v, uint32_t tl, const uint32_t* off)
{
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) v[j] = lds[swz(tl | off[j])];
}

#define SV_K_SWITCH(k, CALL)                                                                                       \
    switch (k) {                                                                                                   \
    case 0: CALL(0); break;                                                                                        \
    case 1: CALL(1); break;                                                                                        \
    case 2: CALL(2); break;                                                                                        \
    default:                                                                                                       \
        if constexpr (RB > 3) { CALL(3); }                                                                         \
        break;                                                                                                     \
    }


// In the register routines below, an op's control mask comes in two parts
// prepared by the host for the op's layout: `cml`, the controls on lane bits
// (tile-local bits), selects per thread between the op's coefficients and the
// identity (SEL); `cmk`, the controls on register bits as register indices,
// gives each register j a test (j & cmk) == cmk that is the same for every
// thread (CHK).  Neither needs the layout's register offsets, which keeps the
// scalar registers free across the op loop.

// Complex 2x2 on register bit K.
// Register-bit control test of register j (a uniform value).  The empty
// volatile asm on the passing side keeps it a scalar branch: without it the
// compiler evaluates the gate for every register and selects per lane, which
// costs more vector instructions than the gate on the passing registers.
__device__ __forceinline__ bool skip_reg(int j, uint32_t cmk)
{
    if (((uint32_t)j & cmk) != cmk) return true;
    asm volatile("");
    return false;
}

template <typename T, int RB, int K, bool CHK>
__device__ __forceinline__ void rpair_k(typename Vec2<T>::type* v, const T* u, uint32_t cmk)
{
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) {
        if (j & (1 << K)) continue;
        if (CHK && skip_reg(j, cmk)) continue;
        const int j1 = j | (1 << K);
        const auto a = v[j], b = v[j1];
        v[j] = cmul_add2<typename Vec2<T>::type, T>(u[0], u[1], a, u[2], u[3], b);
        v[j1] = cmul_add2<typename Vec2<T>::type, T>(u[4], u[5], a, u[6], u[7], b);
    }
}

// Complex 2x2 on register bit K chosen per register pair by register bit
// KS (the selector of FK_PAIRC): u0 where bit KS is 0, u1 where it is 1.
template <typename T, int RB, int K, int KS>
__device__ __forceinline__ void rpairc_k(typename Vec2<T>::type* v, const T* u0, const T* u1)
{
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) {
        if (j & (1 << K)) continue;
        const int j1 = j | (1 << K);
        const T* u = (j & (1 << KS)) ? u1 : u0;
        const auto a = v[j], b = v[j1];
        v[j] = cmul_add2<typename Vec2<T>::type, T>(u[0], u[1], a, u[2], u[3], b);
        v[j1] = cmul_add2<typename Vec2<T>::type, T>(u[4], u[5], a, u[6], u[7], b);
    }
}

// Real 2x2 [[r0, r1], [r2, r3]] on register bit K.
template <typename T, int RB, int K, bool CHK>
__device__ __forceinline__ void rpairr_k(typename Vec2<T>::type* v, const T* r, uint32_t cmk)
{
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) {
        if (j & (1 << K)) continue;
        if (CHK && skip_reg(j, cmk)) continue;
        const int j1 = j | (1 << K);
        const auto a = v[j], b = v[j1];
        v[j].x = r[0] * a.x + r[1] * b.x;
        v[j].y = r[0] * a.y + r[1] * b.y;
        v[j1].x = r[2] * a.x + r[3] * b.x;
        v[j1].y = r[2] * a.y + r[3] * b.y;
    }
}

// Exchange of the pair on register bit K (X); with SEL only where `ok` holds.
template <typename T, int RB, int K, bool CHK, bool SEL>
__device__ __forceinline__ void rpairx_k(typename Vec2<T>::type* v, bool ok, uint32_t cmk)
{
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) {
        if (j & (1 << K)) continue;
        if (CHK && skip_reg(j, cmk)) continue;
        const int j1 = j | (1 << K);
        const auto a = v[j], b = v[j1];
        if constexpr (SEL) {
            v[j].x = ok ? b.x : a.x;
            v[j].y = ok ? b.y : a.y;
            v[j1].x = ok ? a.x : b.x;
            v[j1].y = ok ? a.y : b.y;
        } else {
            v[j] = b;
            v[j1] = a;
        }
    }
}

// Element-wise diagonal d[bit of register K].
template <typename T, int RB, int K, bool CHK>
__device__ __forceinline__ void rdiag_k(typename Vec2<T>::type* v, const T* d, uint32_t cmk)
{
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) {
        if (CHK && skip_reg(j, cmk)) continue;
        const T zr = (j >> K) & 1 ? d[2] : d[0], zi = (j >> K) & 1 ? d[3] : d[1];
        const auto x = v[j];
        v[j].x = zr * x.x - zi * x.y;
        v[j].y = zr * x.y + zi * x.x;
    }
}

// One phase z on every register (passing the register-bit controls).
template <typename T, int RB, bool CHK>
__device__ __forceinline__ void rphase(typename Vec2<T>::type* v, T zr, T zi, uint32_t cmk)
{
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) {
        if (CHK && skip_reg(j, cmk)) continue;
        const auto x = v[j];
        v[j].x = zr * x.x - zi * x.y;
        v[j].y = zr * x.y + zi * x.x;
    }
}

template <typename T, int RB, int KA, int KB, bool CHK, bool SEL>
__device__ __forceinline__ void rswap_k(typename Vec2<T>::type* v, bool ok, uint32_t cmk)
{
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) {
        if (!(j & (1 << KA)) || (j & (1 << KB))) continue;  // j: bit a = 1, bit b = 0
        if (CHK && skip_reg(j, cmk)) continue;
        const int j1 = j ^ (1 << KA) ^ (1 << KB);
        const auto a = v[j], b = v[j1];
        if constexpr (SEL) {
            v[j].x = ok ? b.x : a.x;
            v[j].y = ok ? b.y : a.y;
            v[j1].x = ok ? a.x : b.x;
            v[j1].y = ok ? a.y : b.y;
        } else {
            v[j] = b;
            v[j1] = a;
        }
    }
}

#define SV_RB_PAIRS(X) X(0, 1) X(0, 2) X(1, 0) X(1, 2) X(2, 0) X(2, 1)
#define SV_RB4_PAIRS(X) X(0, 3) X(1, 3) X(2, 3) X(3, 0) X(3, 1) X(3, 2)

template <typename T, int RB, bool CHK, bool SEL>
__device__ __forceinline__ void rswap(int ka, int kb, typename Vec2<T>::type* v, bool ok, uint32_t cmk)
{
    switch (ka * 4 + kb) {
#define SV_CASE(A, B)                                                                                              \
    case A * 4 + B: rswap_k<T, RB, A, B, CHK, SEL>(v, ok, cmk); break;
        SV_RB_PAIRS(SV_CASE)
#undef SV_CASE
    default:
        if constexpr (RB > 3) {
            switch (ka * 4 + kb) {
#define SV_CASE(A, B)                                                                                              \
    case A * 4 + B: rswap_k<T, RB, A, B, CHK, SEL>(v, ok, cmk); break;
                SV_RB4_PAIRS(SV_CASE)
#undef SV_CASE
            default: break;
            }
        }
        break;
    }
}

// TWO: SWAP runs in registers (forward passes); reverse passes leave it to an
// LDS sweep (lds_op).  4x4 ops always take the LDS sweep: their 32 complex
// coefficients would claim 64 scalar registers in this switch and make the
// compiler spill scalar registers across the whole op loop.
// DUAL: the op acts on w as well (a reverse pass un-applies it on phi and
// lambda): one dispatch, the coefficients read once.
template <typename T, int RB, bool CHK, bool SEL, bool TWO, bool DUAL = false>
__device__ __forceinline__ void reg_apply_c(typename Vec2<T>::type* v, typename Vec2<T>::type* w, const FOp& op,
                                            cptr<T> cf, bool dagger, uint32_t tl, uint32_t cmk, bool ok, T pzr, T pzi)
{
    switch (op.kind) {
    case FK_PAIRX: {
#define SV_CALL(K) { rpairx_k<T, RB, K, CHK, SEL>(v, ok, cmk); if constexpr (DUAL) rpairx_k<T, RB, K, CHK, SEL>(w, ok, cmk); }
        SV_K_SWITCH(op.ka, SV_CALL)
#undef SV_CALL
        break;
    }
    case FK_PAIRR: {  // real: the transpose is the inverse's matrix
        T r[4] = {(T)cf[0], (T)cf[2], (T)cf[4], (T)cf[6]};
        if (dagger) {
            const T t = r[1];
            r[1] = r[2];
            r[2] = t;
        }
        if constexpr (SEL) {
            r[0] = ok ? r[0] : T(1);
            r[1] = ok ? r[1] : T(0);
            r[2] = ok ? r[2] : T(0);
            r[3] = ok ? r[3] : T(1);
        }
#define SV_CALL(K) { rpairr_k<T, RB, K, CHK>(v, r, cmk); if constexpr (DUAL) rpairr_k<T, RB, K, CHK>(w, r, cmk); }
        SV_K_SWITCH(op.ka, SV_CALL)
#undef SV_CALL
        break;
    }
    case FK_PAIR: {
        T u[8];
        load2x2<T>(cf, dagger, u);
        if constexpr (SEL) {
#pragma unroll
            for (int k = 0; k < 8; ++k) u[k] = ok ? u[k] : ((k == 0 || k == 6) ? T(1) : T(0));
        }
#define SV_CALL(K) { rpair_k<T, RB, K, CHK>(v, u, cmk); if constexpr (DUAL) rpair_k<T, RB, K, CHK>(w, u, cmk); }
        SV_K_SWITCH(op.ka, SV_CALL)
#undef SV_CALL
        break;
    }
    case FK_DIAG: {
        T d[4] = {(T)cf[0], (T)(dagger ? -cf[1] : cf[1]), (T)cf[2], (T)(dagger ? -cf[3] : cf[3])};
        if constexpr (SEL) {
            d[0] = ok ? d[0] : T(1);
            d[1] = ok ? d[1] : T(0);
            d[2] = ok ? d[2] : T(1);
            d[3] = ok ? d[3] : T(0);
        }
        if (op.ka >= 0) {
#define SV_CALL(K) { rdiag_k<T, RB, K, CHK>(v, d, cmk); if constexpr (DUAL) rdiag_k<T, RB, K, CHK>(w, d, cmk); }
            SV_K_SWITCH(op.ka, SV_CALL)
#undef SV_CALL
        } else {  // target on a lane bit: one phase for all of this thread's registers
            const bool b = (tl >> op.a) & 1u;
            rphase<T, RB, CHK>(v, b ? d[2] : d[0], b ? d[3] : d[1], cmk);
            if constexpr (DUAL) rphase<T, RB, CHK>(w, b ? d[2] : d[0], b ? d[3] : d[1], cmk);
        }
        break;
    }
    case FK_PHASE: {  // the caller supplies the phase (a chain's product, or conjugated in reverse)
        T zr = pzr, zi = pzi;
        if constexpr (SEL) {
            zr = ok ? zr : T(1);
            zi = ok ? zi : T(0);
        }
        rphase<T, RB, CHK>(v, zr, zi, cmk);
        if constexpr (DUAL) rphase<T, RB, CHK>(w, zr, zi, cmk);
        break;
    }
    case FK_SWAP:
        if constexpr (TWO) {
            rswap<T, RB, CHK, SEL>(op.ka, op.kb, v, ok, cmk);
            if constexpr (DUAL) rswap<T, RB, CHK, SEL>(op.ka, op.kb, w, ok, cmk);
        }
        break;
    default: break;
    }
}

// FK_PAIRC in a register layout: with the selector on a lane bit each thread
// takes one of the two matrices (a select of its coefficients); with it on a
// register bit the matrix is fixed per register pair.
template <typename T, int RB>
__device__ __forceinline__ void reg_pairc(typename Vec2<T>::type* v, const FOp& op, cptr<T> cf, uint32_t tl)
{
    T u0[8], u1[8];
    load2x2<T>(cf, false, u0);
    load2x2<T>(cf + 8, false, u1);
    if (op.kb < 0) {
        const bool s = (tl >> op.b) & 1u;
        T u[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) u[k] = s ? u1[k] : u0[k];
#define SV_CALL(K) rpair_k<T, RB, K, false>(v, u, 0u)
        SV_K_SWITCH(op.ka, SV_CALL)
#undef SV_CALL
        return;
    }
    switch (op.ka * 4 + op.kb) {
#define SV_CASE(A, B)                                                                                              \
    case A * 4 + B: rpairc_k<T, RB, A, B>(v, u0, u1); break;
        SV_RB_PAIRS(SV_CASE)
#undef SV_CASE
    default:
        if constexpr (RB > 3) {
            switch (op.ka * 4 + op.kb) {
#define SV_CASE(A, B)                                                                                              \
    case A * 4 + B: rpairc_k<T, RB, A, B>(v, u0, u1); break;
                SV_RB4_PAIRS(SV_CASE)
#undef SV_CASE
            default: break;
            }
        }
        break;
    }
}

// Every thread runs every op (no divergent branch around the registers, which
// would make the compiler copy all of them at each join): a lane-bit control
// turns the op into the identity for threads where it is 0.
// (pzr, pzi): the phase of an FK_PHASE op, supplied by the caller.
template <typename T, int RB, bool TWO = true, bool DUAL = false>
__device__ __forceinline__ void reg_apply(typename Vec2<T>::type* v, const FOp& op, cptr<T> cf, bool dagger,
                                          uint32_t tl, T pzr, T pzi, typename Vec2<T>::type* w = nullptr)
{
    const uint32_t cmk = op.cmk, cml = op.cml;
    const bool ok = (tl & cml) == cml;
    if (cml) {
        if (cmk) reg_apply_c<T, RB, true, true, TWO, DUAL>(v, w, op, cf, dagger, tl, cmk, ok, pzr, pzi);
        else reg_apply_c<T, RB, false, true, TWO, DUAL>(v, w, op, cf, dagger, tl, 0u, ok, pzr, pzi);
    } else {
        if (cmk) reg_apply_c<T, RB, true, false, TWO, DUAL>(v, w, op, cf, dagger, tl, cmk, true, pzr, pzi);
        else reg_apply_c<T, RB, false, false, TWO, DUAL>(v, w, op, cf, dagger, tl, 0u, true, pzr, pzi);
    }
}

// Per-thread Im <lambda|G|phi> over this thread's registers (generator of a
// parameterised one-target op, restricted to its controls; the target's own
// bit is excluded from the mask).
template <typename T, int RB, int K, bool CHK>
__device__ __forceinline__ double rgen_pair_k(const typename Vec2<T>::type* P, const typename Vec2<T>::type* L,
                                              bool gy, uint32_t cmk)
{
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) {
        if (j & (1 << K)) continue;
        if (CHK && skip_reg(j, cmk)) continue;
        const int j1 = j | (1 << K);
        const double a0r = P[j].x, a0i = P[j].y, a1r = P[j1].x, a1i = P[j1].y;
        const double l0r = L[j].x, l0i = L[j].y, l1r = L[j1].x, l1i = L[j1].y;
        if (!gy) acc += (l0r * a1i - l0i * a1r) + (l1r * a0i - l1i * a0r);
        else acc += (l0r * (-a1r) - l0i * a1i) + (l1r * a0r - l1i * (-a0i));
    }
    return acc;
}

// Z-type generators: sign (GEN_Z) or indicator (GEN_P1) of the target bit;
// sel(j) gives that bit for register j.
template <typename T, int RB, bool CHK, typename Sel>
__device__ __forceinline__ double rgen_elem(const typename Vec2<T>::type* P, const typename Vec2<T>::type* L, bool gz,
                                            uint32_t cmk, Sel sel)
{
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) {
        if (CHK && skip_reg(j, cmk)) continue;
        const bool b = sel(j);
        const double t = (double)L[j].x * (double)P[j].y - (double)L[j].y * (double)P[j].x;
        if (gz) acc += b ? -t : t;
        else if (b) acc += t;
    }
    return acc;
}

// Per-thread Im <lambda|M|phi> over this thread's register pairs on bit K
// for a 2x2 complex M (row-major, interleaved; uniform).
template <typename T, int RB, int K, bool CHK>
__device__ __forceinline__ double rgen_m_k(const typename Vec2<T>::type* P, const typename Vec2<T>::type* L,
                                           cptr<T> m, uint32_t cmk)
{
    const double m0r = m[0], m0i = m[1], m1r = m[2], m1i = m[3], m2r = m[4], m2i = m[5], m3r = m[6], m3i = m[7];
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) {
        if (j & (1 << K)) continue;
        if (CHK && skip_reg(j, cmk)) continue;
        const int j1 = j | (1 << K);
        const double a0r = P[j].x, a0i = P[j].y, a1r = P[j1].x, a1i = P[j1].y;
        const double l0r = L[j].x, l0i = L[j].y, l1r = L[j1].x, l1i = L[j1].y;
        // t = M phi on the pair
        const double t0r = m0r * a0r - m0i * a0i + m1r * a1r - m1i * a1i;
        const double t0i = m0r * a0i + m0i * a0r + m1r * a1i + m1i * a1r;
        const double t1r = m2r * a0r - m2i * a0i + m3r * a1r - m3i * a1i;
        const double t1i = m2r * a0i + m2i * a0r + m3r * a1i + m3i * a1r;
        acc += l0r * t0i - l0i * t0r + l1r * t1i - l1i * t1r;
    }
    return acc;
}

// Im <lambda|M|phi> of a reverse pair's first gate (FK_RFUSE): M from the
// coefficient table, the op's controls as for its generator.
template <typename T, int RB>
__device__ __forceinline__ double reg_gen_inner_m(const typename Vec2<T>::type* P, const typename Vec2<T>::type* L,
                                                  const FOp& op, cptr<T> m, uint32_t tl)
{
    const uint32_t cmk = op.cmk & ~(1u << op.ka), cml = op.cml;
    if ((tl & cml) != cml) return 0.0;
    double r = 0.0;
    if (cmk) {
#define SV_CALL(K) r = rgen_m_k<T, RB, K, true>(P, L, m, cmk)
        SV_K_SWITCH(op.ka, SV_CALL)
#undef SV_CALL
    } else {
#define SV_CALL(K) r = rgen_m_k<T, RB, K, false>(P, L, m, 0u)
        SV_K_SWITCH(op.ka, SV_CALL)
#undef SV_CALL
    }
    return r;
}

template <typename T, int RB>
__device__ __forceinline__ double reg_gen_inner(const typename Vec2<T>::type* P, const typename Vec2<T>::type* L,
                                                const FOp& op, uint32_t tl)
{
    // the generator's controls exclude the target (a subset-phase op lists it)
    const uint32_t tk = op.ka >= 0 ? 1u << op.ka : 0u, tlb = op.ka >= 0 ? 0u : 1u << op.a;
    const uint32_t cmk = op.cmk & ~tk, cml = op.cml & ~tlb;
    if ((tl & cml) != cml) return 0.0;
    if (op.gen == GEN_X || op.gen == GEN_Y) {
        const bool gy = op.gen == GEN_Y;
        double r = 0.0;
        if (cmk) {
#define SV_CALL(K) r = rgen_pair_k<T, RB, K, true>(P, L, gy, cmk)
            SV_K_SWITCH(op.ka, SV_CALL)
#undef SV_CALL
        } else {
#define SV_CALL(K) r = rgen_pair_k<T, RB, K, false>(P, L, gy, 0u)
            SV_K_SWITCH(op.ka, SV_CALL)
#undef SV_CALL
        }
        return r;
    }
    const bool gz = op.gen == GEN_Z;
    if (op.ka >= 0) {
        const int ka = op.ka;
        return rgen_elem<T, RB, true>(P, L, gz, cmk, [&](int j) { return ((j >> ka) & 1) != 0; });
    }
    const bool b = (tl >> op.a) & 1u;
    return rgen_elem<T, RB, true>(P, L, gz, cmk, [&](int) { return b; });
}

// Sum per slot of the wave partials, in fixed wave order, to the per-tile table.
__device__ __forceinline__ void flush_slots(const PassTables& tb, const FCirc& cc, int op_begin, int op_end,
                                            int tile, const double* wpart)
{
    if (threadIdx.x != 0) return;
    const int nwaves = blockDim.x >> 6;
    int k = 0;
    for (int o = op_end - 1; o >= op_begin; --o) {
        const FOp op = ld_const(as_const(tb.ops) + o);
        if (op.kind == FK_LAYOUT) continue;
        // slots in the order the kernel filled them: the op's, then (FK_RFUSE) its first gate's
        const int sl[2] = {op.slot, op.kind == FK_RFUSE ? op.b : -1};
        for (int x = 0; x < 2; ++x) {
            if (sl[x] < 0) continue;
            double s = 0.0;
            for (int w = 0; w < nwaves; ++w) s += wpart[k * nwaves + w];
            tb.g_part[cc.g_part_begin + (int64_t)sl[x] * cc.n_tiles + tile] = s;
            ++k;
        }
    }
}

// The coefficient table in the run's precision (complex64 runs read the
// float copy, so no per-use conversion lands in vector registers).
template <typename T>
__device__ __forceinline__ cptr<T> coef_table(const PassTables& tb)
{
    if constexpr (sizeof(T) == 8) return (cptr<T>)as_const(tb.coef);
    else return (cptr<T>)as_const(tb.coef_f);
}

// Tile base: the tile index deposited into the global bits outside the tile.
__device__ __forceinline__ uint64_t tile_base_of(uint64_t free_mask, uint64_t tile)
{
    uint64_t b = 0;
    for (uint64_t m = free_mask; m && tile; m &= m - 1, tile >>= 1)
        if (tile & 1) b |= m & (~m + 1);
    return b;
}

// Whether a subset phase acts on tile `tile`: the tile must hold every bit of
// the op's mask that lies outside the tile (packed in b; a uniform test).
__device__ __forceinline__ bool phase_on(const FOp& op, int tile)
{
    return ((uint32_t)tile & (uint32_t)op.b) == (uint32_t)op.b;
}

// Whether an op acts on tile `tile` (uniform): one-target ops and subset
// phases carry their bits outside the tile packed in b, and act only on the
// tiles whose index holds them all; other kinds use b otherwise.
__device__ __forceinline__ bool op_on(const FOp& op, int tile)
{
    const bool gated = op.kind == FK_PHASE || op.kind == FK_PAIR || op.kind == FK_PAIRR || op.kind == FK_PAIRX ||
                       op.kind == FK_DIAG;
    return !gated || phase_on(op, tile);
}

// Entry of a tile-selected op (FK_PAIRT) for tile `tile`: the tile index's
// bits under the packed mask, gathered in order (uniform).
__device__ __forceinline__ uint32_t tile_select(uint32_t tile, uint32_t mask)
{
    uint32_t e = 0;
    for (int k = 0; mask; mask &= mask - 1u, ++k) e |= ((tile >> __builtin_ctz(mask)) & 1u) << k;
    return e;
}

// A tile-selected op becomes the plain 2x2 of its entry for this tile.
__device__ __forceinline__ void tile_select_op(FOp& op, int tile)
{
    if (op.kind != FK_PAIRT) return;
    op.coef += 8 * (int32_t)tile_select((uint32_t)tile, (uint32_t)op.b);
    op.kind = FK_PAIR;
    op.b = 0;
}

// The next op's descriptor is fetched one op ahead, so its load overlaps the
// current op's arithmetic.
struct OpPre {
    FOp op;
};

__device__ __forceinline__ void op_fetch(const PassTables& tb, int o, OpPre& p) { p.op = ld_const(as_const(tb.ops) + o); }

// A two-target op by a sweep over the LDS tile (4x4 ops in both directions,
// SWAP in reverse passes): the tile goes to LDS, every thread sweeps the op
// over it, and the registers are read back.  These ops are rare in the
// workloads; keeping them out of the register switch keeps its code small.
template <typename T, int RB, typename P>
__device__ __forceinline__ void lds_op(typename Vec2<T>::type* v, typename Vec2<T>::type* lds, const FOp& op, P coef,
                                       bool dagger, int tq, bool active, cptr<FLayout> L)
{
    using V = typename Vec2<T>::type;
    uint32_t tl, off[1 << RB];
    frame_of<RB>(L, threadIdx.x, tl, off);
    if (active) lds_put<V, RB>(lds, v, tl, off);
    __syncthreads();
    lds_apply<T, true, P>(lds, op, coef, dagger, tq);
    __syncthreads();
    if (active) lds_get<V, RB>(lds, v, tl, off);
    __syncthreads();
}

// GATED: the pass holds one-target ops with controls outside the tile, which
// act only on the tiles that hold those bits; passes without them take a
// kernel that does not test for it.
template <typename T, int RB, bool GATED>
__device__ __forceinline__ void item_reg_fwd(const PassTables& tb, const FCirc& cc, int pidx, int tile,
                                             typename Vec2<T>::type* lds)
{
    using V = typename Vec2<T>::type;
    constexpr int R = 1 << RB;
    const int tq = cc.tq;
    const cptr<FPass> pp = as_const(tb.passes) + cc.pass_begin + pidx;
    const cptr<FLayout> lays = as_const(tb.lays);
    const int op_begin = pp->op_begin, op_end = pp->op_end;
    const bool gated = GATED && pp->gated != 0;
    const bool active = threadIdx.x < (1u << (tq - RB));
    const uint64_t tile_base = tile_base_of(pp->free_mask, (uint64_t)tile);
    V* const psi = (V*)cc.psi;
    uint32_t tl;
    V v[R];
    int cur = pp->lay_begin;
    {
        uint32_t off[R];
        frame_of<RB>(lays + cur, threadIdx.x, tl, off);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) v[j].x = v[j].y = T(0);  // threads past the tile keep zeros
    if (active) {
        uint64_t g[R];
        global_frame<RB>(lays + cur, threadIdx.x, tile_base, g);
        if (pidx == 0) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                v[j].x = g[j] == 0 ? T(1) : T(0);
                v[j].y = T(0);
            }
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) v[j] = ldg<true>(psi + g[j]);
        }
    }
    const cptr<T> coef = coef_table<T>(tb);
    OpPre nx;
    if (op_begin < op_end) op_fetch(tb, op_begin, nx);
    for (int o = op_begin; o < op_end; ++o) {
        OpPre p = nx;
        if (o + 1 < op_end) op_fetch(tb, o + 1, nx);
        if constexpr (GATED) tile_select_op(p.op, tile);
        const FOp& op = p.op;
        T pzr = T(1), pzi = T(0);
        if (op.kind == FK_PHASE) {
            // A chained group of subset phases on one local mask (kb 1): the
            // product of the phases of the ops that act on this tile (those whose
            // bits outside the tile the tile holds), applied once by the group's
            // last op.  A run on target a (kb 2, the last 3): members whose
            // other in-tile bit is a lane bit count only on the lanes holding
            // it, so the product is per lane; it is applied once to the
            // amplitudes holding a.
            const cptr<double> cd = as_const(tb.coef);
            double chr = 1.0, chi = 0.0;
            bool any = false;
            int e = o;
            for (;; ++e) {
                const FOp q = e == o ? op : ld_const(as_const(tb.ops) + e);
                if (phase_on(q, tile)) {
                    const uint32_t lc = q.kb >= 2 ? q.cml & ~(1u << q.a) : 0u;
                    const bool in = (tl & lc) == lc;
                    const double zr = cd[q.coef], zi = cd[q.coef + 1];
                    const double r = chr * zr - chi * zi, im = chr * zi + chi * zr;
                    chr = in ? r : chr;
                    chi = in ? im : chi;
                    any = true;
                }
                if (q.kb != 1 && q.kb != 2) break;
            }
            if (e != o) {  // skip the group's other ops; refetch the next descriptor
                o = e;
                if (o + 1 < op_end) op_fetch(tb, o + 1, nx);
            }
            if (!any) continue;
            if (p.op.kb >= 2) {  // a run acts on the amplitudes holding its target only
                p.op.cmk = p.op.ka >= 0 ? (uint8_t)(1u << p.op.ka) : (uint8_t)0;
                p.op.cml = p.op.ka >= 0 ? 0u : 1u << p.op.a;
            }
            pzr = (T)chr;
            pzi = (T)chi;
        }
        if (op.kind == FK_LAYOUT) {
            if (op.a == cur) continue;
            uint32_t off[R];
            frame_of<RB>(lays + cur, threadIdx.x, tl, off);
            if (active) lds_put<V, RB>(lds, v, tl, off);
            __syncthreads();
            cur = op.a;
            frame_of<RB>(lays + cur, threadIdx.x, tl, off);
            if (active) lds_get<V, RB>(lds, v, tl, off);
            __syncthreads();
            continue;
        }
        if (op.kind == FK_QUAD) lds_op<T, RB>(v, lds, op, coef, false, tq, active, lays + cur);
        else if (op.kind == FK_PAIRC) reg_pairc<T, RB>(v, op, coef + op.coef, tl);
        else if (gated && op.kind != FK_PHASE && !op_on(op, tile)) continue;  // controls outside the tile not all 1 here
        else reg_apply<T, RB>(v, op, coef + op.coef, false, tl, pzr, pzi);
    }
    if (active) {
        uint64_t g[R];
        global_frame<RB>(lays + cur, threadIdx.x, tile_base, g);
#pragma unroll
        for (int j = 0; j < R; ++j) stg<true>(psi + g[j], v[j]);
    }
}

// Reverse pass: phi (= psi) and lambda, the reverse op list walked backwards.
template <typename T, int RB>
__device__ __forceinline__ void item_reg_rev(const PassTables& tb, const FCirc& cc, int pidx, int tile,
                                             typename Vec2<T>::type* lds, double* wpart)
{
    using V = typename Vec2<T>::type;
    constexpr int R = 1 << RB;
    const int tq = cc.tq;
    const cptr<FPass> pp = as_const(tb.passes) + cc.pass_begin + pidx;
    const cptr<FLayout> lays = as_const(tb.lays);
    const cptr<T> coef = coef_table<T>(tb);
    const int rop_begin = pp->rop_begin, rop_end = pp->rop_end;
    const bool active = threadIdx.x < (1u << (tq - RB));
    const uint64_t tile_base = tile_base_of(pp->free_mask, (uint64_t)tile);
    V* const psi = (V*)cc.psi;
    V* const lam = (V*)cc.lam;
    uint32_t tl;
    V v[R], w[R];
    int cur = pp->rlay_end;
    {
        uint32_t off[R];
        frame_of<RB>(lays + cur, threadIdx.x, tl, off);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) v[j].x = v[j].y = w[j].x = w[j].y = T(0);  // threads past the tile keep zeros
    if (active) {
        uint64_t g[R];
        global_frame<RB>(lays + cur, threadIdx.x, tile_base, g);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            v[j] = ldg<true>(psi + g[j]);
            w[j] = ldg<true>(lam + g[j]);
        }
    }
    int nslot = 0;
    OpPre nx;
    if (rop_begin < rop_end) op_fetch(tb, rop_end - 1, nx);
    for (int o = rop_end - 1; o >= rop_begin; --o) {
        OpPre p = nx;
        if (o - 1 >= rop_begin) op_fetch(tb, o - 1, nx);
        const FOp& op = p.op;
        if (op.kind == FK_LAYOUT) {
            if (op.b == cur) continue;
            uint32_t tl2, off2[R], off[R];
            frame_of<RB>(lays + cur, threadIdx.x, tl, off);
            frame_of<RB>(lays + op.b, threadIdx.x, tl2, off2);
            if (active) lds_put<V, RB>(lds, v, tl, off);
            __syncthreads();
            if (active) lds_get<V, RB>(lds, v, tl2, off2);
            __syncthreads();
            if (active) lds_put<V, RB>(lds, w, tl, off);
            __syncthreads();
            if (active) lds_get<V, RB>(lds, w, tl2, off2);
            __syncthreads();
            cur = op.b;
            tl = tl2;
            continue;
        }
        // an op with bits outside the tile acts here only if the tile holds them all
        const bool on = op_on(op, tile);
        if (op.slot >= 0) {
            const double c = wave_sum(active && on ? reg_gen_inner<T, RB>(v, w, op, tl) : 0.0);
            if ((threadIdx.x & 63) == 0) wpart[nslot * (blockDim.x >> 6) + (threadIdx.x >> 6)] = c;
            ++nslot;
        }
        if (op.kind == FK_RFUSE) {
            // the pair's first gate: its partial with B G_A B^dagger; then one un-apply of B A
            if (op.b >= 0) {
                const double c = wave_sum(active ? reg_gen_inner_m<T, RB>(v, w, op, coef + op.coef + 8, tl) : 0.0);
                if ((threadIdx.x & 63) == 0) wpart[nslot * (blockDim.x >> 6) + (threadIdx.x >> 6)] = c;
                ++nslot;
            }
            p.op.kind = FK_PAIR;
        }
        if (!on) continue;
        if (op.kind == FK_SWAP || op.kind == FK_QUAD) {
            lds_op<T, RB>(v, lds, op, coef, true, tq, active, lays + cur);
            lds_op<T, RB>(w, lds, op, coef, true, tq, active, lays + cur);
        } else {
            const T pzr = op.kind == FK_PHASE ? (T)coef[op.coef] : T(1);
            const T pzi = op.kind == FK_PHASE ? (T)-coef[op.coef + 1] : T(0);
            reg_apply<T, RB, false, true>(v, op, coef + op.coef, true, tl, pzr, pzi, w);
        }
    }
    __syncthreads();  // every wave's partials are in LDS
    flush_slots(tb, cc, rop_begin, rop_end, tile, wpart);
    if (active) {
        uint64_t g[R];
        global_frame<RB>(lays + cur, threadIdx.x, tile_base, g);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            stg<true>(psi + g[j], v[j]);
            stg<true>(lam + g[j], w[j]);
        }
    }
}

// Observable stage: lambda = O psi on contiguous chunk `tile` and its partial of <psi|O|psi>.
template <typename T>
__device__ __forceinline__ void item_observable(const PassTables& tb, const FCirc& cc, int tile, double* red)
{
    using V = typename Vec2<T>::type;
    V* const psi = (V*)cc.psi;
    V* const lam = (V*)cc.lam;
    const int tq = cc.tq;
    const uint32_t na = 1u << tq;
    const uint64_t base = (uint64_t)tile << tq;
    const uint64_t zzmask = cc.n > 1 ? ((1ull << (cc.n - 1)) - 1ull) : 0ull;
    double acc = 0.0;
    for (uint32_t l = threadIdx.x; l < na; l += blockDim.x) {
        const uint64_t x = base + l;
        const V a = ldg<true>(psi + x);
        const double o = cc.obs_kind == 1 ? (double)(cc.n - 2 * (int)__popcll(x))
                                          : (double)((cc.n - 1) - 2 * (int)__popcll((x ^ (x >> 1)) & zzmask));
        acc += o * ((double)a.x * (double)a.x + (double)a.y * (double)a.y);
        if (tb.with_grad) {
            V r;
            r.x = (T)(o * (double)a.x);
            r.y = (T)(o * (double)a.y);
            stg<true>(lam + x, r);
        }
    }
    const double s = block_sum_fixed(acc, red);
    if (threadIdx.x == 0) tb.e_part[cc.e_part_begin + tile] = s;
}

// A pass of a circuit whose tile is smaller than a workgroup's register tile:
// the tile stays in LDS and every op sweeps it.  GATED as in item_reg_fwd
// (forward passes; reverse passes always test).
template <typename T, bool GATED>
__device__ __forceinline__ void item_lds(const PassTables& tb, const FCirc& cc, bool fwd, int pidx, int tile,
                                         typename Vec2<T>::type* tileA, typename Vec2<T>::type* tileB,
                                         uint64_t* hi_map, double* wpart)
{
    using V = typename Vec2<T>::type;
    V* const psi = (V*)cc.psi;
    V* const lam = (V*)cc.lam;
    const int tq = cc.tq;
    const uint32_t na = 1u << tq;
    const FPass& ps = tb.passes[cc.pass_begin + pidx];
    // tile base: insert zeros at Q into the tile index; hi_map deposits local bits >= cb
    uint64_t base = (uint64_t)tile;
    for (int k = 0; k < tq; ++k) {
        const int p = ps.q[k];
        const uint64_t lo = base & ((1ull << p) - 1ull);
        base = ((base >> p) << (p + 1)) | lo;
    }
    const int cb = cc.cb;  // <= tq; 2^(tq - cb) <= hi_entries
    for (uint32_t h = threadIdx.x; h < (na >> cb); h += blockDim.x) {
        uint64_t g = 0;
        for (int k = cb; k < tq; ++k)
            if ((h >> (k - cb)) & 1u) g |= 1ull << ps.q[k];
        hi_map[h] = g | base;
    }
    __syncthreads();
    const uint32_t lomask = (1u << cb) - 1u;
    if (fwd) {
        if (pidx == 0) {
            for (uint32_t l = threadIdx.x; l < na; l += blockDim.x) {
                const uint64_t g = hi_map[l >> cb] | (l & lomask);
                V v;
                v.x = g == 0 ? T(1) : T(0);
                v.y = T(0);
                tileA[l] = v;
            }
        } else {
            for (uint32_t l = threadIdx.x; l < na; l += blockDim.x)
                tileA[l] = ldg<true>(psi + (hi_map[l >> cb] | (l & lomask)));
        }
        __syncthreads();
        for (int o = ps.op_begin; o < ps.op_end; ++o) {
            FOp op = tb.ops[o];
            if constexpr (GATED) tile_select_op(op, tile);
            // uniform: not on this tile
            if (GATED ? !op_on(op, tile) : op.kind == FK_PHASE && !phase_on(op, tile)) continue;
            if (op.kind == FK_PAIRC) lds_pairc<T>(tileA, op, tb.coef, tq);
            else lds_apply<T>(tileA, op, tb.coef, false, tq);
            __syncthreads();
        }
        for (uint32_t l = threadIdx.x; l < na; l += blockDim.x)
            stg<true>(psi + (hi_map[l >> cb] | (l & lomask)), tileA[l]);
        return;
    }
    for (uint32_t l = threadIdx.x; l < na; l += blockDim.x) {
        const uint64_t g = hi_map[l >> cb] | (l & lomask);
        tileA[l] = ldg<true>(psi + g);
        tileB[l] = ldg<true>(lam + g);
    }
    __syncthreads();
    int nslot = 0;
    for (int o = ps.rop_end - 1; o >= ps.rop_begin; --o) {
        const FOp op = tb.ops[o];
        const bool on = op_on(op, tile);  // uniform
        if (op.slot >= 0) {
            const double c = on ? wave_sum(lds_gen_inner<T>(tileA, tileB, op, tq)) : 0.0;
            if ((threadIdx.x & 63) == 0) wpart[nslot * (blockDim.x >> 6) + (threadIdx.x >> 6)] = c;
            ++nslot;
            __syncthreads();  // every read of the tiles precedes the un-apply below
        }
        if (!on) continue;
        lds_apply<T>(tileA, op, tb.coef, true, tq);
        lds_apply<T>(tileB, op, tb.coef, true, tq);
        __syncthreads();
    }
    flush_slots(tb, cc, ps.rop_begin, ps.rop_end, tile, wpart);
    for (uint32_t l = threadIdx.x; l < na; l += blockDim.x) {
        const uint64_t g = hi_map[l >> cb] | (l & lomask);
        stg<true>(psi + g, tileA[l]);
        stg<true>(lam + g, tileB[l]);
    }
}

// LDS of a run: [tiles][address map][per-slot wave partials (reverse only)]
struct EngineLds {
    void* tileA;
    void* tileB;
    uint64_t* hi_map;
    double* wpart;  // [kMaxPassSlots][waves of the workgroup]
};

template <typename T>
__device__ __forceinline__ EngineLds engine_lds(const PassTables& tb, double* smem)
{
    using V = typename Vec2<T>::type;
    EngineLds e;
    const size_t tile_elems = (size_t)1 << tb.tq_max;
    V* const a = (V*)smem;
    e.tileA = a;
    e.tileB = a + tile_elems;
    e.hi_map = (uint64_t*)(a + (tb.lds_small && tb.with_grad ? 2 * tile_elems : tile_elems));
    e.wpart = (double*)(e.hi_map + (tb.lds_small ? tb.hi_entries : 0));
    return e;
}

// Segment of a work item: the last segment whose first item is <= item.
__device__ __forceinline__ FSeg seg_of(const PassTables& tb, int64_t item)
{
    const cptr<FSeg> segs = as_const(tb.segs);
    int lo = 0, hi = tb.n_segs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].first <= item) lo = mid;
        else hi = mid - 1;
    }
    return ld_const(segs + lo);
}

// Target waves per SIMD, which sets the VGPR budget (512 / waves).  Forward
// complex64 passes and 8-amplitude complex128 forward passes fit 128 VGPRs;
// the complex128 kernels with 16 amplitudes (forward) or 2 x 8 (reverse)
// fit 168 with a few spilled registers; complex64 reverse passes with 2 x 16
// amplitudes need the 256 of two waves.
template <typename T, int RB, bool REV>
constexpr int pass_waves_per_eu()
{
    if constexpr (sizeof(T) == 4) return REV && RB == 4 ? 2 : 4;
    else return !REV && RB == 3 ? 4 : 3;
}

template <typename T, int RB, bool GATED>
__global__ void __launch_bounds__(kMaxPassThreads, (pass_waves_per_eu<T, RB, false>()))
k_pass_fwd(PassTables tb, int64_t item_begin, int64_t item_end)
{
    using V = typename Vec2<T>::type;
    extern __shared__ double smem_d[];
    const EngineLds L = engine_lds<T>(tb, smem_d);
    for (int64_t item = item_begin + blockIdx.x; item < item_end; item += gridDim.x) {
        const FSeg sg = seg_of(tb, item);
        const int tile = (int)(item - sg.first);
        const FCirc cc = ld_const(as_const(tb.circs) + sg.circ);
        if (cc.reg) item_reg_fwd<T, RB, GATED>(tb, cc, sg.stage, tile, (V*)L.tileA);
        else item_lds<T, GATED>(tb, cc, true, sg.stage, tile, (V*)L.tileA, (V*)L.tileB, L.hi_map, L.wpart);
        __syncthreads();  // LDS is reused by the next item of this workgroup
    }
}

template <typename T>
__global__ void __launch_bounds__(kMaxPassThreads)
k_pass_obs(PassTables tb, int64_t item_begin, int64_t item_end)
{
    __shared__ double red[16];
    for (int64_t item = item_begin + blockIdx.x; item < item_end; item += gridDim.x) {
        const FSeg sg = seg_of(tb, item);
        item_observable<T>(tb, ld_const(as_const(tb.circs) + sg.circ), (int)(item - sg.first), red);
        __syncthreads();
    }
}

template <typename T, int RB>
__global__ void __launch_bounds__(kMaxPassThreads, (pass_waves_per_eu<T, RB, true>()))
k_pass_rev(PassTables tb, int64_t item_begin, int64_t item_end)
{
    using V = typename Vec2<T>::type;
    extern __shared__ double smem_d[];
    const EngineLds L = engine_lds<T>(tb, smem_d);
    for (int64_t item = item_begin + blockIdx.x; item < item_end; item += gridDim.x) {
        const FSeg sg = seg_of(tb, item);
        const int tile = (int)(item - sg.first);
        const FCirc cc = ld_const(as_const(tb.circs) + sg.circ);
        const int pidx = 2 * cc.n_pass - sg.stage;  // reverse stage n_pass+1+r -> pass n_pass-1-r
        if (cc.rreg) item_reg_rev<T, RB>(tb, cc, pidx, tile, (V*)L.tileA, L.wpart);
        else item_lds<T, true>(tb, cc, false, pidx, tile, (V*)L.tileA, (V*)L.tileB, L.hi_map, L.wpart);
        __syncthreads();
    }
}

// The 2x2 (row-major, interleaved) of a one-target gate: rotations from the
// parameter, fixed gates from fixed[0..7].
__device__ void gate2x2(const FCoefSpec& f, const double* __restrict__ params, double* u)
{
    const double th = f.pidx >= 0 ? params[f.pidx] : f.value;
    const double ch = cos(th / 2), sh = sin(th / 2);
    switch (f.gate) {
    case SV_RX: u[0] = ch; u[1] = 0; u[2] = 0; u[3] = -sh; u[4] = 0; u[5] = -sh; u[6] = ch; u[7] = 0; break;
    case SV_RY: u[0] = ch; u[1] = 0; u[2] = -sh; u[3] = 0; u[4] = sh; u[5] = 0; u[6] = ch; u[7] = 0; break;
    case SV_RZ: u[0] = ch; u[1] = -sh; u[2] = 0; u[3] = 0; u[4] = 0; u[5] = 0; u[6] = ch; u[7] = sh; break;
    case SV_PHASE: u[0] = 1; u[1] = 0; u[2] = 0; u[3] = 0; u[4] = 0; u[5] = 0; u[6] = cos(th); u[7] = sin(th); break;
    default:
        for (int k = 0; k < 8; ++k) u[k] = f.fixed[k];
        break;
    }
}

// r = a b for 2x2 complex matrices (row-major, interleaved); r may not alias.
__device__ void mul2x2(const double* a, const double* b, double* r)
{
    for (int row = 0; row < 2; ++row)
        for (int col = 0; col < 2; ++col) {
            double re = 0, im = 0;
            for (int t = 0; t < 2; ++t) {
                const double ar = a[2 * (2 * row + t)], ai = a[2 * (2 * row + t) + 1];
                const double br = b[2 * (2 * t + col)], bi = b[2 * (2 * t + col) + 1];
                re += ar * br - ai * bi;
                im += ar * bi + ai * br;
            }
            r[2 * (2 * row + col)] = re;
            r[2 * (2 * row + col) + 1] = im;
        }
}

// One thread per op: gate coefficients from the parameters, in double and
// (if coef_f is set) rounded once to float for complex64 runs.
__global__ void k_pass_coef(const FCoefSpec* __restrict__ spec, int n, const FCoefSpec* __restrict__ factors,
                            const double* __restrict__ params, double* __restrict__ coef, float* __restrict__ coef_f)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const FCoefSpec s = spec[i];
    double* c = coef + s.coef;
    int cnt;
    if (s.nfactor == 2 && s.out_diag == 4) {
        // reverse pair A then B: the product B A, and B G_A B^dagger
        double ua[8], ub[8];
        gate2x2(factors[s.factor_begin], params, ua);
        gate2x2(factors[s.factor_begin + 1], params, ub);
        mul2x2(ub, ua, c);
        if (s.branch > 0) {
            double gm[8] = {0, 0, 0, 0, 0, 0, 0, 0}, t[8], ubd[8];
            switch (s.branch - 1) {
            case GEN_X: gm[2] = 1; gm[4] = 1; break;
            case GEN_Y: gm[3] = -1; gm[5] = 1; break;
            case GEN_Z: gm[0] = 1; gm[6] = -1; break;
            default: gm[6] = 1; break;  // GEN_P1: the projector on |1>
            }
            // B^dagger: conjugate transpose
            ubd[0] = ub[0]; ubd[1] = -ub[1]; ubd[2] = ub[4]; ubd[3] = -ub[5];
            ubd[4] = ub[2]; ubd[5] = -ub[3]; ubd[6] = ub[6]; ubd[7] = -ub[7];
            mul2x2(gm, ubd, t);
            mul2x2(ub, t, c + 8);
        } else {
            for (int k = 8; k < 16; ++k) c[k] = 0.0;
        }
        cnt = 16;
    } else if (s.nfactor > 0 && s.out_diag == 3) {
        // tile-selected product: entry e stands for the tiles whose bits under
        // the mask read e; a factor enters if those bits hold all of its own
        const uint32_t mask = (uint32_t)s.branch;
        const int ne = 1 << __popc(mask);
        for (int e = 0; e < ne; ++e) {
            uint32_t bits = 0;  // e deposited onto the mask's bits
            int k = 0;
            for (uint32_t m = mask; m; m &= m - 1, ++k)
                if ((e >> k) & 1) bits |= m & (~m + 1u);
            double m0[8] = {1, 0, 0, 0, 0, 0, 1, 0};
            for (int f = 0; f < s.nfactor; ++f) {
                const FCoefSpec& fk = factors[s.factor_begin + f];
                if (((uint32_t)fk.branch & ~bits) != 0u) continue;
                double g[8], r[8];
                gate2x2(fk, params, g);
#pragma unroll
                for (int row = 0; row < 2; ++row)
#pragma unroll
                    for (int col = 0; col < 2; ++col) {
                        double re = 0, im = 0;
#pragma unroll
                        for (int t = 0; t < 2; ++t) {
                            const double gr = g[2 * (2 * row + t)], gi = g[2 * (2 * row + t) + 1];
                            const double mr = m0[2 * (2 * t + col)], mi = m0[2 * (2 * t + col) + 1];
                            re += gr * mr - gi * mi;
                            im += gr * mi + gi * mr;
                        }
                        r[2 * (2 * row + col)] = re;
                        r[2 * (2 * row + col) + 1] = im;
                    }
#pragma unroll
                for (int q = 0; q < 8; ++q) m0[q] = r[q];
            }
            for (int q = 0; q < 8; ++q) c[8 * e + q] = m0[q];
        }
        cnt = 8 * ne;
    } else if (s.nfactor > 0) {
        // M = G_last ... G_first; a two-branch product (out_diag 2) keeps M
        // for the selector-0 branch and M1 for the selector-1 branch
        double m[8] = {1, 0, 0, 0, 0, 0, 1, 0}, m1[8] = {1, 0, 0, 0, 0, 0, 1, 0};
        for (int k = 0; k < s.nfactor; ++k) {
            const FCoefSpec& fk = factors[s.factor_begin + k];
            double g[8];
            gate2x2(fk, params, g);
            const int br = s.out_diag == 2 ? fk.branch : 1;
            for (int which = 0; which < 2; ++which) {
                if (!((br >> which) & 1)) continue;
                double* mm = which ? m1 : m;
                double r[8];
#pragma unroll
                for (int row = 0; row < 2; ++row)
#pragma unroll
                    for (int col = 0; col < 2; ++col) {
                        // r[row][col] = sum_t g[row][t] * mm[t][col]
                        double re = 0, im = 0;
#pragma unroll
                        for (int t = 0; t < 2; ++t) {
                            const double gr = g[2 * (2 * row + t)], gi = g[2 * (2 * row + t) + 1];
                            const double mr = mm[2 * (2 * t + col)], mi = mm[2 * (2 * t + col) + 1];
                            re += gr * mr - gi * mi;
                            im += gr * mi + gi * mr;
                        }
                        r[2 * (2 * row + col)] = re;
                        r[2 * (2 * row + col) + 1] = im;
                    }
#pragma unroll
                for (int k2 = 0; k2 < 8; ++k2) mm[k2] = r[k2];
            }
        }
        if (s.out_diag == 2) {
            for (int k = 0; k < 8; ++k) c[k] = m[k];
            for (int k = 0; k < 8; ++k) c[8 + k] = m1[k];
            cnt = 16;
        } else if (s.out_diag) {
            c[0] = m[0]; c[1] = m[1]; c[2] = m[6]; c[3] = m[7];
            cnt = 4;
        } else {
            for (int k = 0; k < 8; ++k) c[k] = m[k];
            cnt = 8;
        }
    } else {
        const double th = s.pidx >= 0 ? params[s.pidx] : s.value;
        const double ch = cos(th / 2), sh = sin(th / 2);
        switch (s.gate) {
        case SV_RX: c[0] = ch; c[1] = 0; c[2] = 0; c[3] = -sh; c[4] = 0; c[5] = -sh; c[6] = ch; c[7] = 0; cnt = 8; break;
        case SV_RY: c[0] = ch; c[1] = 0; c[2] = -sh; c[3] = 0; c[4] = sh; c[5] = 0; c[6] = ch; c[7] = 0; cnt = 8; break;
        case SV_RZ: c[0] = ch; c[1] = -sh; c[2] = ch; c[3] = sh; cnt = 4; break;
        case SV_PHASE: c[0] = cos(th); c[1] = sin(th); cnt = 2; break;
        default:
            for (int k = 0; k < s.nfixed; ++k) c[k] = s.fixed[k];
            cnt = s.nfixed;
            break;
        }
    }
    if (coef_f)
        for (int k = 0; k < cnt; ++k) coef_f[s.coef + k] = (float)c[k];
}

// out[k] = scale[k] * sum_{i < cnt[k]} part[off[k] + i], fixed order.
__global__ void __launch_bounds__(256)
k_pass_segsum(const double* __restrict__ part, const int64_t* __restrict__ off, const int* __restrict__ cnt,
              const double* __restrict__ scale, double* __restrict__ out)
{
    __shared__ double red[4];
    const int k = blockIdx.x;
    const double* p = part + off[k];
    double acc = 0.0;
    for (int i = threadIdx.x; i < cnt[k]; i += blockDim.x) acc += p[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
        out[k] = scale ? scale[k] * s : s;
    }
}

// grad[j] = sum of slot values in the CSR row of parameter j (ascending slots).
__global__ void k_pass_grad_csr(const double* __restrict__ slot_val, const int* __restrict__ rowptr,
                                const int* __restrict__ cols, int n_params, double* __restrict__ grad)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_params) return;
    double g = 0.0;
    for (int k = rowptr[j]; k < rowptr[j + 1]; ++k) g += slot_val[cols[k]];
    grad[j] = g;
}

int pass_engine_threads(int tq_max, int reg_bits)
{
    const int t = tq_max > reg_bits ? 1 << (tq_max - reg_bits) : 1;
    return t < 64 ? 64 : t;
}

size_t pass_engine_lds_bytes(int tq_max, int hi_entries, int with_grad, int dtype, int lds_small, int slot_waves)
{
    const size_t eb = dtype == SV_C128 ? 16 : 8;
    const size_t tiles = (size_t)1 << tq_max;
    return eb * tiles * (lds_small && with_grad ? 2 : 1) + (lds_small ? 8 * (size_t)hi_entries : 0) +
           8 * (size_t)kMaxPassSlots * slot_waves;
}

// The dynamic-LDS limit only grows: batches that are alive at the same time
// launch the same kernels with different LDS sizes.
hipError_t pass_engine_prepare(size_t lds_bytes)
{
    static size_t limit = 0;
    if (lds_bytes <= limit) return hipSuccess;
    const void* f[] = {(const void*)k_pass_fwd<double, 3, false>, (const void*)k_pass_fwd<double, 4, false>,
                       (const void*)k_pass_fwd<double, 3, true>,  (const void*)k_pass_fwd<double, 4, true>,
                       (const void*)k_pass_rev<double, 3>,        (const void*)k_pass_fwd<float, 3, false>,
                       (const void*)k_pass_fwd<float, 4, false>,  (const void*)k_pass_fwd<float, 3, true>,
                       (const void*)k_pass_fwd<float, 4, true>,   (const void*)k_pass_rev<float, 3>,
                       (const void*)k_pass_rev<float, 4>};
    for (const void* k : f) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    limit = lds_bytes;
    return hipSuccess;
}

template <typename T>
static void launch_items_t(const PassTables& tb, int mode, bool gated, unsigned grid, int threads, size_t lds,
                           hipStream_t s, int64_t b, int64_t e)
{
    if (mode == PM_OBS) {
        hipLaunchKernelGGL((k_pass_obs<T>), dim3(grid), dim3(threads), 0, s, tb, b, e);
    } else if (mode == PM_FWD) {
        if (tb.reg_bits == 3) {
            if (gated) hipLaunchKernelGGL((k_pass_fwd<T, 3, true>), dim3(grid), dim3(threads), lds, s, tb, b, e);
            else hipLaunchKernelGGL((k_pass_fwd<T, 3, false>), dim3(grid), dim3(threads), lds, s, tb, b, e);
        } else {
            if (gated) hipLaunchKernelGGL((k_pass_fwd<T, 4, true>), dim3(grid), dim3(threads), lds, s, tb, b, e);
            else hipLaunchKernelGGL((k_pass_fwd<T, 4, false>), dim3(grid), dim3(threads), lds, s, tb, b, e);
        }
    } else if constexpr (sizeof(T) == 8) {
        hipLaunchKernelGGL((k_pass_rev<T, 3>), dim3(grid), dim3(threads), lds, s, tb, b, e);
    } else {
        if (tb.rreg_bits == 3) hipLaunchKernelGGL((k_pass_rev<T, 3>), dim3(grid), dim3(threads), lds, s, tb, b, e);
        else hipLaunchKernelGGL((k_pass_rev<T, 4>), dim3(grid), dim3(threads), lds, s, tb, b, e);
    }
}

hipError_t launch_pass_items(const PassTables& tb, int dtype, int mode, int64_t item_begin, int64_t item_end,
                             int threads, size_t lds_bytes, hipStream_t s, bool gated)
{
    const int64_t n = item_end - item_begin;
    if (n <= 0) return hipSuccess;
    if (threads < 64 || threads > kMaxPassThreads) return hipErrorInvalidValue;
    // one workgroup per item, within the launch limits (blocks below 2^30 and
    // blocks x threads below 2^32); the kernels' item loops cover the rest
    const int64_t cap = std::min<int64_t>(1 << 30, 0xffffffffll / threads);
    const unsigned grid = (unsigned)(n < cap ? n : cap);
    if (dtype == SV_C128) launch_items_t<double>(tb, mode, gated, grid, threads, lds_bytes, s, item_begin, item_end);
    else launch_items_t<float>(tb, mode, gated, grid, threads, lds_bytes, s, item_begin, item_end);
    return hipGetLastError();
}

hipError_t launch_pass_coef(const FCoefSpec* spec, int n, const FCoefSpec* factors, const double* params,
                            double* coef, float* coef_f, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pass_coef, dim3((n + 127) / 128), dim3(128), 0, s, spec, n, factors, params, coef, coef_f);
    return hipGetLastError();
}

hipError_t launch_pass_segsum(const double* part, const int64_t* off, const int* cnt, const double* scale, double* out,
                              int n_seg, hipStream_t s)
{
    if (n_seg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pass_segsum, dim3(n_seg), dim3(256), 0, s, part, off, cnt, scale, out);
    return hipGetLastError();
}

hipError_t launch_pass_grad_csr(const double* slot_val, const int* rowptr, const int* cols, int n_params, double* grad,
                                hipStream_t s)
{
    if (n_params <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pass_grad_csr, dim3((n_params + 255) / 256), dim3(256), 0, s, slot_val, rowptr, cols,
                       n_params, grad);
    return hipGetLastError();
}

}  // namespace svk
