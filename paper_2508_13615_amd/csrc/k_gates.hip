// k_gates.hip -- gate kernels for gfx950 (MI355X).
//
// Sec. 2 of the paper: each gate is applied only through the non-zero
// elements of its logic matrix, and a control only selects where it acts.
// The kernels below are the GPU form of that rule, one per gate class:
//   k_pair    two members per group (base + o0, base + o1): permutations
//             (X, CNOT, Toffoli, SWAP: pure moves), butterflies (H, RX,
//             RY, Y, U2 and their controlled forms) and the two-phase
//             diagonal RZ, which touches every amplitude of its subspace;
//   k_one     one member per group: phase on the |1..1> subspace of the
//             gate's qubits (Z, S, T, PHASE, CZ, controlled phase);
//   k_quad    four members per group (U4 on two targets);
//   k_general the dense 2^K x 2^K product with no structure used (the
//             "general approach" of Sec. 3.1, the baseline).
//
// All kernels are HBM-bound streams.  Each thread owns U groups spaced one
// block apart, so every load instruction of a wavefront reads consecutive
// groups; when the lowest inserted bit is >= 3 (complex128) those are whole
// 128-byte lines, below that the loads of a wave together cover every line
// they touch.  All U groups are loaded before any is written.  Measured on
// MI355X at 30 qubits, one group per thread in small blocks with
// non-temporal loads and stores streams fastest once the touched runs span
// at least 64 bytes; below that (a gate or control on bit 0 or 1 of a
// complex128 state) non-temporal accesses of partial lines cost up to 35%,
// so the launch table (sv_api.hip) switches them off there.
#include <algorithm>
#include <type_traits>

#include "sv_core.h"

namespace svk {

template <typename V, typename T>
__device__ __forceinline__ V cmul(T ur, T ui, V a)
{
    V r;
    r.x = ur * a.x - ui * a.y;
    r.y = ur * a.y + ui * a.x;
    return r;
}

template <typename V, typename T>
__device__ __forceinline__ V cmad2(T ar_, T ai_, V a, T br_, T bi_, V b)
{
    V r;
    r.x = (ar_ * a.x - ai_ * a.y) + (br_ * b.x - bi_ * b.y);
    r.y = (ar_ * a.y + ai_ * a.x) + (br_ * b.y + bi_ * b.x);
    return r;
}

template <int OP, typename T, typename V>
__device__ __forceinline__ void pair_apply(const V a0, const V a1, const Coef2<T>& c, V& r0, V& r1)
{
    if constexpr (OP == PAIR_SWAP) {
        r0 = a1;
        r1 = a0;
    } else if constexpr (OP == PAIR_Y) {
        r0.x = a1.y;
        r0.y = -a1.x;
        r1.x = -a0.y;
        r1.y = a0.x;
    } else if constexpr (OP == PAIR_REAL) {
        r0.x = c.m[0] * a0.x + c.m[2] * a1.x;
        r0.y = c.m[0] * a0.y + c.m[2] * a1.y;
        r1.x = c.m[4] * a0.x + c.m[6] * a1.x;
        r1.y = c.m[4] * a0.y + c.m[6] * a1.y;
    } else if constexpr (OP == PAIR_DIAG) {
        r0 = cmul<V, T>(c.m[0], c.m[1], a0);
        r1 = cmul<V, T>(c.m[6], c.m[7], a1);
    } else if constexpr (OP == PAIR_RX) {
        const T cc = c.m[0], s = -c.m[3];  // m01 = -i s
        r0.x = cc * a0.x + s * a1.y;
        r0.y = cc * a0.y - s * a1.x;
        r1.x = cc * a1.x + s * a0.y;
        r1.y = cc * a1.y - s * a0.x;
    } else {
        r0 = cmad2<V, T>(c.m[0], c.m[1], a0, c.m[2], c.m[3], a1);
        r1 = cmad2<V, T>(c.m[4], c.m[5], a0, c.m[6], c.m[7], a1);
    }
}

template <typename T, int OP, int U, bool NT>
__global__ void __launch_bounds__(1024)
k_pair(typename Vec2<T>::type* __restrict__ psi, GroupSpec gs, uint64_t o0, uint64_t o1, Coef2<T> c)
{
    using V = typename Vec2<T>::type;
    const uint64_t per_block = (uint64_t)blockDim.x * U;
    const uint64_t stride = (uint64_t)gridDim.x * per_block;
    const uint64_t first = block_slot(blockIdx.x, gridDim.x, gs.order) * per_block;
    for (uint64_t g0 = first + threadIdx.x; g0 < gs.n_groups + threadIdx.x; g0 += stride) {
        uint64_t b[U];
        V a0[U], a1[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t g = g0 + (uint64_t)j * blockDim.x;
            if (g < gs.n_groups) {
                b[j] = group_base(g, gs);
                a0[j] = ldg<NT>(psi + b[j] + o0);
                a1[j] = ldg<NT>(psi + b[j] + o1);
            }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t g = g0 + (uint64_t)j * blockDim.x;
            if (g < gs.n_groups) {
                V r0, r1;
                pair_apply<OP, T, V>(a0[j], a1[j], c, r0, r1);
                if ((b[j] & gs.pmask) != gs.pmask) {
                    r0 = a0[j];
                    r1 = a1[j];
                }
                stg<NT>(psi + b[j] + o0, r0);
                stg<NT>(psi + b[j] + o1, r1);
            }
        }
    }
}

// Paired update for a target t < 6 with the partner fetched across lanes.
// The lane's own output is row bit_t(x) of the 2x2 product; groups failing the
// control predicate keep their amplitude.  Every lane of a wavefront runs the
// shuffles (the loop bound is uniform per block), so inactive tail lanes only
// supply values nobody reads: the partner of a valid x is x ^ 2^t < 2^n.
template <typename T, int OP, int U, bool NT>
__global__ void __launch_bounds__(1024)
k_wpair(typename Vec2<T>::type* __restrict__ psi, GroupSpec gs, int t, Coef2<T> c)
{
    using V = typename Vec2<T>::type;
    const uint64_t per_block = (uint64_t)blockDim.x * U;
    const uint64_t stride = (uint64_t)gridDim.x * per_block;
    const int lm = 1 << t;
    const uint64_t first = block_slot(blockIdx.x, gridDim.x, gs.order) * per_block;
    for (uint64_t g0 = first + threadIdx.x; g0 < gs.n_groups + threadIdx.x; g0 += stride) {
        uint64_t x[U];
        V a[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t g = g0 + (uint64_t)j * blockDim.x;
            x[j] = group_base(g < gs.n_groups ? g : 0, gs);
            if (g < gs.n_groups) {
                a[j] = ldg<NT>(psi + x[j]);
            } else {
                a[j].x = T(0);
                a[j].y = T(0);
            }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t g = g0 + (uint64_t)j * blockDim.x;
            const bool hi = (x[j] >> t) & 1ull;
            V r;
            if constexpr (OP == PAIR_DIAG) {
                // a diagonal needs no partner: the lane's own phase by its bit t
                r = hi ? cmul<V, T>(c.m[6], c.m[7], a[j]) : cmul<V, T>(c.m[0], c.m[1], a[j]);
            } else {
                V p;
                p.x = __shfl_xor(a[j].x, lm, 64);
                p.y = __shfl_xor(a[j].y, lm, 64);
                V r0, r1;
                pair_apply<OP, T, V>(hi ? p : a[j], hi ? a[j] : p, c, r0, r1);
                r = hi ? r1 : r0;
            }
            if (g < gs.n_groups) {
                if ((x[j] & gs.pmask) != gs.pmask) r = a[j];
                stg<NT>(psi + x[j], r);
            }
        }
    }
}

template <typename T, int OP, int U, bool NT>
__global__ void __launch_bounds__(1024)
k_one(typename Vec2<T>::type* __restrict__ psi, GroupSpec gs, T zr, T zi)
{
    using V = typename Vec2<T>::type;
    const uint64_t per_block = (uint64_t)blockDim.x * U;
    const uint64_t stride = (uint64_t)gridDim.x * per_block;
    const uint64_t first = block_slot(blockIdx.x, gridDim.x, gs.order) * per_block;
    for (uint64_t g0 = first + threadIdx.x; g0 < gs.n_groups + threadIdx.x; g0 += stride) {
        uint64_t b[U];
        V a[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t g = g0 + (uint64_t)j * blockDim.x;
            if (g < gs.n_groups) {
                b[j] = group_base(g, gs);
                a[j] = ldg<NT>(psi + b[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t g = g0 + (uint64_t)j * blockDim.x;
            if (g < gs.n_groups) {
                V r;
                if constexpr (OP == ONE_NEG) {
                    r.x = -a[j].x;
                    r.y = -a[j].y;
                } else if constexpr (OP == ONE_MULI) {
                    // zr = +1: i*a = (-a.y, a.x); zr = -1: -i*a = (a.y, -a.x)
                    r.x = zr > T(0) ? -a[j].y : a[j].y;
                    r.y = zr > T(0) ? a[j].x : -a[j].x;
                } else {
                    r = cmul<V, T>(zr, zi, a[j]);
                }
                if ((b[j] & gs.pmask) != gs.pmask) r = a[j];
                stg<NT>(psi + b[j], r);
            }
        }
    }
}

template <typename T, int U, bool NT>
__global__ void __launch_bounds__(1024)
k_quad(typename Vec2<T>::type* __restrict__ psi, GroupSpec gs, uint64_t o1, uint64_t o2, uint64_t o3,
       Coef4<T> c)
{
    using V = typename Vec2<T>::type;
    const uint64_t per_block = (uint64_t)blockDim.x * U;
    const uint64_t stride = (uint64_t)gridDim.x * per_block;
    const uint64_t first = block_slot(blockIdx.x, gridDim.x, gs.order) * per_block;
    for (uint64_t g0 = first + threadIdx.x; g0 < gs.n_groups + threadIdx.x; g0 += stride) {
        uint64_t b[U];
        V a[U][4];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t g = g0 + (uint64_t)j * blockDim.x;
            if (g < gs.n_groups) {
                b[j] = group_base(g, gs);
                a[j][0] = ldg<NT>(psi + b[j]);
                a[j][1] = ldg<NT>(psi + b[j] + o1);
                a[j][2] = ldg<NT>(psi + b[j] + o2);
                a[j][3] = ldg<NT>(psi + b[j] + o3);
            }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t g = g0 + (uint64_t)j * blockDim.x;
            if (g < gs.n_groups) {
                // each row is stored as soon as it is formed (holding all four
                // results until the end measured 2-5% slower at 30 qubits)
                const bool act = (b[j] & gs.pmask) == gs.pmask;
#pragma unroll
                for (int row = 0; row < 4; ++row) {
                    T sr = T(0), si = T(0);
#pragma unroll
                    for (int col = 0; col < 4; ++col) {
                        const T ur = c.m[2 * (4 * row + col)], ui = c.m[2 * (4 * row + col) + 1];
                        sr += ur * a[j][col].x - ui * a[j][col].y;
                        si += ur * a[j][col].y + ui * a[j][col].x;
                    }
                    V r;
                    r.x = act ? sr : a[j][row].x;
                    r.y = act ? si : a[j][row].y;
                    stg<NT>(psi + b[j] + (row == 0 ? 0 : row == 1 ? o1 : row == 2 ? o2 : o3), r);
                }
            }
        }
    }
}

template <typename T, int K, int U, bool NT>
__global__ void __launch_bounds__(1024)
k_general(typename Vec2<T>::type* __restrict__ psi, GroupSpec gs, GeneralSpec<T, K> sp)
{
    using V = typename Vec2<T>::type;
    constexpr int M = 1 << K;
    const uint64_t per_block = (uint64_t)blockDim.x * U;
    const uint64_t stride = (uint64_t)gridDim.x * per_block;
    const uint64_t first = block_slot(blockIdx.x, gridDim.x, gs.order) * per_block;
    for (uint64_t g0 = first + threadIdx.x; g0 < gs.n_groups + threadIdx.x; g0 += stride) {
        uint64_t b[U];
        V a[U][M];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t g = g0 + (uint64_t)j * blockDim.x;
            if (g < gs.n_groups) {
                b[j] = group_base(g, gs);
#pragma unroll
                for (int r = 0; r < M; ++r) a[j][r] = ldg<NT>(psi + b[j] + sp.off[r]);
            }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t g = g0 + (uint64_t)j * blockDim.x;
            if (g < gs.n_groups) {
#pragma unroll
                for (int row = 0; row < M; ++row) {
                    T sr = T(0), si = T(0);
#pragma unroll
                    for (int col = 0; col < M; ++col) {
                        const T ur = sp.m[2 * (M * row + col)], ui = sp.m[2 * (M * row + col) + 1];
                        sr += ur * a[j][col].x - ui * a[j][col].y;
                        si += ur * a[j][col].y + ui * a[j][col].x;
                    }
                    V r;
                    r.x = sr;
                    r.y = si;
                    stg<NT>(psi + b[j] + sp.off[row], r);
                }
            }
        }
    }
}

// LDS-staged gate for gates with a low qubit (runs under 1 KiB): whole
// contiguous chunks are streamed in and out non-temporally, so every access is
// a full line however low the gate's qubits sit; the gate itself runs in LDS.
template <typename T, int K, int OP, bool NT, int B>
__global__ void __launch_bounds__(1024)
k_lds_gate(typename Vec2<T>::type* __restrict__ psi, GroupSpec tiles, LdsSpec ls, GeneralSpec<T, K> sp)
{
    using V = typename Vec2<T>::type;
    extern __shared__ double st_raw[];  // 2^(C + h) amplitudes, sized at launch
    V* const st = (V*)st_raw;
    constexpr int C = kLdsChunkBits;
    constexpr int M = 1 << K;
    const uint32_t nl = 1u << (C + ls.h);
    const uint32_t cmask_lo = (1u << C) - 1u;
    // stage element l (0 .. nl - 1) <-> state index: its low C bits stay in
    // place, bit j of l >> C goes to gate qubit hq[j]
    auto index_of = [&](uint64_t base, uint32_t l) {
        uint64_t g = base | (l & cmask_lo);
        const uint32_t hc = l >> C;
        for (int j = 0; j < ls.h; ++j)
            if ((hc >> j) & 1u) g |= 1ull << ls.hq[j];
        return g;
    };
    // B > 1: a thread issues B loads before its first LDS write (and B LDS
    // reads before its first store), so B lines per thread are in flight.
    // That pays where the gate's registers already limit the waves per SIMD
    // (the 3-qubit form); B = 1 keeps the registers, and with them the waves
    // in flight, at their lowest.
    const uint32_t step = blockDim.x * B;
    for (uint64_t tile = block_slot(blockIdx.x, gridDim.x, tiles.order); tile < tiles.n_groups; tile += gridDim.x) {
        const uint64_t base = (group_base(tile, tiles) << C) | ls.cmask;
        if constexpr (B == 1) {
            for (uint32_t l = threadIdx.x; l < nl; l += blockDim.x) st[l] = ldg<NT>(psi + index_of(base, l));
        } else {
            for (uint32_t l0 = threadIdx.x; l0 < nl; l0 += step) {
                V buf[B];
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const uint32_t l = l0 + u * blockDim.x;
                    if (l < nl) buf[u] = ldg<NT>(psi + index_of(base, l));
                }
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const uint32_t l = l0 + u * blockDim.x;
                    if (l < nl) st[l] = buf[u];
                }
            }
        }
        __syncthreads();
        const uint32_t ng = nl >> K;
        for (uint32_t p = threadIdx.x; p < ng; p += blockDim.x) {
            uint32_t lb = p;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int q = ls.lsort[j];
                lb = ((lb >> q) << (q + 1)) | (lb & ((1u << q) - 1u));
            }
            if ((lb & ls.pmask) != ls.pmask) continue;
            uint32_t idx[M];
#pragma unroll
            for (int r = 0; r < M; ++r) {
                uint32_t o = lb;
#pragma unroll
                for (int j = 0; j < K; ++j)
                    if ((r >> (K - 1 - j)) & 1) o |= 1u << ls.lpos[j];
                idx[r] = o;
            }
            if constexpr (OP == 1) {
                const V a = st[idx[1]];
                st[idx[1]] = st[idx[2]];
                st[idx[2]] = a;
            } else {
                V v[M];
#pragma unroll
                for (int r = 0; r < M; ++r) v[r] = st[idx[r]];
#pragma unroll
                for (int row = 0; row < M; ++row) {
                    T sr = T(0), si = T(0);
#pragma unroll
                    for (int col = 0; col < M; ++col) {
                        const T ur = sp.m[2 * (M * row + col)], ui = sp.m[2 * (M * row + col) + 1];
                        sr += ur * v[col].x - ui * v[col].y;
                        si += ur * v[col].y + ui * v[col].x;
                    }
                    V w;
                    w.x = sr;
                    w.y = si;
                    st[idx[row]] = w;
                }
            }
        }
        __syncthreads();
        if constexpr (B == 1) {
            for (uint32_t l = threadIdx.x; l < nl; l += blockDim.x) stg<NT>(psi + index_of(base, l), st[l]);
        } else {
            for (uint32_t l0 = threadIdx.x; l0 < nl; l0 += step) {
                V buf[B];
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const uint32_t l = l0 + u * blockDim.x;
                    if (l < nl) buf[u] = st[l];
                }
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const uint32_t l = l0 + u * blockDim.x;
                    if (l < nl) stg<NT>(psi + index_of(base, l), buf[u]);
                }
            }
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void k_set_basis(typename Vec2<T>::type* __restrict__ psi, uint64_t n_amps, uint64_t index)
{
    using V = typename Vec2<T>::type;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n_amps; x += stride) {
        V v;
        v.x = x == index ? T(1) : T(0);
        v.y = T(0);
        psi[x] = v;
    }
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
// Workgroups for a grid-stride loop over n work units of `per` each: at most
// 2^30 of them, and blocks x threads below 2^32 (the launch limit of one grid
// dimension; 32-qubit states reach it).
static uint64_t grid_cap(uint64_t nb, int block)
{
    const uint64_t lim = std::min<uint64_t>(1ull << 30, 0xffffffffull / (uint64_t)block);
    return nb < 1 ? 1 : (nb > lim ? lim : nb);
}

static dim3 grid_for(uint64_t n_groups, int block, int unroll)
{
    const uint64_t per = (uint64_t)block * (uint64_t)unroll;
    return dim3((unsigned)grid_cap((n_groups + per - 1) / per, block));  // the stride loop covers the rest
}

// Launch-shape dispatch: unroll U in {1, 2, 4} and the non-temporal flag.
#define SV_SHAPE_SWITCH(lc, ...)                                                        \
    do {                                                                                \
        if ((lc).nt) {                                                                  \
            constexpr bool NTT = true;                                                  \
            switch ((lc).unroll) {                                                      \
            case 1: { constexpr int UU = 1; __VA_ARGS__; } break;                       \
            case 2: { constexpr int UU = 2; __VA_ARGS__; } break;                       \
            default: { constexpr int UU = 4; __VA_ARGS__; } break;                      \
            }                                                                           \
        } else {                                                                        \
            constexpr bool NTT = false;                                                 \
            switch ((lc).unroll) {                                                      \
            case 1: { constexpr int UU = 1; __VA_ARGS__; } break;                       \
            case 2: { constexpr int UU = 2; __VA_ARGS__; } break;                       \
            default: { constexpr int UU = 4; __VA_ARGS__; } break;                      \
            }                                                                           \
        }                                                                               \
    } while (0)

template <typename T>
hipError_t launch_pair(void* psi, const GroupSpec& gs, uint64_t o0, uint64_t o1, int op, const Coef2<T>& c,
                       hipStream_t s, Launch lc)
{
    using V = typename Vec2<T>::type;
    if (gs.n_groups == 0) return hipSuccess;
    V* p = (V*)psi;
    SV_SHAPE_SWITCH(lc, {
        const dim3 grid = grid_for(gs.n_groups, lc.block, UU);
        const dim3 blk(lc.block);
        switch (op) {
        case PAIR_SWAP: hipLaunchKernelGGL((k_pair<T, PAIR_SWAP, UU, NTT>), grid, blk, 0, s, p, gs, o0, o1, c); break;
        case PAIR_Y: hipLaunchKernelGGL((k_pair<T, PAIR_Y, UU, NTT>), grid, blk, 0, s, p, gs, o0, o1, c); break;
        case PAIR_REAL: hipLaunchKernelGGL((k_pair<T, PAIR_REAL, UU, NTT>), grid, blk, 0, s, p, gs, o0, o1, c); break;
        case PAIR_RX: hipLaunchKernelGGL((k_pair<T, PAIR_RX, UU, NTT>), grid, blk, 0, s, p, gs, o0, o1, c); break;
        case PAIR_DIAG: hipLaunchKernelGGL((k_pair<T, PAIR_DIAG, UU, NTT>), grid, blk, 0, s, p, gs, o0, o1, c); break;
        default: hipLaunchKernelGGL((k_pair<T, PAIR_DENSE, UU, NTT>), grid, blk, 0, s, p, gs, o0, o1, c); break;
        }
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_wpair(void* psi, const GroupSpec& gs, int t, int op, const Coef2<T>& c, hipStream_t s,
                        Launch lc)
{
    using V = typename Vec2<T>::type;
    if (gs.n_groups == 0) return hipSuccess;
    if (t < 0 || t > 5 || (lc.block & 63)) return hipErrorInvalidValue;
    V* p = (V*)psi;
    SV_SHAPE_SWITCH(lc, {
        const dim3 grid = grid_for(gs.n_groups, lc.block, UU);
        const dim3 blk(lc.block);
        switch (op) {
        case PAIR_SWAP: hipLaunchKernelGGL((k_wpair<T, PAIR_SWAP, UU, NTT>), grid, blk, 0, s, p, gs, t, c); break;
        case PAIR_Y: hipLaunchKernelGGL((k_wpair<T, PAIR_Y, UU, NTT>), grid, blk, 0, s, p, gs, t, c); break;
        case PAIR_REAL: hipLaunchKernelGGL((k_wpair<T, PAIR_REAL, UU, NTT>), grid, blk, 0, s, p, gs, t, c); break;
        case PAIR_RX: hipLaunchKernelGGL((k_wpair<T, PAIR_RX, UU, NTT>), grid, blk, 0, s, p, gs, t, c); break;
        case PAIR_DIAG: hipLaunchKernelGGL((k_wpair<T, PAIR_DIAG, UU, NTT>), grid, blk, 0, s, p, gs, t, c); break;
        default: hipLaunchKernelGGL((k_wpair<T, PAIR_DENSE, UU, NTT>), grid, blk, 0, s, p, gs, t, c); break;
        }
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_one(void* psi, const GroupSpec& gs, int op, T zr, T zi, hipStream_t s, Launch lc)
{
    using V = typename Vec2<T>::type;
    if (gs.n_groups == 0) return hipSuccess;
    V* p = (V*)psi;
    SV_SHAPE_SWITCH(lc, {
        const dim3 grid = grid_for(gs.n_groups, lc.block, UU);
        const dim3 blk(lc.block);
        switch (op) {
        case ONE_NEG: hipLaunchKernelGGL((k_one<T, ONE_NEG, UU, NTT>), grid, blk, 0, s, p, gs, zr, zi); break;
        case ONE_MULI: hipLaunchKernelGGL((k_one<T, ONE_MULI, UU, NTT>), grid, blk, 0, s, p, gs, zr, zi); break;
        default: hipLaunchKernelGGL((k_one<T, ONE_MUL, UU, NTT>), grid, blk, 0, s, p, gs, zr, zi); break;
        }
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_quad(void* psi, const GroupSpec& gs, const uint64_t off[4], const Coef4<T>& c, hipStream_t s,
                       Launch lc)
{
    using V = typename Vec2<T>::type;
    if (gs.n_groups == 0) return hipSuccess;
    V* p = (V*)psi;
    SV_SHAPE_SWITCH(lc, {
        hipLaunchKernelGGL((k_quad<T, UU, NTT>), grid_for(gs.n_groups, lc.block, UU), dim3(lc.block), 0, s, p, gs,
                           off[1], off[2], off[3], c);
    });
    return hipGetLastError();
}

template <typename T, int K>
static hipError_t launch_general_k(typename Vec2<T>::type* p, const GroupSpec& gs, const uint64_t* off,
                                   const T* m, hipStream_t s, Launch lc)
{
    GeneralSpec<T, K> sp;
    for (int r = 0; r < (1 << K); ++r) sp.off[r] = off[r];
    for (int i = 0; i < 2 * (1 << K) * (1 << K); ++i) sp.m[i] = m[i];
    SV_SHAPE_SWITCH(lc, {
        hipLaunchKernelGGL((k_general<T, K, UU, NTT>), grid_for(gs.n_groups, lc.block, UU), dim3(lc.block), 0, s, p,
                           gs, sp);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_general(void* psi, const GroupSpec& gs, int k, const uint64_t* off, const T* m, hipStream_t s,
                          Launch lc)
{
    using V = typename Vec2<T>::type;
    if (gs.n_groups == 0) return hipSuccess;
    V* p = (V*)psi;
    switch (k) {
    case 1: return launch_general_k<T, 1>(p, gs, off, m, s, lc);
    case 2: return launch_general_k<T, 2>(p, gs, off, m, s, lc);
    case 3: return launch_general_k<T, 3>(p, gs, off, m, s, lc);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int K>
static hipError_t launch_lds_k(typename Vec2<T>::type* p, const GroupSpec& tiles, const LdsSpec& ls, int op,
                               const T* m, hipStream_t s, Launch lc)
{
    GeneralSpec<T, K> sp{};
    if (m)
        for (int i = 0; i < 2 * (1 << K) * (1 << K); ++i) sp.m[i] = m[i];
    const int block = lds_block(K, ls.h, op, (int)sizeof(typename Vec2<T>::type), lc.block);
    const dim3 grid((unsigned)grid_cap(tiles.n_groups, block)), blk(block);
    const size_t lds = sizeof(typename Vec2<T>::type) << (kLdsChunkBits + ls.h);
    if (op == 1 && K != 2) return hipErrorInvalidValue;
    // lines a thread stages per round trip: lds_stage_depth (the 3-qubit form
    // takes the launch shape's unroll; complex128 2-qubit forms stage one,
    // measured faster at 30 qubits: 5.62 against 5.76 ms per gate)
    auto go = [&](auto nt_tag, auto b_tag) {
        constexpr bool NTv = decltype(nt_tag)::value;
        constexpr int Bv = decltype(b_tag)::value;
        if (op == 1) {
            if constexpr (K == 2) hipLaunchKernelGGL((k_lds_gate<T, 2, 1, NTv, Bv>), grid, blk, lds, s, p, tiles, ls, sp);
        } else {
            hipLaunchKernelGGL((k_lds_gate<T, K, 0, NTv, Bv>), grid, blk, lds, s, p, tiles, ls, sp);
        }
    };
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I4 = std::integral_constant<int, 4>;
    const int b = lds_stage_depth(K, lc.unroll, (int)sizeof(typename Vec2<T>::type));
    if (lc.nt) {
        if constexpr (K == 3) {
            if (b == 4) go(std::true_type{}, I4{});
            else if (b == 2) go(std::true_type{}, I2{});
            else go(std::true_type{}, I1{});
        } else if constexpr (K == 2 && sizeof(T) == 4) {
            if (b == 2) go(std::true_type{}, I2{});
            else go(std::true_type{}, I1{});
        } else {
            go(std::true_type{}, I1{});
        }
    } else {
        if constexpr (K == 3) {
            if (b == 4) go(std::false_type{}, I4{});
            else if (b == 2) go(std::false_type{}, I2{});
            else go(std::false_type{}, I1{});
        } else if constexpr (K == 2 && sizeof(T) == 4) {
            if (b == 2) go(std::false_type{}, I2{});
            else go(std::false_type{}, I1{});
        } else {
            go(std::false_type{}, I1{});
        }
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_lds_gate(void* psi, const GroupSpec& tiles, const LdsSpec& ls, int op, const T* m, hipStream_t s,
                           Launch lc)
{
    using V = typename Vec2<T>::type;
    if (tiles.n_groups == 0) return hipSuccess;
    if (ls.h < 0 || ls.h > 3 || (lc.block & 63)) return hipErrorInvalidValue;
    V* p = (V*)psi;
    switch (ls.k) {
    case 1: return launch_lds_k<T, 1>(p, tiles, ls, op, m, s, lc);
    case 2: return launch_lds_k<T, 2>(p, tiles, ls, op, m, s, lc);
    case 3: return launch_lds_k<T, 3>(p, tiles, ls, op, m, s, lc);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_set_basis(void* psi, uint64_t n_amps, uint64_t index, hipStream_t s)
{
    using V = typename Vec2<T>::type;
    uint64_t nb = (n_amps + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL((k_set_basis<T>), dim3((unsigned)nb), dim3(256), 0, s, (V*)psi, n_amps, index);
    return hipGetLastError();
}

#define SV_INSTANTIATE(T)                                                                                   \
    template hipError_t launch_pair<T>(void*, const GroupSpec&, uint64_t, uint64_t, int, const Coef2<T>&,   \
                                       hipStream_t, Launch);                                                \
    template hipError_t launch_one<T>(void*, const GroupSpec&, int, T, T, hipStream_t, Launch);             \
    template hipError_t launch_wpair<T>(void*, const GroupSpec&, int, int, const Coef2<T>&, hipStream_t,      \
                                        Launch);                                                            \
    template hipError_t launch_quad<T>(void*, const GroupSpec&, const uint64_t[4], const Coef4<T>&,         \
                                       hipStream_t, Launch);                                                \
    template hipError_t launch_general<T>(void*, const GroupSpec&, int, const uint64_t*, const T*,          \
                                          hipStream_t, Launch);                                             \
    template hipError_t launch_set_basis<T>(void*, uint64_t, uint64_t, hipStream_t);                         \
    template hipError_t launch_lds_gate<T>(void*, const GroupSpec&, const LdsSpec&, int, const T*, hipStream_t, \
                                           Launch);

SV_INSTANTIATE(double)
SV_INSTANTIATE(float)

}  // namespace svk
