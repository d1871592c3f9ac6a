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

template <typename V, typename T>
__device__ __forceinline__ V cmul_add2(T ar_, T ai_, V a, T br_, T bi_, V b)
{
    V r;
    r.x = (ar_ * a.x - ai_ * a.y) + (br_ * b.x - bi_ * b.y);
    r.y = (ar_ * a.y + ai_ * a.x) + (br_ * b.y + bi_ * b.x);
    return r;
}

__device__ __forceinline__ uint32_t ins0(uint32_t x, int p)
{
    const uint32_t lo = x & ((1u << p) - 1u);
    return ((x >> p) << (p + 1)) | lo;
}

// Coefficients of a 2x2 (row-major, interleaved) or its conjugate transpose.
template <typename T>
__device__ __forceinline__ void load2x2(const double* cf, bool dagger, T* u)
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

// Apply one op (or its inverse) to an LDS tile of 2^tq amplitudes.
template <typename T>
__device__ void lds_apply(typename Vec2<T>::type* A, const FOp& op, const double* __restrict__ coef, bool dagger,
                          int tq)
{
    using V = typename Vec2<T>::type;
    const int nthr = blockDim.x;
    const uint32_t cm = op.cm;
    const double* cf = coef + op.coef;
    switch (op.kind) {
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

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
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

template <typename T>
__global__ void __launch_bounds__(1024)
k_pass_engine(PassTables tb, int64_t item_begin, int64_t item_end)
{
    using V = typename Vec2<T>::type;
    extern __shared__ double smem_d[];
    V* const tileA = (V*)smem_d;
    V* const tileB = tileA + (1 << tb.tq_max);
    uint64_t* const hi_map = (uint64_t*)(tileB + (tb.with_grad ? (1 << tb.tq_max) : 0));
    double* const wpart = (double*)(hi_map + tb.hi_entries);  // [kMaxPassSlots][16 waves]
    double* const red = wpart + kMaxPassSlots * 16;
    const int nwaves = blockDim.x >> 6;

    for (int64_t item = item_begin + blockIdx.x; item < item_end; item += gridDim.x) {
        // decode: last segment whose first item is <= item
        int lo = 0, hi = tb.n_segs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tb.segs[mid].first <= item) lo = mid;
            else hi = mid - 1;
        }
        const FSeg sg = tb.segs[lo];
        struct {
            int circ, stage, tile;
        } it = {sg.circ, sg.stage, (int)(item - sg.first)};
        const FCirc cc = tb.circs[it.circ];
        V* const psi = (V*)cc.psi;
        V* const lam = (V*)cc.lam;
        const int tq = cc.tq;
        const uint32_t na = 1u << tq;
        const int nfwd = cc.n_pass;
        if (it.stage == nfwd) {
            // observable stage: contiguous chunk it.tile
            const uint64_t base = (uint64_t)it.tile << tq;
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
            if (threadIdx.x == 0) tb.e_part[cc.e_part_begin + it.tile] = s;
        } else {
            const bool fwd = it.stage < nfwd;
            const int pidx = fwd ? it.stage : (2 * nfwd - it.stage);  // reverse stage nfwd+1+r -> pass nfwd-1-r
            const FPass ps = tb.passes[cc.pass_begin + pidx];
            // tile base: insert zeros at Q into the tile index; hi_map deposits local bits >= c_bits
            uint64_t base = (uint64_t)it.tile;
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
                    lds_apply<T>(tileA, tb.ops[o], tb.coef, false, tq);
                    __syncthreads();
                }
                for (uint32_t l = threadIdx.x; l < na; l += blockDim.x)
                    stg<true>(psi + (hi_map[l >> cb] | (l & lomask)), tileA[l]);
            } else {
                for (uint32_t l = threadIdx.x; l < na; l += blockDim.x) {
                    const uint64_t g = hi_map[l >> cb] | (l & lomask);
                    tileA[l] = ldg<true>(psi + g);
                    tileB[l] = ldg<true>(lam + g);
                }
                __syncthreads();
                int nslot = 0;
                for (int o = ps.op_end - 1; o >= ps.op_begin; --o) {
                    const FOp op = tb.ops[o];
                    if (op.slot >= 0) {
                        const double c = wave_sum(lds_gen_inner<T>(tileA, tileB, op, tq));
                        if ((threadIdx.x & 63) == 0) wpart[nslot * 16 + (threadIdx.x >> 6)] = c;
                        ++nslot;
                        __syncthreads();  // every read of the tiles precedes the un-apply below
                    }
                    lds_apply<T>(tileA, op, tb.coef, true, tq);
                    lds_apply<T>(tileB, op, tb.coef, true, tq);
                    __syncthreads();
                }
                // per-op partials of this tile, in fixed wave order
                {
                    int k = 0;
                    for (int o = ps.op_end - 1; o >= ps.op_begin; --o) {
                        const FOp& op = tb.ops[o];
                        if (op.slot < 0) continue;
                        if (threadIdx.x == 0) {
                            double s = 0.0;
                            for (int w = 0; w < nwaves; ++w) s += wpart[k * 16 + w];
                            tb.g_part[cc.g_part_begin + (int64_t)op.slot * cc.n_tiles + it.tile] = s;
                        }
                        ++k;
                    }
                }
                for (uint32_t l = threadIdx.x; l < na; l += blockDim.x) {
                    const uint64_t g = hi_map[l >> cb] | (l & lomask);
                    stg<true>(psi + g, tileA[l]);
                    stg<true>(lam + g, tileB[l]);
                }
            }
        }
        __syncthreads();  // the LDS tiles are reused by the next item of this workgroup
    }
}

// One thread per op: gate coefficients from the parameters.
__global__ void k_pass_coef(const FCoefSpec* __restrict__ spec, int n, const double* __restrict__ params,
                            double* __restrict__ coef)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const FCoefSpec s = spec[i];
    double* c = coef + s.coef;
    const double th = s.pidx >= 0 ? params[s.pidx] : s.value;
    const double ch = cos(th / 2), sh = sin(th / 2);
    switch (s.gate) {
    case SV_RX: c[0] = ch; c[1] = 0; c[2] = 0; c[3] = -sh; c[4] = 0; c[5] = -sh; c[6] = ch; c[7] = 0; break;
    case SV_RY: c[0] = ch; c[1] = 0; c[2] = -sh; c[3] = 0; c[4] = sh; c[5] = 0; c[6] = ch; c[7] = 0; break;
    case SV_RZ: c[0] = ch; c[1] = -sh; c[2] = ch; c[3] = sh; break;
    case SV_PHASE: c[0] = cos(th); c[1] = sin(th); break;
    default:
        for (int k = 0; k < s.nfixed; ++k) c[k] = s.fixed[k];
        break;
    }
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

size_t pass_engine_lds_bytes(int tq_max, int hi_entries, int with_grad, int dtype)
{
    const size_t eb = dtype == SV_C128 ? 16 : 8;
    return eb * ((size_t)1 << tq_max) * (with_grad ? 2 : 1) + 8 * (size_t)hi_entries +
           8 * (size_t)kMaxPassSlots * 16 + 8 * 16;
}

hipError_t pass_engine_prepare(int dtype, size_t lds_bytes)
{
    if (dtype == SV_C128)
        return hipFuncSetAttribute((const void*)k_pass_engine<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds_bytes);
    return hipFuncSetAttribute((const void*)k_pass_engine<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds_bytes);
}

hipError_t launch_pass_level(const PassTables& tb, int dtype, int64_t item_begin, int64_t item_end, int threads,
                             size_t lds_bytes, hipStream_t s)
{
    const int64_t n = item_end - item_begin;
    if (n <= 0) return hipSuccess;
    const unsigned grid = (unsigned)(n < (1 << 30) ? n : (1 << 30));
    if (dtype == SV_C128)
        hipLaunchKernelGGL(k_pass_engine<double>, dim3(grid), dim3(threads), lds_bytes, s, tb, item_begin, item_end);
    else
        hipLaunchKernelGGL(k_pass_engine<float>, dim3(grid), dim3(threads), lds_bytes, s, tb, item_begin, item_end);
    return hipGetLastError();
}

hipError_t launch_pass_coef(const FCoefSpec* spec, int n, const double* params, double* coef, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pass_coef, dim3((n + 127) / 128), dim3(128), 0, s, spec, n, params, coef);
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
