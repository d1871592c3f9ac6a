// k_reduce.hip -- measurement reductions for gfx950.
//
// Expectation values of Pauli strings and of Pauli sums (the "measurement
// processes" routines of Sec. 2; Listing 1 takes <H> of a Hamiltonian).
// For P with X/Y positions f = xmask and Z/Y positions zmask:
//   P|x> = i^{nY} (-1)^{popcount(x & zmask)} |x ^ f>,
//   <psi|P|psi> = sum_x conj(psi[x ^ f]) i^{nY} (-1)^{pc(x & zmask)} psi[x].
// For f = 0 this is sum_x |psi_x|^2 (-1)^{pc(x & zmask)}.  For f != 0 the
// terms of x and x ^ f are complex conjugates (P is Hermitian), so only x with
// bit p = 0 (p = top bit of f) is visited and the term counted as 2 Re(.):
// every amplitude is read exactly once.
//
// Accumulation: complex64 loads are widened to fp64 before any product
// (expectations); the norm of a complex64 state sums one chunk per thread
// in fp32 and everything above that in fp64.  Stage 1 writes one fp64
// partial per block of a fixed grid, stage 2 sums partials in fixed order:
// repeated calls give bit-identical results.
#include "sv_core.h"

namespace svk {

// Deterministic block sum (wavefront butterfly, then waves in order).
// Valid on thread 0.
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double sm[kReduceThreads / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sm[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sm[w];
    }
    return s;
}

static int reduce_grid(uint64_t n_items)
{
    uint64_t per = (uint64_t)kReduceThreads * 4;
    uint64_t nb = (n_items + per - 1) / per;
    if (nb < 1) nb = 1;
    if (nb > (uint64_t)kReduceBlocks) nb = kReduceBlocks;
    return (int)nb;
}

template <typename T>
__global__ void __launch_bounds__(kReduceThreads)
k_norm_partial(const typename Vec2<T>::type* __restrict__ psi, uint64_t n, double* __restrict__ partials)
{
    using V = typename Vec2<T>::type;
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 4;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x * 4 + threadIdx.x; i0 < n + threadIdx.x; i0 += stride) {
        V a[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t i = i0 + (uint64_t)j * blockDim.x;
            if (i < n) a[j] = psi[i];
            else { a[j].x = T(0); a[j].y = T(0); }
        }
        T loc = T(0);  // fp32 per-chunk sum for complex64, fp64 for complex128
#pragma unroll
        for (int j = 0; j < 4; ++j) loc += a[j].x * a[j].x + a[j].y * a[j].y;
        acc += (double)loc;
    }
    const double s = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <typename T>
__global__ void __launch_bounds__(kReduceThreads)
k_pauli_partial(const typename Vec2<T>::type* __restrict__ psi, GroupSpec gs, uint64_t xmask, uint64_t zmask,
                int ny, double coeff, double* __restrict__ partials)
{
    using V = typename Vec2<T>::type;
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 4;
    const uint64_t n = gs.n_groups;
    for (uint64_t g0 = (uint64_t)blockIdx.x * blockDim.x * 4 + threadIdx.x; g0 < n + threadIdx.x; g0 += stride) {
        uint64_t x[4];
        V a[4], b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t g = g0 + (uint64_t)j * blockDim.x;
            if (g < n) {
                x[j] = group_base(g, gs);
                a[j] = psi[x[j]];
                if (xmask) b[j] = psi[x[j] ^ xmask];
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t g = g0 + (uint64_t)j * blockDim.x;
            if (g < n) {
                const double sgn = (__popcll(x[j] & zmask) & 1) ? -1.0 : 1.0;
                const double ar = (double)a[j].x, ai = (double)a[j].y;
                if (xmask == 0) {
                    acc += sgn * (ar * ar + ai * ai);
                } else {
                    const double br = (double)b[j].x, bi = (double)b[j].y;
                    // w = conj(b) * a
                    const double wr = br * ar + bi * ai;
                    const double wi = br * ai - bi * ar;
                    // Re(i^ny * w)
                    double re;
                    switch (ny & 3) {
                    case 0: re = wr; break;
                    case 1: re = -wi; break;
                    case 2: re = -wr; break;
                    default: re = wi; break;
                    }
                    acc += 2.0 * sgn * re;
                }
            }
        }
    }
    const double s = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = coeff * s;
}

struct DiagTerms {
    int32_t nterms;
    double c[kDiagTermsPerPass];
    uint64_t z[kDiagTermsPerPass];
};

// kind 1: o(x) = n - 2 pc(x)                           (sum_i Z_i)
// kind 2: o(x) = (n-1) - 2 pc((x ^ (x>>1)) & (2^(n-1)-1))  (sum_i Z_i Z_{i+1})
// kind 0: o(x) = sum_k c_k (-1)^{pc(x & z_k)}
template <typename T>
__global__ void __launch_bounds__(kReduceThreads)
k_diag_obs_partial(const typename Vec2<T>::type* __restrict__ psi, uint64_t n_amps, int nq, int kind,
                   double coeff, DiagTerms terms, double* __restrict__ partials)
{
    using V = typename Vec2<T>::type;
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 4;
    const uint64_t zzmask = nq > 1 ? ((1ull << (nq - 1)) - 1ull) : 0ull;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x * 4 + threadIdx.x; i0 < n_amps + threadIdx.x;
         i0 += stride) {
        V a[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t i = i0 + (uint64_t)j * blockDim.x;
            if (i < n_amps) a[j] = psi[i];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t x = i0 + (uint64_t)j * blockDim.x;
            if (x < n_amps) {
                double o;
                if (kind == 1) {
                    o = (double)(nq - 2 * (int)__popcll(x));
                } else if (kind == 2) {
                    o = (double)((nq - 1) - 2 * (int)__popcll((x ^ (x >> 1)) & zzmask));
                } else {
                    o = 0.0;
                    for (int k = 0; k < terms.nterms; ++k)
                        o += (__popcll(x & terms.z[k]) & 1) ? -terms.c[k] : terms.c[k];
                }
                const double ar = (double)a[j].x, ai = (double)a[j].y;
                acc += o * (ar * ar + ai * ai);
            }
        }
    }
    const double s = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = coeff * s;
}

// out[seg] = scale[seg] * sum of partials[seg * seg_len .. +seg_len) (fixed order);
// one block per segment.
__global__ void __launch_bounds__(kReduceThreads)
k_sum_segments(const double* __restrict__ partials, int seg_len, const double* __restrict__ scale,
               double* __restrict__ out)
{
    const double* p = partials + (size_t)blockIdx.x * seg_len;
    double acc = 0.0;
    for (int i = threadIdx.x; i < seg_len; i += blockDim.x) acc += p[i];
    const double s = block_sum(acc);
    if (threadIdx.x == 0) out[blockIdx.x] = scale ? scale[blockIdx.x] * s : s;
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
template <typename T>
hipError_t launch_norm_partial(const void* psi, uint64_t n_amps, double* partials, hipStream_t s)
{
    using V = typename Vec2<T>::type;
    const int nb = reduce_grid(n_amps);
    hipLaunchKernelGGL((k_norm_partial<T>), dim3(nb), dim3(kReduceThreads), 0, s, (const V*)psi, n_amps,
                       partials);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pauli_partial(const void* psi, int n, uint64_t xmask, uint64_t zmask, int ny, double coeff,
                                double* partials, hipStream_t s)
{
    using V = typename Vec2<T>::type;
    GroupSpec gs{};
    if (xmask == 0) {
        gs.n_groups = 1ull << n;
        gs.nins = 0;
    } else {
        gs.n_groups = 1ull << (n - 1);
        gs.nins = 1;
        gs.pos[0] = 63 - __builtin_clzll(xmask);
    }
    gs.set_mask = 0;
    const int nb = reduce_grid(gs.n_groups);
    hipLaunchKernelGGL((k_pauli_partial<T>), dim3(nb), dim3(kReduceThreads), 0, s, (const V*)psi, gs, xmask, zmask,
                       ny, coeff, partials);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_diag_obs_partial(const void* psi, int n, int kind, double coeff, const double* hcoef,
                                   const uint64_t* hz, int nterms, double* partials, hipStream_t s)
{
    using V = typename Vec2<T>::type;
    DiagTerms terms{};
    if (nterms > kDiagTermsPerPass) return hipErrorInvalidValue;
    terms.nterms = kind == 0 ? nterms : 0;
    for (int k = 0; k < terms.nterms; ++k) {
        terms.c[k] = hcoef[k];
        terms.z[k] = hz[k];
    }
    const uint64_t n_amps = 1ull << n;
    const int nb = reduce_grid(n_amps);
    hipLaunchKernelGGL((k_diag_obs_partial<T>), dim3(nb), dim3(kReduceThreads), 0, s, (const V*)psi, n_amps, n,
                       kind, coeff, terms, partials);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double* partials, int count, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_segments, dim3(1), dim3(kReduceThreads), 0, s, partials, count, (const double*)nullptr,
                       out);
    return hipGetLastError();
}

hipError_t launch_sum_segments(const double* partials, int seg_len, int n_seg, const double* scale, double* out,
                               hipStream_t s)
{
    if (n_seg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_segments, dim3(n_seg), dim3(kReduceThreads), 0, s, partials, seg_len, scale, out);
    return hipGetLastError();
}

int reduce_blocks_for(uint64_t n_items) { return reduce_grid(n_items); }

template hipError_t launch_norm_partial<double>(const void*, uint64_t, double*, hipStream_t);
template hipError_t launch_norm_partial<float>(const void*, uint64_t, double*, hipStream_t);
template hipError_t launch_pauli_partial<double>(const void*, int, uint64_t, uint64_t, int, double, double*,
                                                 hipStream_t);
template hipError_t launch_pauli_partial<float>(const void*, int, uint64_t, uint64_t, int, double, double*,
                                                hipStream_t);
template hipError_t launch_diag_obs_partial<double>(const void*, int, int, double, const double*, const uint64_t*,
                                                    int, double*, hipStream_t);
template hipError_t launch_diag_obs_partial<float>(const void*, int, int, double, const double*, const uint64_t*,
                                                   int, double*, hipStream_t);

}  // namespace svk
