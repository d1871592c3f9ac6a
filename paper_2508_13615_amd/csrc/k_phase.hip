// A run of diagonal gates in one pass over the state.  Diagonal gates commute
// and only rescale amplitudes (Sec. 2: a Z-type gate changes the amplitudes
// whose target bit is 1), so a run of them is one phase per amplitude: the
// sum of the angles of the terms whose bits the index contains.  One read and
// one write of each touched amplitude replaces one per gate (the QFT's
// controlled phases on a target become one half-touch pass).
//
// Angles are carried in half-turns and evaluated with sincospi, so phases at
// multiples of pi/2 (Z, S, CZ) come out exactly.  Every pass streams whole
// amplitudes once: loads and stores are non-temporal.
#include <algorithm>

#include "sv.h"
#include "sv_core.h"
#include "sv_phase.h"

namespace svk {

// One workgroup per chunk of work (a grid-stride loop only past the launch
// limits: 2^30 blocks, 2^32 threads): measured faster than a capped,
// persistent grid for these streaming passes.
static int64_t phase_grid(int64_t blocks, int threads)
{
    const int64_t lim = std::min<int64_t>(1ll << 30, 0xffffffffll / threads);
    return blocks < 1 ? 1 : (blocks > lim ? lim : blocks);
}

template <typename T>
struct PhaseCplx;
template <>
struct PhaseCplx<double> {
    using type = double2;
};
template <>
struct PhaseCplx<float> {
    using type = float2;
};

// The run's terms, staged in LDS once per workgroup: the per-amplitude loop
// then reads them without a dependent scalar load per term.
struct PhaseLds {
    uint64_t mask[kMaxPhaseTerms];
    double turns[kMaxPhaseTerms];
};

__device__ __forceinline__ void stage_terms(const PhaseRun& pr, PhaseLds& sm)
{
    for (int t = threadIdx.x; t < pr.n_terms; t += blockDim.x) {
        sm.mask[t] = pr.mask[t];
        sm.turns[t] = pr.turns[t];
    }
    __syncthreads();
}

// Sum of the angles (half-turns) of terms [begin, end) whose bits x holds.
template <typename T>
__device__ __forceinline__ T run_turns(uint64_t x, const PhaseLds& sm, int begin, int end)
{
    T th = T(0);
#pragma unroll 4
    for (int t = begin; t < end; ++t) {
        const uint64_t m = sm.mask[t];
        const T a = (T)sm.turns[t];
        th += (x & m) == m ? a : T(0);
    }
    return th;
}

template <typename T>
__global__ void __launch_bounds__(256) k_phase_run(typename PhaseCplx<T>::type* __restrict__ psi, PhaseRun pr)
{
    using V = typename PhaseCplx<T>::type;
    __shared__ PhaseLds sm;
    stage_terms(pr, sm);
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < pr.groups; g += step) {
        uint64_t x = (uint64_t)g;
        for (int j = 0; j < pr.n_common; ++j) {
            const int q = pr.common_pos[j];
            const uint64_t lo = x & ((1ull << q) - 1ull);
            x = ((x >> q) << (q + 1)) | (1ull << q) | lo;
        }
        const T th = run_turns<T>(x, sm, 0, pr.n_terms);
        T sn, cs;
        if constexpr (sizeof(T) == 8) sincospi(th, &sn, &cs);
        else sincospif(th, &sn, &cs);
        const V a = ldg<true>(psi + x);
        stg<true>(psi + x, V{cs * a.x - sn * a.y, cs * a.y + sn * a.x});
    }
}

// A one-target gate u (row-major 2x2, interleaved) on qubit t followed by a
// phase run, in one pass over the pairs of amplitudes that differ in bit t.
// The first n_with terms hold bit t: only the partner with bit t set can
// contain them.  The others hold neither or both partners alike, so each
// term is tested once; with none of them the bit-0 partner keeps its phase.

template <typename T>
__global__ void __launch_bounds__(256) k_pair_phase_run(typename PhaseCplx<T>::type* __restrict__ psi, int tq,
                                                        PairCoef u, PhaseRun pr, int n_with)
{
    using V = typename PhaseCplx<T>::type;
    const T u0r = (T)u.m[0], u0i = (T)u.m[1], u1r = (T)u.m[2], u1i = (T)u.m[3];
    const T u2r = (T)u.m[4], u2i = (T)u.m[5], u3r = (T)u.m[6], u3i = (T)u.m[7];
    __shared__ PhaseLds sm;
    stage_terms(pr, sm);
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < pr.groups; g += step) {
        const uint64_t lo = (uint64_t)g & ((1ull << tq) - 1ull);
        const uint64_t x0 = (((uint64_t)g >> tq) << (tq + 1)) | lo, x1 = x0 | (1ull << tq);
        const V a = ldg<true>(psi + x0), b = ldg<true>(psi + x1);
        const V p{u0r * a.x - u0i * a.y + u1r * b.x - u1i * b.y, u0r * a.y + u0i * a.x + u1r * b.y + u1i * b.x};
        const V q{u2r * a.x - u2i * a.y + u3r * b.x - u3i * b.y, u2r * a.y + u2i * a.x + u3r * b.y + u3i * b.x};
        const T th_both = run_turns<T>(x0, sm, n_with, pr.n_terms);
        const T th1 = th_both + run_turns<T>(x1, sm, 0, n_with);
        T s1, c1;
        if constexpr (sizeof(T) == 8) sincospi(th1, &s1, &c1);
        else sincospif(th1, &s1, &c1);
        stg<true>(psi + x1, V{c1 * q.x - s1 * q.y, c1 * q.y + s1 * q.x});
        if (n_with == pr.n_terms) {  // uniform: no term can hold the bit-0 partner
            stg<true>(psi + x0, p);
        } else {
            T s0, c0;
            if constexpr (sizeof(T) == 8) sincospi(th_both, &s0, &c0);
            else sincospif(th_both, &s0, &c0);
            stg<true>(psi + x0, V{c0 * p.x - s0 * p.y, c0 * p.y + s0 * p.x});
        }
    }
}

hipError_t launch_pair_phase_run(void* psi, int dtype, int t, const PairCoef& u, const PhaseRun& pr, int n_with,
                                 hipStream_t s)
{
    if (pr.groups <= 0 || pr.n_terms < 1 || pr.n_terms > kMaxPhaseTerms || pr.n_common != 0 || n_with < 0 ||
        n_with > pr.n_terms)
        return hipErrorInvalidValue;
    const int threads = 256;
    const int64_t blocks = phase_grid((pr.groups + threads - 1) / threads, threads);
    if (dtype == SV_C128)
        hipLaunchKernelGGL(k_pair_phase_run<double>, dim3((unsigned)blocks), dim3(threads), 0, s, (double2*)psi, t, u,
                           pr, n_with);
    else
        hipLaunchKernelGGL(k_pair_phase_run<float>, dim3((unsigned)blocks), dim3(threads), 0, s, (float2*)psi, t, u, pr,
                           n_with);
    return hipGetLastError();
}

// The same when every term holds bit t and at most one other bit (the QFT's
// controlled phases): the 1-side phase is exp(i pi sum_b turns_of_bit[b] x_b),
// a product over the index's bytes.  One small kernel tabulates, per byte, the
// 256 phases of that byte's bits; a pair then takes one (cached) table entry
// per byte instead of a term loop and a sincospi.
template <typename T>
__global__ void __launch_bounds__(256) k_linear_tables(typename PhaseCplx<T>::type* __restrict__ tab, LinearPhase lp)
{
    using V = typename PhaseCplx<T>::type;
    for (int e = threadIdx.x; e < lp.n_bytes * 256; e += blockDim.x) {
        const int k = e >> 8, v = e & 255;
        double th = k == 0 ? lp.turns_const : 0.0;
        for (int b = 0; b < 8; ++b)
            if ((v >> b) & 1) th += lp.turns_of_bit[8 * k + b];
        double sn, cs;
        sincospi(th, &sn, &cs);
        tab[e] = V{(T)cs, (T)sn};
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_pair_linear_phase(typename PhaseCplx<T>::type* __restrict__ psi, int tq,
                                                           PairCoef u, const typename PhaseCplx<T>::type* __restrict__ tab,
                                                           int n_bytes, int64_t groups)
{
    using V = typename PhaseCplx<T>::type;
    const T u0r = (T)u.m[0], u0i = (T)u.m[1], u1r = (T)u.m[2], u1i = (T)u.m[3];
    const T u2r = (T)u.m[4], u2i = (T)u.m[5], u3r = (T)u.m[6], u3i = (T)u.m[7];
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < groups; g += step) {
        const uint64_t lo = (uint64_t)g & ((1ull << tq) - 1ull);
        const uint64_t x0 = (((uint64_t)g >> tq) << (tq + 1)) | lo, x1 = x0 | (1ull << tq);
        const V a = ldg<true>(psi + x0), b = ldg<true>(psi + x1);
        const V p{u0r * a.x - u0i * a.y + u1r * b.x - u1i * b.y, u0r * a.y + u0i * a.x + u1r * b.y + u1i * b.x};
        V q{u2r * a.x - u2i * a.y + u3r * b.x - u3i * b.y, u2r * a.y + u2i * a.x + u3r * b.y + u3i * b.x};
        for (int k = 0; k < n_bytes; ++k) {
            const V z = tab[256 * k + ((x1 >> (8 * k)) & 255u)];
            q = V{z.x * q.x - z.y * q.y, z.x * q.y + z.y * q.x};
        }
        stg<true>(psi + x0, p);
        stg<true>(psi + x1, q);
    }
}

hipError_t launch_pair_linear_phase(void* psi, int dtype, int t, const PairCoef& u, const LinearPhase& lp,
                                    int64_t groups, void* table, hipStream_t s)
{
    if (groups <= 0 || lp.n_bytes < 1 || lp.n_bytes > kLinearPhaseBytes || !table) return hipErrorInvalidValue;
    const int threads = 256;
    const int64_t blocks = phase_grid((groups + threads - 1) / threads, threads);
    if (dtype == SV_C128) {
        hipLaunchKernelGGL(k_linear_tables<double>, dim3(1), dim3(256), 0, s, (double2*)table, lp);
        hipLaunchKernelGGL(k_pair_linear_phase<double>, dim3((unsigned)blocks), dim3(threads), 0, s, (double2*)psi, t,
                           u, (const double2*)table, lp.n_bytes, groups);
    } else {
        hipLaunchKernelGGL(k_linear_tables<float>, dim3(1), dim3(256), 0, s, (float2*)table, lp);
        hipLaunchKernelGGL(k_pair_linear_phase<float>, dim3((unsigned)blocks), dim3(threads), 0, s, (float2*)psi, t, u,
                           (const float2*)table, lp.n_bytes, groups);
    }
    return hipGetLastError();
}

hipError_t launch_phase_run(void* psi, int dtype, const PhaseRun& pr, hipStream_t s)
{
    if (pr.groups <= 0 || pr.n_terms < 1 || pr.n_terms > kMaxPhaseTerms) return hipErrorInvalidValue;
    const int threads = 256;
    const int64_t blocks = phase_grid((pr.groups + threads - 1) / threads, threads);
    if (dtype == SV_C128)
        hipLaunchKernelGGL(k_phase_run<double>, dim3((unsigned)blocks), dim3(threads), 0, s, (double2*)psi, pr);
    else hipLaunchKernelGGL(k_phase_run<float>, dim3((unsigned)blocks), dim3(threads), 0, s, (float2*)psi, pr);
    return hipGetLastError();
}

}  // namespace svk
