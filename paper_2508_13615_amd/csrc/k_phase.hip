// A run of diagonal gates in one pass over the state.  Diagonal gates commute
// and only rescale amplitudes (Sec. 2: a Z-type gate changes the amplitudes
// whose target bit is 1), so a run of them is one phase per amplitude: the
// sum of the angles of the terms whose bits the index contains.  One read and
// one write of each touched amplitude replaces one per gate (the QFT's
// controlled phases on a target become one half-touch pass).
//
// Angles are carried in half-turns and evaluated with sincospi, so phases at
// multiples of pi/2 (Z, S, CZ) come out exactly.
#include <algorithm>

#include "sv.h"
#include "sv_phase.h"

namespace svk {

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

template <typename T>
__global__ void __launch_bounds__(256) k_phase_run(typename PhaseCplx<T>::type* __restrict__ psi, PhaseRun pr)
{
    using V = typename PhaseCplx<T>::type;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < pr.groups; g += step) {
        uint64_t x = (uint64_t)g;
        for (int j = 0; j < pr.n_common; ++j) {
            const int q = pr.common_pos[j];
            const uint64_t lo = x & ((1ull << q) - 1ull);
            x = ((x >> q) << (q + 1)) | (1ull << q) | lo;
        }
        T th = T(0);
        for (int t = 0; t < pr.n_terms; ++t)
            if ((x & pr.mask[t]) == pr.mask[t]) th += (T)pr.turns[t];
        T sn, cs;
        if constexpr (sizeof(T) == 8) sincospi(th, &sn, &cs);
        else sincospif(th, &sn, &cs);
        const V a = psi[x];
        psi[x] = V{cs * a.x - sn * a.y, cs * a.y + sn * a.x};
    }
}

hipError_t launch_phase_run(void* psi, int dtype, const PhaseRun& pr, hipStream_t s)
{
    if (pr.groups <= 0 || pr.n_terms < 1 || pr.n_terms > kMaxPhaseTerms) return hipErrorInvalidValue;
    const int threads = 256;
    const int64_t blocks = std::min<int64_t>((pr.groups + threads - 1) / threads, 256 * 64);
    if (dtype == SV_C128)
        hipLaunchKernelGGL(k_phase_run<double>, dim3((unsigned)blocks), dim3(threads), 0, s, (double2*)psi, pr);
    else hipLaunchKernelGGL(k_phase_run<float>, dim3((unsigned)blocks), dim3(threads), 0, s, (float2*)psi, pr);
    return hipGetLastError();
}

}  // namespace svk
