// Dense k-qubit unitary (4 <= k <= 6) on the matrix cores: the fused dense
// block the gate-specific kernels are set against (Sec. 2 applies a gate's
// small logic matrix to the amplitude groups its qubits select; here one
// 2^k x 2^k matrix stands for a run of gates on k qubits).
//
// The amplitudes of group g form a row of 2^(k+1) reals (re, im interleaved
// in matrix-index order).  The output row is that row times the real form of
// U (dense_real_form), so a block of 16 groups is a 16 x 2^(k+1) by
// 2^(k+1) x 2^(k+1) real product: 16x16x4 MFMA steps, FP64 for complex128
// and FP32 for complex64.  Per amplitude that is 8 * 2^k flops for 32 (or
// 16) bytes moved: HBM-bound up to k = 5, matrix-core-bound at k = 6
// (complex128).
//
// Operand layouts (16x16x4, one wavefront): lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; accumulator value r of lane l is D[l / 16 + 4 r][l % 16]
// in FP64 and D[4 (l / 16) + r][l % 16] in FP32.
#include <algorithm>

#include "sv.h"
#include "sv_dense.h"

namespace svk {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

template <typename T>
struct DenseAcc;
template <>
struct DenseAcc<double> {
    using type = dbl4;
};
template <>
struct DenseAcc<float> {
    using type = flt4;
};

__device__ __forceinline__ dbl4 mfma16x16x4(double a, double b, dbl4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ flt4 mfma16x16x4(float a, float b, flt4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Accumulator row held by lane l's value r.
template <typename T>
__device__ __forceinline__ int acc_row(int l, int r)
{
    if constexpr (sizeof(T) == 8) return (l >> 4) + 4 * r;
    else return 4 * (l >> 4) + r;
}

// Group index -> amplitude index with zeros at the (ascending) target bits.
template <int K>
__device__ __forceinline__ uint64_t group_base(uint64_t g, const DenseSpec& sp)
{
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int q = sp.qs_sorted[j];
        const uint64_t lo = g & ((1ull << q) - 1ull);
        g = ((g >> q) << (q + 1)) | lo;
    }
    return g;
}

template <typename T, int K>
__global__ void __launch_bounds__(512) k_dense(T* __restrict__ psi, const T* __restrict__ B, DenseSpec sp)
{
    constexpr int N2 = 2 << K;   // reals per group
    constexpr int KS = N2 / 4;   // MFMA steps along the input
    constexpr int NT = N2 / 16;  // 16-column output tiles
    constexpr int CH = KS < 8 ? KS : 8;  // MFMA steps per chunk of input loads
    using Acc = typename DenseAcc<T>::type;
    extern __shared__ double dense_smem[];
    T* const Bl = (T*)dense_smem;
    __shared__ uint64_t dep[1 << K];
    for (int i = threadIdx.x; i < N2 * N2; i += blockDim.x) Bl[i] = B[i];
    for (int i = threadIdx.x; i < (1 << K); i += blockDim.x) dep[i] = sp.dep[i];
    __syncthreads();

    const int l = threadIdx.x & 63;
    const int wpg = blockDim.x >> 6;
    const int64_t nblk = (sp.groups + 15) >> 4;
    for (int64_t blk = (int64_t)blockIdx.x * wpg + (threadIdx.x >> 6); blk < nblk; blk += (int64_t)gridDim.x * wpg) {
        const int64_t g = blk * 16 + (l & 15);
        const bool valid = g < sp.groups;  // the last block of a small state is partial
        const uint64_t base = group_base<K>(valid ? (uint64_t)g : 0ull, sp);
        const T* const row = psi + 2 * base + ((l >> 4) & 1);  // this lane's component
        // lane l reads input real m = 4 ks + l / 16: amplitude 2 ks + l / 32
        auto load_chunk = [&](int kc, T* a) {
#pragma unroll
            for (int i = 0; i < CH; ++i) a[i] = valid ? row[2 * dep[2 * (kc + i) + (l >> 5)]] : T(0);
        };
        Acc acc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = Acc{0, 0, 0, 0};
        T a_cur[CH], a_nxt[CH];
        load_chunk(0, a_cur);
#pragma unroll 1
        for (int kc = 0; kc < KS; kc += CH) {
            if (kc + CH < KS) load_chunk(kc + CH, a_nxt);  // in flight during this chunk's products
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const T* const brow = Bl + (4 * (kc + i) + (l >> 4)) * N2 + (l & 15);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[nt] = mfma16x16x4(a_cur[i], brow[16 * nt], acc[nt]);
            }
#pragma unroll
            for (int i = 0; i < CH; ++i) a_cur[i] = a_nxt[i];
        }
        // every amplitude of this block was read above (the products depend
        // on all of them), and no other wavefront touches these groups
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t gi = blk * 16 + acc_row<T>(l, r);
            if (gi >= sp.groups) continue;
            const uint64_t bi = group_base<K>((uint64_t)gi, sp);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int m = 16 * nt + (l & 15);
                psi[2 * (bi | dep[m >> 1]) + (m & 1)] = acc[nt][r];
            }
        }
    }
}

void dense_real_form(const double* U, int k, double* B)
{
    const int M = 1 << k, N2 = 2 * M;
    for (int r = 0; r < M; ++r)
        for (int c = 0; c < M; ++c) {
            const double ur = U[2 * (r * M + c)], ui = U[2 * (r * M + c) + 1];
            B[(2 * c) * N2 + 2 * r] = ur;
            B[(2 * c + 1) * N2 + 2 * r] = -ui;
            B[(2 * c) * N2 + 2 * r + 1] = ui;
            B[(2 * c + 1) * N2 + 2 * r + 1] = ur;
        }
}

size_t dense_lds_bytes(int k, int dtype)
{
    const size_t n2 = (size_t)2 << k;
    return n2 * n2 * (dtype == SV_C128 ? sizeof(double) : sizeof(float));
}

template <typename T, int K>
static hipError_t launch_k(T* psi, const T* B, const DenseSpec& sp, hipStream_t s)
{
    // k = 6 holds a 128 KiB (complex128) real form per workgroup: one
    // workgroup per CU, so it gets 8 wavefronts; smaller k get 4
    const int threads = K == 6 ? 512 : 256;
    const size_t lds = dense_lds_bytes(K, sizeof(T) == 8 ? SV_C128 : SV_C64);
    static bool attr_set = false;
    if (!attr_set) {
        const hipError_t e =
            hipFuncSetAttribute((const void*)k_dense<T, K>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int64_t nblk = (sp.groups + 15) / 16;
    const int64_t wpg = threads / 64;
    const int64_t grid = std::min<int64_t>((nblk + wpg - 1) / wpg, 256 * 16);
    hipLaunchKernelGGL((k_dense<T, K>), dim3((unsigned)grid), dim3(threads), lds, s, psi, B, sp);
    return hipGetLastError();
}

hipError_t launch_dense(void* psi, int dtype, const void* B, const DenseSpec& sp, hipStream_t s)
{
    if (sp.groups <= 0 || sp.k < kDenseMinK || sp.k > kDenseMaxK) return hipErrorInvalidValue;
    if (dtype == SV_C128) {
        double* p = (double*)psi;
        const double* b = (const double*)B;
        switch (sp.k) {
        case 4: return launch_k<double, 4>(p, b, sp, s);
        case 5: return launch_k<double, 5>(p, b, sp, s);
        default: return launch_k<double, 6>(p, b, sp, s);
        }
    }
    float* p = (float*)psi;
    const float* b = (const float*)B;
    switch (sp.k) {
    case 4: return launch_k<float, 4>(p, b, sp, s);
    case 5: return launch_k<float, 5>(p, b, sp, s);
    default: return launch_k<float, 6>(p, b, sp, s);
    }
}

}  // namespace svk
