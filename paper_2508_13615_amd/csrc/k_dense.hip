// Dense k-qubit unitary (4 <= k <= 6) on the matrix cores: the fused dense
// block the gate-specific kernels are set against (Sec. 2 applies a gate's
// small logic matrix to the amplitude groups its qubits select; here one
// 2^k x 2^k matrix stands for a run of gates on k qubits).
//
// The amplitudes of group g form a row of 2^(k+1) reals.  The output row is
// that row times a real form of U (dense_real_form), so a block of 16 groups
// is a 16 x 2^(k+1) by 2^(k+1) x 2^(k+1) real product: 16x16x4 MFMA steps,
// FP64 for complex128 and FP32 for complex64.  Per amplitude that is
// 8 * 2^k flops for 32 (or 16) bytes moved: HBM-bound up to k = 5,
// matrix-core-bound at k = 6 (complex128).
//
// Operand layouts (16x16x4, one wavefront): lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; accumulator value r of lane l is D[l / 16 + 4 r][l % 16]
// in FP64 and D[4 (l / 16) + r][l % 16] in FP32.  The order of the reals is
// free (it is the real form's row and column order), and is chosen so that
// every access is a whole amplitude: at steps 2j and 2j + 1 the lanes with
// l / 16 = kk take the real and the imaginary part of amplitude 4 j + kk
// (one 16- or 8-byte load for two steps), and output tiles 2t and 2t + 1 hold
// the real and the imaginary parts of amplitudes 16 t .. 16 t + 15 (one store
// per amplitude).  A load instruction takes 4 consecutive amplitudes of each
// of 16 groups, so a line is often completed by the next instruction: plain
// (cached) accesses, which measured faster here than non-temporal ones.
#include <algorithm>

#include "sv.h"
#include "sv_core.h"
#include "sv_dense.h"

namespace svk {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Cplx;
template <>
struct Cplx<double> {
    using type = double2;
};
template <>
struct Cplx<float> {
    using type = float2;
};

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
    using V = typename Cplx<T>::type;
    extern __shared__ double dense_smem[];
    T* const Bl = (T*)dense_smem;
    __shared__ uint64_t dep[1 << K];
    for (int i = threadIdx.x; i < N2 * N2; i += blockDim.x) Bl[i] = B[i];
    for (int i = threadIdx.x; i < (1 << K); i += blockDim.x) dep[i] = sp.dep[i];
    __syncthreads();

    const int l = threadIdx.x & 63;
    const int wpg = blockDim.x >> 6;
    const int64_t nblk = (sp.groups + 15) >> 4;
    // this lane's group row of block b (the last block of a small state is
    // partial: rows past the groups read zeros and are not stored)
    auto row_of = [&](int64_t b, bool& valid) {
        const int64_t g = b * 16 + (l & 15);
        valid = g < sp.groups;
        return (const V*)psi + group_base<K>(valid ? (uint64_t)g : 0ull, sp);
    };
    // chunk of CH steps = CH / 2 amplitudes per lane: 4 j + l / 16 for step pair j
    auto load_chunk = [&](const V* row, bool valid, int kc, V* a) {
#pragma unroll
        for (int i = 0; i < CH / 2; ++i) {
            const int j = kc / 2 + i;
            a[i] = valid ? row[dep[4 * j + (l >> 4)]] : V{T(0), T(0)};
        }
    };
    // Teams of sp.team consecutive workgroups each own a contiguous run of
    // sp.per_team blocks and walk it with a stride of the team's wavefronts
    // (team = 1: a run per workgroup; team = grid: one grid-stride walk).
    const int64_t wg = (int64_t)block_slot(blockIdx.x, gridDim.x, sp.order);
    const int64_t team = wg / sp.team, local = wg % sp.team;
    int64_t blk = team * sp.per_team + local * wpg + (threadIdx.x >> 6);
    const int64_t end = std::min<int64_t>(nblk, (team + 1) * sp.per_team);
    const int64_t step = (int64_t)sp.team * wpg;
    V a_cur[CH / 2], a_nxt[CH / 2];
    bool valid = false;
    const V* row = nullptr;
    if (blk < end) {
        row = row_of(blk, valid);
        load_chunk(row, valid, 0, a_cur);
    }
    for (; blk < end; blk += step) {
        const int64_t nb = blk + step;
        bool nvalid = false;
        const V* const nrow = nb < end ? row_of(nb, nvalid) : nullptr;
        Acc acc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = Acc{0, 0, 0, 0};
#pragma unroll 1
        for (int kc = 0; kc < KS; kc += CH) {
            // in flight during this chunk's products: the next chunk, or the
            // first chunk of this wavefront's next block (other groups)
            if (kc + CH < KS) load_chunk(row, valid, kc + CH, a_nxt);
            else if (nb < end) load_chunk(nrow, nvalid, 0, a_nxt);
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const T* const brow = Bl + (4 * (kc + i) + (l >> 4)) * N2 + (l & 15);
                const T av = (i & 1) ? a_cur[i >> 1].y : a_cur[i >> 1].x;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[nt] = mfma16x16x4(av, brow[16 * nt], acc[nt]);
            }
#pragma unroll
            for (int i = 0; i < CH / 2; ++i) a_cur[i] = a_nxt[i];
        }
        // every amplitude of this block was read above (the products depend
        // on all of them), and no other wavefront touches these groups
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t gi = blk * 16 + acc_row<T>(l, r);
            if (gi >= sp.groups) continue;
            V* const orow = (V*)psi + group_base<K>((uint64_t)gi, sp);
#pragma unroll
            for (int t = 0; t < NT / 2; ++t) orow[dep[16 * t + (l & 15)]] = V{acc[2 * t][r], acc[2 * t + 1][r]};
        }
        row = nrow;
        valid = nvalid;
    }
}

// Row of the real form that holds component p of input amplitude c, and
// column that holds component q of output amplitude r (the kernel's order).
static int in_pos(int c, int p) { return 4 * (2 * (c >> 2) + p) + (c & 3); }
static int out_pos(int r, int q) { return 16 * (2 * (r >> 4) + q) + (r & 15); }

void dense_real_form(const double* U, int k, double* B)
{
    const int M = 1 << k, N2 = 2 * M;
    for (int r = 0; r < M; ++r)
        for (int c = 0; c < M; ++c) {
            const double ur = U[2 * (r * M + c)], ui = U[2 * (r * M + c) + 1];
            B[in_pos(c, 0) * N2 + out_pos(r, 0)] = ur;   // re(out) += ur re(in)
            B[in_pos(c, 1) * N2 + out_pos(r, 0)] = -ui;  // re(out) -= ui im(in)
            B[in_pos(c, 0) * N2 + out_pos(r, 1)] = ui;   // im(out) += ui re(in)
            B[in_pos(c, 1) * N2 + out_pos(r, 1)] = ur;   // im(out) += ur im(in)
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
    // every workgroup loads the real form into LDS first: k = 6 (128 KiB,
    // complex128) amortises it over many blocks per workgroup; smaller forms
    // take a larger grid, whose concurrent workgroups stream closer together
    const int64_t cap = K == 6 ? 256 * 16 : 256 * 256;
    int64_t grid = std::min<int64_t>((nblk + wpg - 1) / wpg, cap);
    DenseSpec spl = sp;
    // whole teams only: every residue of a team's stride needs its workgroup
    spl.team = (int)std::min<int64_t>(std::max(sp.team, 1), grid);
    grid = grid / spl.team * spl.team;
    const int64_t teams = grid / spl.team;
    spl.per_team = (nblk + teams - 1) / teams;
    hipLaunchKernelGGL((k_dense<T, K>), dim3((unsigned)grid), dim3(threads), lds, s, psi, B, spl);
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
