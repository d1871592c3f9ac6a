// k_adjoint.hip -- adjoint differentiation kernels for gfx950.
//
// Adjoint method (Jones & Gacon 2020, arXiv 2009.02823), a project addition
// to the paper's simulator (its Listing 1 differentiates a circuit through an
// autograd interface without naming the method).  For
// E = <psi|O|psi>, psi = U_P ... U_1 |psi_in>:
//   phi_k = U_k ... U_1 |psi_in>,  lambda_k = U_{k+1}^dag ... U_P^dag O psi,
//   dE/dth_k = 2 Re <lambda_k| dU_k/dth |phi_{k-1}>.
// With U = exp(-i th P / 2) this is Im <lambda_k| P |phi_k>; with
// PHASE(th) = exp(i th |1><1|) it is -2 Im <lambda_k| |1><1| |phi_k>.  The
// sweep starts from phi = psi, lambda = O psi and walks the ops backwards,
// un-applying each op on both states; a parameterised op first adds its
// generator inner product.  k_adj_rot does both in one pass: it reads the
// pair of phi and the pair of lambda once, and writes both back.
#include "sv_core.h"

namespace svk {

__device__ __forceinline__ double block_sum_adj(double v)
{
    __shared__ double sm[1024 / 64];
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

template <typename V, typename T>
__device__ __forceinline__ V cmad2a(T ar_, T ai_, V a, T br_, T bi_, V b)
{
    V r;
    r.x = (ar_ * a.x - ai_ * a.y) + (br_ * b.x - bi_ * b.y);
    r.y = (ar_ * a.y + ai_ * a.x) + (br_ * b.y + bi_ * b.x);
    return r;
}

// Im( conj(l) * g ) in fp64
template <typename V>
__device__ __forceinline__ double im_conj_mul(const V l, double gr, double gi)
{
    return (double)l.x * gi - (double)l.y * gr;
}

template <typename T, int GEN>
__global__ void __launch_bounds__(kReduceThreads)
k_adj_rot(typename Vec2<T>::type* __restrict__ phi, typename Vec2<T>::type* __restrict__ lam, GroupSpec gs,
          uint64_t off, Coef2<T> u, double* __restrict__ partials)
{
    using V = typename Vec2<T>::type;
    constexpr int UN = 2;
    double acc = 0.0;
    const uint64_t per_block = (uint64_t)blockDim.x * UN;
    const uint64_t stride = (uint64_t)gridDim.x * per_block;
    for (uint64_t g0 = (uint64_t)blockIdx.x * per_block + threadIdx.x; g0 < gs.n_groups + threadIdx.x;
         g0 += stride) {
        uint64_t b[UN];
        V p0[UN], p1[UN], l0[UN], l1[UN];
#pragma unroll
        for (int j = 0; j < UN; ++j) {
            const uint64_t g = g0 + (uint64_t)j * blockDim.x;
            if (g < gs.n_groups) {
                b[j] = group_base(g, gs);
                p0[j] = phi[b[j]];
                p1[j] = phi[b[j] + off];
                l0[j] = lam[b[j]];
                l1[j] = lam[b[j] + off];
            }
        }
#pragma unroll
        for (int j = 0; j < UN; ++j) {
            const uint64_t g = g0 + (uint64_t)j * blockDim.x;
            if (g < gs.n_groups) {
                // generator applied to phi's pair, in fp64
                const double a0r = p0[j].x, a0i = p0[j].y, a1r = p1[j].x, a1i = p1[j].y;
                double c;
                if constexpr (GEN == GEN_X) {  // X (a0, a1) = (a1, a0)
                    c = im_conj_mul(l0[j], a1r, a1i) + im_conj_mul(l1[j], a0r, a0i);
                } else if constexpr (GEN == GEN_Y) {  // Y (a0, a1) = (-i a1, i a0)
                    c = im_conj_mul(l0[j], a1i, -a1r) + im_conj_mul(l1[j], -a0i, a0r);
                } else if constexpr (GEN == GEN_Z) {  // Z (a0, a1) = (a0, -a1)
                    c = im_conj_mul(l0[j], a0r, a0i) - im_conj_mul(l1[j], a1r, a1i);
                } else {  // |1><1| (a0, a1) = (0, a1)
                    c = im_conj_mul(l1[j], a1r, a1i);
                }
                acc += c;
                const V q0 = cmad2a<V, T>(u.m[0], u.m[1], p0[j], u.m[2], u.m[3], p1[j]);
                const V q1 = cmad2a<V, T>(u.m[4], u.m[5], p0[j], u.m[6], u.m[7], p1[j]);
                const V m0 = cmad2a<V, T>(u.m[0], u.m[1], l0[j], u.m[2], u.m[3], l1[j]);
                const V m1 = cmad2a<V, T>(u.m[4], u.m[5], l0[j], u.m[6], u.m[7], l1[j]);
                phi[b[j]] = q0;
                phi[b[j] + off] = q1;
                lam[b[j]] = m0;
                lam[b[j] + off] = m1;
            }
        }
    }
    const double s = block_sum_adj(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

struct ObsTerms {
    int32_t nterms;
    double c[kDiagTermsPerPass];
    uint64_t z[kDiagTermsPerPass];
};

// lam[x] (=|+=) o(x) psi[x] for a diagonal observable.
template <typename T>
__global__ void __launch_bounds__(256)
k_obs_diag_apply(const typename Vec2<T>::type* __restrict__ psi, typename Vec2<T>::type* __restrict__ lam,
                 uint64_t n_amps, int nq, int kind, double coeff, ObsTerms terms, int accumulate)
{
    using V = typename Vec2<T>::type;
    const uint64_t zzmask = nq > 1 ? ((1ull << (nq - 1)) - 1ull) : 0ull;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n_amps; x += stride) {
        double o;
        if (kind == 1) {
            o = (double)(nq - 2 * (int)__popcll(x));
        } else if (kind == 2) {
            o = (double)((nq - 1) - 2 * (int)__popcll((x ^ (x >> 1)) & zzmask));
        } else {
            o = 0.0;
            for (int k = 0; k < terms.nterms; ++k) o += (__popcll(x & terms.z[k]) & 1) ? -terms.c[k] : terms.c[k];
        }
        o *= coeff;
        const V a = psi[x];
        V r;
        if (accumulate) {
            const V l = lam[x];
            r.x = (T)((double)l.x + o * (double)a.x);
            r.y = (T)((double)l.y + o * (double)a.y);
        } else {
            r.x = (T)(o * (double)a.x);
            r.y = (T)(o * (double)a.y);
        }
        lam[x] = r;
    }
}

// lam[y] += coeff * i^ny * (-1)^{pc((y ^ f) & z)} * psi[y ^ f]
template <typename T>
__global__ void __launch_bounds__(256)
k_obs_pauli_apply(const typename Vec2<T>::type* __restrict__ psi, typename Vec2<T>::type* __restrict__ lam,
                  uint64_t n_amps, uint64_t f, uint64_t z, int ny, double coeff)
{
    using V = typename Vec2<T>::type;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t y = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; y < n_amps; y += stride) {
        const uint64_t x = y ^ f;
        const V a = psi[x];
        const double sg = ((__popcll(x & z) & 1) ? -coeff : coeff);
        double wr = sg * (double)a.x, wi = sg * (double)a.y;
        double tr, ti;  // multiply by i^ny
        switch (ny & 3) {
        case 0: tr = wr; ti = wi; break;
        case 1: tr = -wi; ti = wr; break;
        case 2: tr = -wr; ti = -wi; break;
        default: tr = wi; ti = -wr; break;
        }
        const V l = lam[y];
        V r;
        r.x = (T)((double)l.x + tr);
        r.y = (T)((double)l.y + ti);
        lam[y] = r;
    }
}

template <typename T>
__global__ void __launch_bounds__(kReduceThreads)
k_inner_partial(const typename Vec2<T>::type* __restrict__ a, const typename Vec2<T>::type* __restrict__ b,
                uint64_t n, double* __restrict__ partials)
{
    using V = typename Vec2<T>::type;
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 2;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x * 2 + threadIdx.x; i0 < n + threadIdx.x; i0 += stride) {
        V va[2], vb[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const uint64_t i = i0 + (uint64_t)j * blockDim.x;
            if (i < n) {
                va[j] = a[i];
                vb[j] = b[i];
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const uint64_t i = i0 + (uint64_t)j * blockDim.x;
            if (i < n) acc += (double)va[j].x * (double)vb[j].x + (double)va[j].y * (double)vb[j].y;
        }
    }
    const double s = block_sum_adj(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void k_scatter_grads(const double* __restrict__ slot_val, const int* __restrict__ slot_param,
                                const double* __restrict__ slot_scale, int n_slots, double* __restrict__ grad,
                                int n_params)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_params) return;
    double g = 0.0;
    for (int s = 0; s < n_slots; ++s)
        if (slot_param[s] == j) g += slot_scale[s] * slot_val[s];
    grad[j] = g;
}

// --------------------------------------------------------------------------
template <typename T>
hipError_t launch_adj_rot(void* phi, void* lam, const GroupSpec& gs, uint64_t off, int gen, const Coef2<T>& udag,
                          double* partials, int nblocks, hipStream_t s)
{
    using V = typename Vec2<T>::type;
    V* p = (V*)phi;
    V* l = (V*)lam;
    const dim3 g((unsigned)nblocks), b(kReduceThreads);
    switch (gen) {
    case GEN_X: hipLaunchKernelGGL((k_adj_rot<T, GEN_X>), g, b, 0, s, p, l, gs, off, udag, partials); break;
    case GEN_Y: hipLaunchKernelGGL((k_adj_rot<T, GEN_Y>), g, b, 0, s, p, l, gs, off, udag, partials); break;
    case GEN_Z: hipLaunchKernelGGL((k_adj_rot<T, GEN_Z>), g, b, 0, s, p, l, gs, off, udag, partials); break;
    default: hipLaunchKernelGGL((k_adj_rot<T, GEN_P1>), g, b, 0, s, p, l, gs, off, udag, partials); break;
    }
    return hipGetLastError();
}

static unsigned elementwise_grid(uint64_t n)
{
    uint64_t nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    if (nb < 1) nb = 1;
    return (unsigned)nb;
}

template <typename T>
hipError_t launch_obs_diag_apply(const void* psi, void* lam, int n, int kind, double coeff, const double* hcoef,
                                 const uint64_t* hz, int nterms, int accumulate, hipStream_t s)
{
    using V = typename Vec2<T>::type;
    ObsTerms t{};
    if (nterms > kDiagTermsPerPass) return hipErrorInvalidValue;
    t.nterms = kind == 0 ? nterms : 0;
    for (int k = 0; k < t.nterms; ++k) {
        t.c[k] = hcoef[k];
        t.z[k] = hz[k];
    }
    const uint64_t na = 1ull << n;
    hipLaunchKernelGGL((k_obs_diag_apply<T>), dim3(elementwise_grid(na)), dim3(256), 0, s, (const V*)psi, (V*)lam,
                       na, n, kind, coeff, t, accumulate);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_obs_pauli_apply(const void* psi, void* lam, int n, uint64_t xmask, uint64_t zmask, int ny,
                                  double coeff, hipStream_t s)
{
    using V = typename Vec2<T>::type;
    const uint64_t na = 1ull << n;
    hipLaunchKernelGGL((k_obs_pauli_apply<T>), dim3(elementwise_grid(na)), dim3(256), 0, s, (const V*)psi, (V*)lam,
                       na, xmask, zmask, ny, coeff);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_inner_partial(const void* a, const void* b, uint64_t n_amps, double* partials, hipStream_t s)
{
    using V = typename Vec2<T>::type;
    const int nb = reduce_blocks_for(n_amps);
    hipLaunchKernelGGL((k_inner_partial<T>), dim3(nb), dim3(kReduceThreads), 0, s, (const V*)a, (const V*)b, n_amps,
                       partials);
    return hipGetLastError();
}

hipError_t launch_scatter_grads(const double* slot_val, const int* slot_param, const double* slot_scale, int n_slots,
                                double* grad, int n_params, hipStream_t s)
{
    if (n_params <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_grads, dim3((n_params + 255) / 256), dim3(256), 0, s, slot_val, slot_param,
                       slot_scale, n_slots, grad, n_params);
    return hipGetLastError();
}

#define SV_ADJ_INST(T)                                                                                          \
    template hipError_t launch_adj_rot<T>(void*, void*, const GroupSpec&, uint64_t, int, const Coef2<T>&,       \
                                          double*, int, hipStream_t);                                           \
    template hipError_t launch_obs_diag_apply<T>(const void*, void*, int, int, double, const double*,           \
                                                 const uint64_t*, int, int, hipStream_t);                       \
    template hipError_t launch_obs_pauli_apply<T>(const void*, void*, int, uint64_t, uint64_t, int, double,     \
                                                  hipStream_t);                                                 \
    template hipError_t launch_inner_partial<T>(const void*, const void*, uint64_t, double*, hipStream_t);

SV_ADJ_INST(double)
SV_ADJ_INST(float)

}  // namespace svk
