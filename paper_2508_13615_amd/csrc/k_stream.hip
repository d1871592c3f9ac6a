// k_stream.hip -- the measured HBM ceiling the gate kernels are compared
// against: plain streaming kernels (copy, read-only, write-only, in-place
// read-and-write) with 16-byte
// non-temporal accesses, in the same work layout as the gate kernels (each
// workgroup owns one tile of block * unroll vectors, thread i handles
// vectors i, i + block, ...: every load instruction of a wavefront covers
// 1 KiB of consecutive bytes).  A gate that moves B bytes can at best match
// B / (time of this kernel moving B bytes).
#include <algorithm>
#include <cstdio>

#include "sv_core.h"

namespace svk {

template <int MODE, int U>
__global__ void __launch_bounds__(1024)
k_stream(const double2* __restrict__ src, double2* __restrict__ dst, uint64_t n, double2* __restrict__ sink)
{
    const uint64_t per_block = (uint64_t)blockDim.x * U;
    const uint64_t stride = (uint64_t)gridDim.x * per_block;
    double acc = 0.0;
    // the in-place form reads and writes dst, like a gate on its state
    const double2* __restrict__ in = MODE == 3 ? (const double2*)dst : src;
    for (uint64_t i0 = (uint64_t)blockIdx.x * per_block + threadIdx.x; i0 < n + threadIdx.x; i0 += stride) {
        double2 v[U];
        if constexpr (MODE != 2) {
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const uint64_t i = i0 + (uint64_t)j * blockDim.x;
                if (i < n) {
                    v[j].x = __builtin_nontemporal_load(&in[i].x);
                    v[j].y = __builtin_nontemporal_load(&in[i].y);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t i = i0 + (uint64_t)j * blockDim.x;
            if (i < n) {
                if constexpr (MODE == 0) {
                    __builtin_nontemporal_store(v[j].x, &dst[i].x);
                    __builtin_nontemporal_store(v[j].y, &dst[i].y);
                } else if constexpr (MODE == 1) {
                    acc += v[j].x + v[j].y;
                } else if constexpr (MODE == 3) {
                    // negated, so the store cannot be dropped as a no-op
                    __builtin_nontemporal_store(-v[j].x, &dst[i].x);
                    __builtin_nontemporal_store(-v[j].y, &dst[i].y);
                } else {
                    __builtin_nontemporal_store(0.0, &dst[i].x);
                    __builtin_nontemporal_store(0.0, &dst[i].y);
                }
            }
        }
    }
    if constexpr (MODE == 1) {
        // keeps the loads: the sum is stored only if it is exactly this
        // value, which a finite input sums to with negligible probability
        if (acc == 1.2345678901234567e300 && sink) {
            double2 w;
            w.x = acc;
            w.y = 0.0;
            sink[0] = w;
        }
    }
}

hipError_t launch_stream(int mode, void* dst, const void* src, uint64_t n16, int block, int unroll, hipStream_t s)
{
    if (n16 == 0) return hipSuccess;
    const uint64_t per = (uint64_t)block * (uint64_t)unroll;
    uint64_t nb = (n16 + per - 1) / per;
    const uint64_t lim = std::min<uint64_t>(1ull << 30, 0xffffffffull / (uint64_t)block);
    if (nb > lim) nb = lim;  // the stride loop covers the rest
    const dim3 grid((unsigned)nb), blk((unsigned)block);
    const double2* sp = (const double2*)src;
    double2* dp = (double2*)dst;
#define SV_STREAM_GO(M)                                                                                    \
    switch (unroll) {                                                                                      \
    case 1: hipLaunchKernelGGL((k_stream<M, 1>), grid, blk, 0, s, sp, dp, n16, dp); break;                 \
    case 2: hipLaunchKernelGGL((k_stream<M, 2>), grid, blk, 0, s, sp, dp, n16, dp); break;                 \
    case 4: hipLaunchKernelGGL((k_stream<M, 4>), grid, blk, 0, s, sp, dp, n16, dp); break;                 \
    default: hipLaunchKernelGGL((k_stream<M, 8>), grid, blk, 0, s, sp, dp, n16, dp); break;                \
    }
    if (mode == 0) {
        SV_STREAM_GO(0)
    } else if (mode == 1) {
        SV_STREAM_GO(1)
    } else if (mode == 2) {
        SV_STREAM_GO(2)
    } else {
        SV_STREAM_GO(3)
    }
#undef SV_STREAM_GO
    return hipGetLastError();
}

}  // namespace svk

using namespace svk;

sv_status sv_stream_bench(int mode, void* dst, const void* src, size_t bytes, int block, int unroll, void* stream)
{
    if (mode < 0 || mode > 3) return set_error(SV_ERR_ARG, "mode must be 0 (copy), 1 (read), 2 (write) or 3 (in place)");
    if (bytes == 0 || bytes % 16) return set_error(SV_ERR_ARG, "bytes must be a positive multiple of 16");
    if (block < 64 || block > 1024 || (block & 63)) return set_error(SV_ERR_ARG, "block must be a multiple of 64 in [64, 1024]");
    if (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8) return set_error(SV_ERR_ARG, "unroll must be 1, 2, 4 or 8");
    const bool reads_src = mode == 0 || mode == 1, writes_dst = mode != 1;
    if (reads_src && (!src || ((uintptr_t)src) % 16)) return set_error(SV_ERR_ARG, "src must be 16-byte aligned");
    if (writes_dst && (!dst || ((uintptr_t)dst) % 16)) return set_error(SV_ERR_ARG, "dst must be 16-byte aligned");
    // the read-only form may store one vector into dst when given one; without
    // a dst it stores nothing
    const hipError_t e = launch_stream(mode, dst, src, bytes / 16, block, unroll, (hipStream_t)stream);
    if (e != hipSuccess) {
        char buf[160];
        snprintf(buf, sizeof buf, "stream kernel: %s", hipGetErrorString(e));
        return set_error(SV_ERR_HIP, buf);
    }
    return SV_OK;
}
