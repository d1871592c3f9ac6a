// Dense k-qubit unitaries (4 <= k <= 6) on the matrix cores: declarations
// shared by the entry point (sv_api.hip) and the kernels (k_dense.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace svk {

constexpr int kDenseMinK = 4;
constexpr int kDenseMaxK = 6;

// Where a group's amplitudes live: the group index g (0 .. 2^(n-k) - 1) gets a
// zero bit inserted at each target position (ascending), and amplitude c of
// the group (c = matrix index, first-listed target its most significant bit)
// sits at base(g) | dep[c].
struct DenseSpec {
    int k;
    int qs_sorted[kDenseMaxK];
    uint64_t dep[1 << kDenseMaxK];
    int64_t groups;  // 2^(n-k)
    int order;       // workgroup walk order (block_slot in sv_core.h)
    int team;          // workgroups that walk one contiguous run of 16-group blocks together (capped at the grid)
    int64_t per_team;  // blocks per team (set by the launcher)
};

// Real form of the 2^k x 2^k complex matrix U: 2^(k+1) x 2^(k+1), row-major,
// entry [row of (c, p)][column of (r, q)] the weight of component p (0 re,
// 1 im) of input amplitude c in component q of output amplitude r, rows and
// columns in the kernels' order (k_dense.hip).
void dense_real_form(const double* U, int k, double* B);

// psi (interleaved complex128 or complex64, per `dtype`) <- U on the spec's
// targets; B: the real form in the state's precision, in device memory.
hipError_t launch_dense(void* psi, int dtype, const void* B, const DenseSpec& spec, hipStream_t s);

// Dynamic LDS of one workgroup for k (the real form of U).
size_t dense_lds_bytes(int k, int dtype);

}  // namespace svk
