// Runs of diagonal gates as one pass: declarations shared by the entry points
// (sv_api.hip) and the kernel (k_phase.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace svk {

constexpr int kMaxPhaseTerms = 64;
constexpr int kMaxPhaseCommon = 40;

// psi[x] *= exp(i pi sum_t turns[t] [x contains mask[t]]).  Amplitudes without
// every bit of `common` (the bits all masks share) are not touched: the pass
// enumerates the others, inserting `common`'s bits (ascending positions) as 1.
struct PhaseRun {
    int n_terms;
    int n_common;
    int common_pos[kMaxPhaseCommon];
    int64_t groups;  // 2^(n - n_common)
    uint64_t mask[kMaxPhaseTerms];
    double turns[kMaxPhaseTerms];  // angle / pi
};

hipError_t launch_phase_run(void* psi, int dtype, const PhaseRun& pr, hipStream_t s);

// Row-major 2x2 of a one-target gate, interleaved (re, im).
struct PairCoef {
    double m[8];
};

// The one-target gate u on qubit t, then the phase run, in one pass over the
// amplitude pairs of bit t (pr.groups = 2^(n-1), pr.n_common = 0); the
// run's first n_with terms hold bit t, the others do not.
hipError_t launch_pair_phase_run(void* psi, int dtype, int t, const PairCoef& u, const PhaseRun& pr, int n_with,
                                 hipStream_t s);

// A phase run linear in the index's bits on the 1 side of a pair gate:
// exp(i pi (turns_const + sum_b turns_of_bit[b] x_b)), bits 0 .. 8 n_bytes - 1.
constexpr int kLinearPhaseBytes = 5;
struct LinearPhase {
    int n_bytes;
    double turns_const;
    double turns_of_bit[8 * kLinearPhaseBytes];
};

// table: device scratch of at least kLinearPhaseTableBytes (stream-ordered use).
constexpr size_t kLinearPhaseTableBytes = (size_t)kLinearPhaseBytes * 256 * 16;
hipError_t launch_pair_linear_phase(void* psi, int dtype, int t, const PairCoef& u, const LinearPhase& lp,
                                    int64_t groups, void* table, hipStream_t s);

}  // namespace svk
