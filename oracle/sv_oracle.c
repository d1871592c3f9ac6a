/*
 * sv_oracle.c -- plain CPU reference simulator (the oracle).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file's library.  The HIP
 * product library shares no code, header, table or constant with it.
 *
 * What it computes (Kang & Ryu, "PennyLane-Lightning MPI", arXiv 2508.13615):
 *   Sec. 2 -- an N-qubit state is a vector of 2^N complex amplitudes; every
 *   gate is a small logic matrix (at most 8x8) applied to the amplitudes that
 *   differ only in the gate's qubits, and the "general approach" of Sec. 3.1 is
 *   exactly that dense matrix-vector product.  Gate-specific kernels skip only
 *   zero terms, so the dense product *is* the plain definition they must
 *   reproduce.  A control qubit (Sec. 2, CNOT discussion; Sec. 3.1) only
 *   selects where the gate acts: the gate acts iff every control bit is 1.
 *
 * Conventions:
 *   - amplitudes are complex128, stored as interleaved (re, im) doubles;
 *   - qubit q is bit q (weight 2^q) of the amplitude index: Sec. 2 numbers
 *     qubits from zero and calls the first L of them local under an even block
 *     partition, which makes them the low index bits (partner rank distance
 *     2^(q_T - L) confirms it);
 *   - a k-qubit matrix on targets (t_0 .. t_{k-1}) is row-major 2^k x 2^k
 *     (interleaved complex); its row/column index is
 *     r = sum_j bit_{t_j}(x) * 2^(k-1-j), i.e. the first-listed target is the
 *     most significant bit of the matrix index (the paper is silent; this is
 *     the textbook CNOT(c,t) layout).
 *
 * Precision: fp64 throughout; compiled without fast-math and without FP
 * contraction, every sum taken in ascending index order.
 *
 * The one optional parallel construct is an OpenMP loop over independent
 * amplitude groups in oracle_apply_matrix / the move routines: each group is
 * computed exactly as in the serial loop, so results do not depend on the
 * thread count.  Reductions are always serial.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EARG 1
#define ORACLE_EQUBIT 2
#define ORACLE_EOOM 3

#define ORACLE_MAX_QUBITS 40
#define ORACLE_MAX_K 6

static int bit_of(uint64_t x, int q) { return (int)((x >> q) & 1u); }

/* Every listed qubit must be in [0, n) and appear once across controls and
 * targets. */
static int check_qubits(int n, const int* ctrl, int nc, const int* tgt, int k)
{
    uint64_t seen = 0;
    if (n < 1 || n > ORACLE_MAX_QUBITS) return ORACLE_EARG;
    if (nc < 0 || k < 0 || nc + k > ORACLE_MAX_QUBITS) return ORACLE_EARG;
    for (int j = 0; j < nc + k; ++j) {
        int q = j < nc ? ctrl[j] : tgt[j - nc];
        if (q < 0 || q >= n) return ORACLE_EQUBIT;
        if (seen & (1ull << q)) return ORACLE_EQUBIT;
        seen |= 1ull << q;
    }
    return ORACLE_OK;
}

/*
 * Dense application of a k-qubit matrix U, restricted to the indices whose
 * control bits are all 1 (Sec. 2 / Sec. 3.1 general approach; controls as in
 * the CNOT discussion of Sec. 2).
 *
 * For every index x whose target bits are all 0 and whose control bits are all
 * 1: gather v[r] = psi[x + sum_j ((r >> (k-1-j)) & 1) * 2^{t_j}], form
 * w[r] = sum_c U[r][c] * v[c] (ascending c), scatter w back.
 */
int oracle_apply_matrix(double* psi, int n, const int* ctrl, int nc,
                        const int* tgt, int k, const double* U)
{
    int rc = check_qubits(n, ctrl, nc, tgt, k);
    if (rc) return rc;
    if (k < 1 || k > ORACLE_MAX_K || psi == NULL || U == NULL) return ORACLE_EARG;
    const int64_t dim = (int64_t)1 << n;
    const int m = 1 << k;

#pragma omp parallel for schedule(static)
    for (int64_t xs = 0; xs < dim; ++xs) {
        uint64_t x = (uint64_t)xs;
        int skip = 0;
        for (int j = 0; j < k; ++j)
            if (bit_of(x, tgt[j])) skip = 1;
        for (int j = 0; j < nc; ++j)
            if (!bit_of(x, ctrl[j])) skip = 1;
        if (skip) continue;

        uint64_t idx[1 << ORACLE_MAX_K];
        double vr[1 << ORACLE_MAX_K], vi[1 << ORACLE_MAX_K];
        double wr[1 << ORACLE_MAX_K], wi[1 << ORACLE_MAX_K];
        for (int r = 0; r < m; ++r) {
            uint64_t y = x;
            for (int j = 0; j < k; ++j)
                if ((r >> (k - 1 - j)) & 1) y |= 1ull << tgt[j];
            idx[r] = y;
            vr[r] = psi[2 * y];
            vi[r] = psi[2 * y + 1];
        }
        for (int r = 0; r < m; ++r) {
            double sr = 0.0, si = 0.0;
            for (int c = 0; c < m; ++c) {
                double ur = U[2 * (r * m + c)];
                double ui = U[2 * (r * m + c) + 1];
                sr = sr + (ur * vr[c] - ui * vi[c]);
                si = si + (ur * vi[c] + ui * vr[c]);
            }
            wr[r] = sr;
            wi[r] = si;
        }
        for (int r = 0; r < m; ++r) {
            psi[2 * idx[r]] = wr[r];
            psi[2 * idx[r] + 1] = wi[r];
        }
    }
    return ORACLE_OK;
}

static void swap_elems(unsigned char* base, size_t es, uint64_t a, uint64_t b)
{
    unsigned char tmp[32];
    memcpy(tmp, base + a * es, es);
    memcpy(base + a * es, base + b * es, es);
    memcpy(base + b * es, tmp, es);
}

/*
 * Pauli-X on target t restricted to control bits = 1 (X, CNOT, Toffoli and
 * multi-controlled X).  Sec. 2: X exchanges each amplitude pair that differs
 * only in the target bit; a control only decides where that happens.  Done as
 * a pure move of elem_bytes-sized elements (8 = complex64, 16 = complex128),
 * so the result is bit-exact in either precision.
 */
int oracle_move_x(void* psi, int elem_bytes, int n, const int* ctrl, int nc, int t)
{
    int rc = check_qubits(n, ctrl, nc, &t, 1);
    if (rc) return rc;
    if (psi == NULL || (elem_bytes != 8 && elem_bytes != 16)) return ORACLE_EARG;
    const int64_t dim = (int64_t)1 << n;
    unsigned char* p = (unsigned char*)psi;
#pragma omp parallel for schedule(static)
    for (int64_t xs = 0; xs < dim; ++xs) {
        uint64_t x = (uint64_t)xs;
        int act = !bit_of(x, t);
        for (int j = 0; j < nc; ++j)
            if (!bit_of(x, ctrl[j])) act = 0;
        if (act) swap_elems(p, (size_t)elem_bytes, x, x | (1ull << t));
    }
    return ORACLE_OK;
}

/*
 * SWAP of qubits a and b (restricted to control bits = 1): the amplitudes of
 * |..1_a..0_b..> and |..0_a..1_b..> trade places.  Pure move.
 */
int oracle_move_swap(void* psi, int elem_bytes, int n, const int* ctrl, int nc, int a, int b)
{
    int ab[2] = {a, b};
    int rc = check_qubits(n, ctrl, nc, ab, 2);
    if (rc) return rc;
    if (psi == NULL || (elem_bytes != 8 && elem_bytes != 16)) return ORACLE_EARG;
    const int64_t dim = (int64_t)1 << n;
    unsigned char* p = (unsigned char*)psi;
#pragma omp parallel for schedule(static)
    for (int64_t xs = 0; xs < dim; ++xs) {
        uint64_t x = (uint64_t)xs;
        int act = bit_of(x, a) && !bit_of(x, b);
        for (int j = 0; j < nc; ++j)
            if (!bit_of(x, ctrl[j])) act = 0;
        if (act) swap_elems(p, (size_t)elem_bytes, x, (x ^ (1ull << a)) ^ (1ull << b));
    }
    return ORACLE_OK;
}

/*
 * Inner product <phi|chi> = sum_x conj(phi_x) * chi_x, summed serially in
 * ascending x.  out[0] = real part, out[1] = imaginary part.
 */
int oracle_inner(const double* phi, const double* chi, int n, double* out)
{
    if (n < 1 || n > ORACLE_MAX_QUBITS || !phi || !chi || !out) return ORACLE_EARG;
    const uint64_t dim = 1ull << n;
    double sr = 0.0, si = 0.0;
    for (uint64_t x = 0; x < dim; ++x) {
        double ar = phi[2 * x], ai = phi[2 * x + 1];
        double br = chi[2 * x], bi = chi[2 * x + 1];
        sr = sr + (ar * br + ai * bi);
        si = si + (ar * bi - ai * br);
    }
    out[0] = sr;
    out[1] = si;
    return ORACLE_OK;
}

/*
 * Expectation value of a Pauli string, <psi| P |psi>, the measurement the
 * Python binding exposes as expval (Sec. 2 "measurement processes"; Listing 1
 * calls it on a Hamiltonian).  By definition: copy psi, apply each listed
 * Pauli's 2x2 matrix with oracle_apply_matrix, take the inner product.
 * 'I' letters are skipped.  out[0] = Re E, out[1] = Im E (zero up to rounding).
 */
int oracle_expval_pauli(const double* psi, int n, const char* paulis,
                        const int* qubits, int np, double* out)
{
    static const double PX[8] = {0, 0, 1, 0, 1, 0, 0, 0};
    static const double PY[8] = {0, 0, 0, -1, 0, 1, 0, 0};
    static const double PZ[8] = {1, 0, 0, 0, 0, 0, -1, 0};
    int rc = check_qubits(n, NULL, 0, qubits, np);
    if (rc) return rc;
    if (!psi || !out || (np > 0 && !paulis)) return ORACLE_EARG;
    const uint64_t dim = 1ull << n;
    double* tmp = (double*)malloc(sizeof(double) * 2 * dim);
    if (!tmp) return ORACLE_EOOM;
    memcpy(tmp, psi, sizeof(double) * 2 * dim);
    for (int j = 0; j < np; ++j) {
        const double* m = NULL;
        switch (paulis[j]) {
        case 'I': continue;
        case 'X': m = PX; break;
        case 'Y': m = PY; break;
        case 'Z': m = PZ; break;
        default: free(tmp); return ORACLE_EARG;
        }
        rc = oracle_apply_matrix(tmp, n, NULL, 0, &qubits[j], 1, m);
        if (rc) { free(tmp); return rc; }
    }
    rc = oracle_inner(psi, tmp, n, out);
    free(tmp);
    return rc;
}

int oracle_version(void) { return 1; }

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
