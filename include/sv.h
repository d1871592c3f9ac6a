/*
 * sv.h -- C ABI of libsv, a state-vector gate engine for AMD Instinct MI355X
 * (gfx950).
 *
 * Method: Kang & Ryu, "PennyLane-Lightning MPI: a massively scalable quantum
 * circuit simulator based on distributed computing in CPU clusters"
 * (arXiv 2508.13615).  Sec. 2 states the problem this library solves on one
 * device: an N-qubit state is 2^N complex amplitudes, gates are small logic
 * matrices (at most 8x8) "conducted to" qubit indices, and only the non-zero
 * elements of a gate's matrix are used, so each gate gets its own index- and
 * gate-specific routine: permutation gates move amplitudes, diagonal gates
 * multiply a subset in place, a control bit only selects where a gate acts.
 * Sec. 3.1 compares such routines with the "general approach", a dense
 * matrix-vector product, which is exported here as sv_apply_general.
 *
 * Conventions for every entry point:
 *   - Qubit q is bit q (weight 2^q) of the amplitude index (Sec. 2 numbers
 *     qubits from zero; the first L are the local ones of a block partition,
 *     i.e. the low bits).
 *   - Amplitudes are interleaved (re, im): complex128 = two doubles,
 *     complex64 = two floats, contiguous, 2^N of them.
 *   - A k-qubit matrix argument is a HOST array of 2 * 4^k doubles: row-major
 *     2^k x 2^k, interleaved complex, with row/column index
 *     r = sum_j bit_{targets[j]} * 2^(k-1-j) (the first-listed target is the
 *     most significant bit).  For a complex64 state it is rounded to float
 *     once, on the host.
 *   - Controls are 1-controls: the gate acts only where every control bit is 1.
 *   - Rotations are exp(-i th P / 2) for P in {X, Y, Z}; PHASE(phi) is
 *     diag(1, e^{i phi}).
 *   - Host arrays passed in are read during the call only; the library keeps
 *     no pointer to them.
 *   - Every call validates its arguments on the host before any device work.
 *     On a validation failure nothing is launched and nothing is modified;
 *     the status says why and sv_last_error() returns a message.
 *   - Device work is queued on the state's HIP stream and is asynchronous
 *     unless the entry point returns a host value (then it synchronises that
 *     stream).  A fault in a queued kernel is reported as SV_ERR_HIP by the
 *     next synchronising call.
 *   - Calls on one state are not thread-safe with respect to each other;
 *     sv_last_error() is per thread.
 *   - Handles (sv_state, sv_circuit, sv_batch) are opaque values, not
 *     addresses.  Each carries its kind and a generation: after sv_free (or
 *     sv_circuit_free / sv_batch_free) every copy of the handle is rejected
 *     with SV_ERR_HANDLE, and so is a handle of another kind, even when a
 *     new object reuses the freed one's memory.
 */
#ifndef SV_ABI_H_INCLUDED
#define SV_ABI_H_INCLUDED

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SV_MAX_QUBITS 40   /* validation limit; allocation fails earlier if HBM is short */
#define SV_MAX_CONTROLS 8
#define SV_MAX_GENERAL_K 3 /* dense baseline: up to 8x8 (Sec. 2: logic matrices up to 8x8) */
#define SV_OP_MAX_QUBITS 10

typedef struct sv_state_s* sv_state;
typedef struct sv_circuit_s* sv_circuit;
typedef struct sv_batch_s* sv_batch;

typedef enum { SV_C64 = 1, SV_C128 = 2 } sv_dtype;

typedef enum {
    SV_OK = 0,
    SV_ERR_ARG = 1,         /* malformed argument (null pointer, bad size, bad enum) */
    SV_ERR_QUBIT = 2,       /* qubit index out of range or repeated */
    SV_ERR_OOM = 3,         /* device allocation failed */
    SV_ERR_HIP = 4,         /* HIP runtime error (launch or earlier asynchronous fault) */
    SV_ERR_UNSUPPORTED = 5, /* valid request this build does not implement */
    SV_ERR_HANDLE = 6       /* null or freed handle */
} sv_status;

typedef enum {
    SV_I = 0,
    SV_X = 1,     /* permutation: with 0/1/2 controls = X / CNOT / Toffoli */
    SV_Y = 2,
    SV_Z = 3,     /* diagonal; with controls = CZ, CCZ ... */
    SV_H = 4,
    SV_S = 5,
    SV_T = 6,
    SV_RX = 7,    /* params[0] = theta */
    SV_RY = 8,
    SV_RZ = 9,
    SV_PHASE = 10, /* params[0] = phi; with one control = controlled phase (QFT) */
    SV_SWAP = 11, /* two targets; permutation */
    SV_U2 = 12,   /* matrix gate, one target */
    SV_U4 = 13    /* matrix gate, two targets */
} sv_gate;

/* ------------------------------------------------------------------------
 * State lifecycle and data movement
 * ------------------------------------------------------------------------ */

/* Allocate a 2^n_qubits state in device memory and set it to |0...0>.
 * stream: a hipStream_t (NULL = the null stream) on which all work on this
 * state is queued.  The library owns the memory; release with sv_free.
 * Errors: SV_ERR_ARG (n_qubits outside [1, SV_MAX_QUBITS], bad dtype, null
 * out), SV_ERR_OOM (device allocation failed). */
sv_status sv_alloc(int n_qubits, sv_dtype dtype, void* stream, sv_state* out);

/* Wrap caller-owned device memory (e.g. a torch tensor) holding 2^n_qubits
 * amplitudes of `dtype`, 16-byte aligned.  The contents are left as they are;
 * sv_free releases only the handle, never dev_ptr. */
sv_status sv_wrap(void* dev_ptr, int n_qubits, sv_dtype dtype, void* stream, sv_state* out);

/* Release a handle (and its memory if sv_alloc made it).  Synchronises the
 * state's stream first.  Later use of the handle returns SV_ERR_HANDLE. */
sv_status sv_free(sv_state st);

sv_status sv_set_stream(sv_state st, void* stream);
sv_status sv_get_info(sv_state st, int* n_qubits, int* dtype, void** dev_ptr);
size_t sv_state_bytes(int n_qubits, sv_dtype dtype); /* 2^n * (8 or 16); 0 if invalid */

/* Set the state to the computational basis state |index>. */
sv_status sv_set_basis(sv_state st, uint64_t index);

/* Copy the whole state to / from host memory of exactly sv_state_bytes bytes.
 * Synchronous. */
sv_status sv_copy_to_host(sv_state st, void* host, size_t bytes);
sv_status sv_copy_from_host(sv_state st, const void* host, size_t bytes);

/* Device-to-device copy of a whole state (same size and dtype). */
sv_status sv_copy_state(sv_state dst, sv_state src);

/* Wait for all work queued on the state's stream; reports queued faults. */
sv_status sv_synchronize(sv_state st);

/* ------------------------------------------------------------------------
 * Gates (Sec. 2; gate-specific routines)
 * ------------------------------------------------------------------------ */

/* Apply a named gate to `targets` (1 target, or 2 for SV_SWAP / SV_U4).
 * params: host array, params[0] read for SV_RX/RY/RZ/PHASE, else may be NULL.
 * matrix: host 2x2 (SV_U2) or 4x4 (SV_U4) complex matrix, else NULL.
 * adjoint != 0 applies the gate's inverse (conjugate transpose).
 * The gate is dispatched by class: X/SWAP are pure amplitude moves
 * (bit-exact), Z/S/T/PHASE multiply only the amplitudes whose target bit is 1,
 * RZ is an element-wise phase, H/RX/RY/Y/U2 are paired updates, U4 is a
 * 4-amplitude update.
 * Errors: SV_ERR_HANDLE, SV_ERR_ARG (bad gate, nt, missing params/matrix),
 * SV_ERR_QUBIT (index out of range or repeated). */
sv_status sv_apply_gate(sv_state st, sv_gate gate, const int* targets, int nt,
                        const double* params, const double* matrix, int adjoint);

/* As sv_apply_gate, restricted to the amplitudes whose `controls` bits are
 * all 1 (nc in [0, SV_MAX_CONTROLS]); the work covers only that subset
 * (Sec. 2: a control only decides which part of the state the gate acts
 * on).  CNOT = SV_X with one control, Toffoli = SV_X with two, controlled
 * phase = SV_PHASE with one. */
sv_status sv_apply_controlled(sv_state st, sv_gate gate, const int* controls, int nc,
                              const int* targets, int nt, const double* params,
                              const double* matrix, int adjoint);

/* The general approach of Sec. 3.1: a dense 2^k x 2^k matrix-vector product
 * on every group of 2^k amplitudes that differ only in `qubits`, k in [1, 3],
 * with no use of the matrix's structure (CNOT as 4x4, Toffoli as 8x8).  The
 * baseline the gate-specific routines are measured against. */
sv_status sv_apply_general(sv_state st, const int* qubits, int k, const double* matrix);

/* A dense 2^k x 2^k unitary on k in [4, 6] qubits, on the matrix cores: the
 * fused dense block that stands for a run of gates on k qubits (Sec. 2's
 * logic-matrix application, one group of 2^k amplitudes per matrix-vector
 * product).  The complex product runs as a real one (FP64 MFMA for
 * complex128, FP32 MFMA for complex64), 8 * 2^k flops per amplitude.
 * qubits: k distinct indices < n, the first the most significant bit of the
 * matrix index (as in sv_apply_general).  matrix: host, row-major,
 * interleaved (re, im), 2 * 4^k doubles, read during the call (it is staged
 * in pinned memory and uploaded on the state's stream).  The state keeps a
 * 128 KiB device buffer and a 128 KiB pinned buffer from the first call
 * until sv_free.  Asynchronous on the state's stream, except that a call
 * waits for the previous call's upload to finish.
 * Errors: SV_ERR_ARG (k outside [4, 6], null matrix), SV_ERR_QUBIT (bad or
 * repeated qubits), SV_ERR_OOM (buffers), SV_ERR_HIP. */
sv_status sv_apply_dense(sv_state st, const int* qubits, int k, const double* matrix);

/* ------------------------------------------------------------------------
 * Measurement (Sec. 2: routines for "measurement processes"; Listing 1 takes
 * the expectation of a Hamiltonian).  All sums use fp64 with a fixed
 * two-stage order, so repeated calls return bit-identical values.
 * ------------------------------------------------------------------------ */

/* <psi|psi> into *out (host).  Synchronous. */
sv_status sv_norm2(sv_state st, double* out);

/* <psi|P|psi> of one Pauli string: paulis[j] in "IXYZ" acts on qubits[j],
 * n letters, distinct qubits.  Real part into *out (host).  Synchronous. */
sv_status sv_expval_pauli(sv_state st, const char* paulis, const int* qubits, int n, double* out);

/* A Pauli-sum observable sum_k coeffs[k] * P_k.  Term k is given by bit masks
 * over qubits: xmask[k] has the X and Y positions, zmask[k] the Z and Y
 * positions.  All three arrays are host arrays of n_terms entries.
 * Diagonal terms (xmask = 0) are evaluated together in one pass; the closed
 * forms sum_i Z_i and sum_i Z_i Z_{i+1} (unit coefficients) are recognised. */
typedef struct {
    int n_terms;
    const double* coeffs;
    const uint64_t* xmask;
    const uint64_t* zmask;
} sv_obs;

/* sum_k c_k <psi|P_k|psi> into *out (host).  Synchronous. */
sv_status sv_expval_obs(sv_state st, const sv_obs* obs, double* out);

/* Same value written to device memory out_dev (one double); asynchronous on
 * the state's stream.  The reduction partials live in a per-state device
 * workspace, allocated (or grown) on the first call that needs it. */
sv_status sv_expval_obs_dev(sv_state st, const sv_obs* obs, double* out_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the value
 * of sv_expval_obs_dev, computed by the same kernels in the same order
 * (bit-identical), with every intermediate in a static device array that
 * each GPU holds from the library's first use until the process ends
 * (512 KiB).  No hipMalloc, hipFree or other allocating device call is
 * made, and on success the host side allocates nothing either (only an
 * error's message does).
 * Limit: the observable may need at most 64 reduction passes (one per off-
 * diagonal term, one per 32 diagonal terms, one for sum Z_i or
 * sum Z_i Z_i+1); larger ones are rejected with SV_ERR_ARG before any device
 * work.  The state must live on the current device.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (different streams
 * or threads without ordering between them) race and give wrong values.
 * Asynchronous on the state's stream.
 * Errors: as sv_expval_obs_dev, SV_ERR_ARG for too many passes. */
sv_status sv_expval_obs_dev_noalloc(sv_state st, const sv_obs* obs, double* out_dev);

/* <psi|P|psi> of one Pauli string (as sv_expval_pauli) written to device
 * memory out_dev (one double); asynchronous on the state's stream, so it can
 * sit between gate launches without a host round trip.
 * Errors: as sv_expval_pauli, SV_ERR_ARG for a null out_dev. */
sv_status sv_expval_pauli_dev(sv_state st, const char* paulis, const int* qubits, int n, double* out_dev);

/* ------------------------------------------------------------------------
 * Circuits and adjoint differentiation (a project addition beyond the
 * paper, whose Listing 1 differentiates a circuit through autograd without
 * naming the method).  Method: Jones & Gacon 2020 (arXiv 2009.02823).
 * ------------------------------------------------------------------------ */

/* One operation of a circuit.  qubits[0 .. n_controls-1] are the controls,
 * the next n_targets entries the targets.  A rotation / PHASE angle is
 * params[param_index] when param_index >= 0, else `value`.  matrix: host
 * pointer for SV_U2 / SV_U4 (read when the circuit is created), else NULL. */
typedef struct {
    int32_t gate;
    int32_t n_controls;
    int32_t n_targets;
    int32_t param_index;
    int32_t qubits[SV_OP_MAX_QUBITS];
    double value;
    const double* matrix;
} sv_op;

/* Validate and copy an op list (matrices included) into a circuit object for
 * states of n_qubits.  Parameters are bound later, per run.  The circuit
 * holds a small device table of per-op gate coefficients. */
sv_status sv_circuit_create(int n_qubits, const sv_op* ops, int n_ops, int n_params, sv_circuit* out);
sv_status sv_circuit_free(sv_circuit c);

/* Apply the circuit to st (in place) with host parameters params[n_params]. */
sv_status sv_circuit_apply(sv_circuit c, sv_state st, const double* params);

/* As sv_circuit_apply, with every run of two or more consecutive diagonal
 * ops (Z, S, T, PHASE, RZ, any controls; identity) applied as one pass of
 * sv_apply_phases: one read and write of the touched amplitudes per run
 * instead of per gate (diagonal gates commute; Sec. 2's Z-type gates only
 * rescale amplitudes).  Consecutive uncontrolled one-target gates (X, Y, H,
 * RX, RY, U2) on one qubit are multiplied into one 2x2 on the host and
 * applied once; such a gate (or product) directly followed by a diagonal
 * run shares that run's pass: the QFT becomes one pass per target.  The
 * result equals sv_circuit_apply's within rounding (phases are summed as
 * angles, 2x2 products formed in double precision). */
sv_status sv_circuit_apply_fused(sv_circuit c, sv_state st, const double* params);

/* As sv_circuit_apply, with the circuit packed into dense blocks of at most
 * k qubits (k in [4, 6]) applied on the matrix cores (sv_apply_dense): a
 * block starts from the earliest unapplied op and absorbs ready ops (every
 * earlier op on their qubits already in a block; ops on disjoint qubits
 * commute) that grow its qubit set least, while it spans at most k qubits.
 * Each block's 2^k x 2^k matrix is formed on the host in double precision
 * from the parameters; a block of a single op runs that op's own kernel, and
 * blocks under 4 qubits are padded with further qubits.  The result equals
 * sv_circuit_apply's within rounding.  *n_dense_blocks (may be NULL)
 * receives the number of matrix-core blocks launched.
 * Errors: as sv_circuit_apply; SV_ERR_ARG for k outside [4, 6] or a state
 * of fewer than 4 qubits. */
sv_status sv_circuit_apply_blocks(sv_circuit c, sv_state st, const double* params, int k, int* n_dense_blocks);

/* Host-only: how sv_circuit_apply_blocks packs an op list (as given to
 * sv_circuit_create) for block size k.  info[0] dense blocks, info[1] ops
 * run alone, info[2] ops inside dense blocks (info[1] + info[2] = n_ops),
 * info[3] the widest block in qubits (before padding).  Errors: SV_ERR_ARG,
 * SV_ERR_QUBIT (bad or repeated qubits). */
sv_status sv_block_plan(int n_qubits, const sv_op* ops, int n_ops, int k, int64_t* info);

/* One pass of diagonal phases: psi[x] *= exp(i sum_t angles[t]) over the
 * terms t whose mask bits are all set in x (mask 0: every amplitude).  A
 * controlled phase on qubits S is the term (bits of S, phi).  Amplitudes
 * lacking a bit common to every mask are not touched.  n_terms in [1, 64];
 * masks and angles (radians) are host arrays read during the call; angles
 * at multiples of pi/2 give exact phases.  Asynchronous on the state's
 * stream.  Errors: SV_ERR_ARG (term count, null arrays), SV_ERR_QUBIT (a mask
 * bit at or above n). */
sv_status sv_apply_phases(sv_state st, int n_terms, const uint64_t* masks, const double* angles);

/* Adjoint gradient of E(th) = <psi(th)|O|psi(th)>, psi(th) = U(th)|psi_in>.
 * The op list comes as a circuit object (sv_circuit_create) rather than as a
 * raw sv_op array, so that validation and the per-op tables are built once
 * and reused across calls; outputs are host arrays (the batched form,
 * sv_batch_run, writes device outputs).
 * On entry psi holds |psi_in> (not modified in the end beyond rounding: the
 * reverse sweep un-applies every gate).  lam is a work state of the same size
 * and dtype (its contents are overwritten).  E goes to *expval_out and
 * dE/dparams[j] to grad_out[j] (host arrays, n_params entries; parameters used
 * by several ops get the sum).  The gradient of an op with generator G
 * (U = exp(-i th G / 2)) is Im <lambda|G|phi> at that op, as in the reference
 * method; PHASE uses its projector generator.  Synchronous.
 * Errors: as sv_circuit_apply, plus SV_ERR_ARG for a mismatched lam. */
sv_status sv_adjoint_grad(sv_circuit c, sv_state psi, sv_state lam, const double* params,
                          const sv_obs* obs, double* expval_out, double* grad_out);

/* ------------------------------------------------------------------------
 * Batched, fused execution (a project addition beyond the paper): many
 * independent circuits -- or one large one -- run as one hipGraph launch
 * (captured on first use and replayed): one kernel per stage level, one
 * workgroup per state tile, every circuit's tiles of a level together.
 *
 * Each circuit's ops are grouped into passes whose qubits fit one LDS tile
 * (2^12 complex128 or 2^13 complex64 amplitudes by default); ops on disjoint
 * qubits may move ahead of each other to fill a pass.  One pass moves the
 * state through HBM once, however many gates it holds.  A run executes, per
 * circuit: the forward passes from |0...0>, the expectation of a diagonal
 * observable, and (with_grad) the adjoint reverse sweep giving dE/dtheta for
 * every parameter (Jones & Gacon 2020).  The library owns every circuit's
 * state (and adjoint work state).
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_qubits;
    int32_t n_ops;
    const sv_op* ops;    /* host array, read during sv_batch_create */
    int32_t n_params;    /* parameters of this circuit; ops use indices 0..n_params-1 */
    int32_t obs_kind;    /* 1 = sum_i Z_i, 2 = sum_i Z_i Z_{i+1} */
} sv_batch_circuit;

typedef struct {
    int32_t tile_qubits; /* 0 = the engine shape (sv_tune_engine_set), else 2..13 */
    int32_t amps_per_thread; /* 0 = the engine shape; 8 or 16: amplitudes of a tile each thread
                              * holds in registers (workgroup = 2^tile_qubits / this, >= 64) */
    int32_t use_graph;   /* capture the run on first use, replay afterwards */
    int32_t with_grad;   /* also run the adjoint sweep */
} sv_batch_opts;

/* Validate, schedule and allocate a batch.  opts may be NULL (defaults,
 * use_graph = 1, with_grad = 1).  The batch runs on a stream of its own.
 * Errors: SV_ERR_ARG / SV_ERR_QUBIT (validation, nothing allocated),
 * SV_ERR_UNSUPPORTED (an op wider than a tile), SV_ERR_OOM. */
sv_status sv_batch_create(const sv_batch_circuit* circuits, int n_circuits, sv_dtype dtype,
                          const sv_batch_opts* opts, sv_batch* out);

/* Run the batch.  params: the circuits' parameters concatenated in circuit
 * order (sum of n_params doubles), in device memory if params_on_device.
 * expvals: n_circuits doubles; grads: sum of n_params doubles (with_grad
 * only); both in device memory if outputs_on_device.  Synchronous.
 * Ordering with the caller's stream (sv_batch_set_stream; the null stream
 * until set): the run starts after the work queued on that stream before the
 * call (which may still be writing params or clearing the outputs), and work
 * queued there afterwards sees the outputs.
 * Errors: SV_ERR_ARG, SV_ERR_HIP. */
sv_status sv_batch_run(sv_batch b, const double* params, int params_on_device, double* expvals, double* grads,
                       int outputs_on_device);

/* The caller's stream that sv_batch_run orders itself against (a hipStream_t;
 * NULL = the null stream).  The batch's kernels still run on its own stream.
 * Errors: SV_ERR_HANDLE. */
sv_status sv_batch_set_stream(sv_batch b, void* stream);

/* Host-only: validate and schedule a batch exactly as sv_batch_create would,
 * without any device work, and report its sv_batch_info figures. */
sv_status sv_batch_plan(const sv_batch_circuit* circuits, int n_circuits, sv_dtype dtype,
                        const sv_batch_opts* opts, int64_t* info);

/* info[0..11]: circuits, work items, passes, max passes per circuit, gate
 * ops scheduled, parameters, state bytes, algorithmic HBM bytes per run,
 * stage levels (each launches up to three kernels: forward, observable and
 * reverse items), LDS bytes per workgroup, layout changes in the forward
 * passes (each an LDS exchange of every tile), workgroup size of forward
 * passes. */
sv_status sv_batch_info(sv_batch b, int64_t* info);

/* Device pointer to a circuit's state (after a forward-only run: U|0...0>). */
sv_status sv_batch_state(sv_batch b, int circuit, void** dev_ptr, int* n_qubits);

/* Copy a circuit's state to host memory of exactly 2^n * element bytes.
 * Synchronous. */
sv_status sv_batch_copy_state(sv_batch b, int circuit, void* host, size_t bytes);
sv_status sv_batch_free(sv_batch b);

/* ------------------------------------------------------------------------
 * Launch shapes (written by the autotuner, read by every gate launch).
 * Kernel classes: 0 paired (permutation / butterfly / two-phase diagonal),
 * 1 subset phase, 2 retired (rejected), 3 two-target, 4 general, 5 paired with the
 * partner fetched across the lanes of a wavefront (targets 0..5), 6 staged
 * through LDS in whole contiguous chunks (general / U4 / SWAP whose lowest
 * qubit has runs under 1 KiB).  Tier: bytes spanned by
 * one run of consecutive touched amplitudes, 2^(lowest touched qubit) times
 * the element size: 0 (< 64 B), 1 (< 1 KiB), 2 (larger).  block is a
 * multiple of 64 in [64, 1024] (for class 6 an upper bound: a launch takes
 * one thread per 4 staged amplitudes for complex128 2-qubit matrices, per 2
 * for the complex128 SWAP move and per 8 otherwise, at least 64 threads and
 * at most block; sv_plan_info reports the block a launch takes); unroll is 1, 2 or 4: groups per thread,
 * and for class 6 the chunk elements a thread of a 3-qubit gate loads (and
 * stores) per round trip between HBM and LDS (2-qubit gates: two in
 * complex64 when unroll >= 2, else one; sv_plan_info reports the depth a
 * launch uses); nt = 1 makes the kernel's loads and stores non-temporal.  The table is
 * process-wide; set it from one thread before launching work.
 * Errors: SV_ERR_ARG for a bad key or shape.
 * ------------------------------------------------------------------------ */
sv_status sv_tune_set(int kernel_class, int dtype, int tier, int block, int unroll, int nt);
sv_status sv_tune_get(int kernel_class, int dtype, int tier, int* block, int* unroll, int* nt);

/* Order in which a gate launch's workgroups walk the state.  The hardware
 * deals consecutive workgroups to the 8 XCDs in turn; order 0 walks the
 * groups in launch order, order 1 gives each XCD one contiguous eighth of
 * them.  -1 (the default) picks per launch: order 1 for complex128 gates
 * with a member offset (a target bit) of 32..128 MiB, which run slower in
 * launch order (measured on MI355X), else order 0.  The environment variable
 * SV_BLOCK_ORDER=0 or 1, read at the first launch, forces an order until
 * this call changes it.  Results do not depend on the order: every group is
 * still touched once with the same arithmetic.  Process-wide; set it from
 * one thread before launching work.
 * Errors: SV_ERR_ARG for an order outside {-1, 0, 1}. */
sv_status sv_set_block_order(int order);
sv_status sv_get_block_order(int* order);

/* Engine tile shape (written by the autotuner, read by sv_batch_create and
 * sv_batch_plan where sv_batch_opts leaves tile_qubits or amps_per_thread at
 * 0), one per dtype and per stage mix: with_grad = 0 for forward-only
 * batches, 1 for batches that also run the adjoint sweep (its reverse
 * workgroups hold two states, so they favour other tiles).  tile_qubits 0 =
 * the built-in default, 12 for complex128 and 13 for complex64 (64 KiB
 * tiles), capped so that a workgroup holding one tile has at most 512
 * threads (complex128 reverse passes keep 8 amplitudes of each state per
 * thread; forward-only batches have no reverse workgroups, so complex128
 * tiles of 2^13 fit there); amps_per_thread 0 = 16.  Process-wide; set it from one thread
 * before creating batches; existing batches keep their shape.
 * sv_tune_engine_get reports the shape a batch with zeroed options gets.
 * Errors: SV_ERR_ARG for a bad dtype or with_grad, amps_per_thread not
 * 0/8/16, tile_qubits outside {0} U [2, 13] or too large for the thread
 * limit. */
sv_status sv_tune_engine_set(int dtype, int with_grad, int tile_qubits, int amps_per_thread);
sv_status sv_tune_engine_get(int dtype, int with_grad, int* tile_qubits, int* amps_per_thread);

/* Environment read by the library (each once, at first use):
 *   SV_BLOCK_ORDER=0|1  forces a workgroup walk order (sv_set_block_order);
 *   SV_FORCE_TIER=0|1|2 gives every gate launch the launch shape of that
 *                       tier (the kernel a gate runs is unchanged; other
 *                       values are ignored);
 * and by the Python binding at import: SV_TUNING_FILE=path loads that tuning
 * table instead of the one shipped beside the library ("none" loads none).
 * Determinism needs no switch: every reduction (norms, expectations,
 * gradient sums, the engine's per-tile partials) runs in a fixed order with
 * no floating-point atomics, so a call repeated on the same inputs with the
 * same launch shapes returns bit-identical results. */

/* Host-only report of how a gate would be launched on an n_qubits state of
 * `dtype`: kernel class, tier, operation code (the pair/subset operation;
 * for the general kernel, k; for class 6, 16 * k + (1 for SWAP, else 0)) and
 * the launch shape (tier: the one whose shape the launch takes, which
 * SV_FORCE_TIER overrides).  gate = -1 asks about the
 * general dense kernel on `targets` (nc must be 0).  No device work.
 * Errors: as sv_apply_controlled's validation; SV_ERR_ARG for SV_I. */
sv_status sv_plan_info(int n_qubits, int dtype, int gate, const int* controls, int nc, const int* targets, int nt,
                       int* kernel_class, int* tier, int* op, int* block, int* unroll, int* nt_flag);

/* ------------------------------------------------------------------------
 * Diagnostics
 * ------------------------------------------------------------------------ */

/* Measured HBM ceiling: a plain streaming kernel over `bytes` of device
 * memory with 16-byte non-temporal accesses, the yardstick the gate kernels'
 * bandwidth is compared against.  mode 0 copies src to dst (bytes read and
 * bytes written), 1 only reads src (a sum that is never stored unless it
 * hits an impossible value keeps the loads alive), 2 only writes dst (zeros),
 * 3 reads dst and writes it back negated in place (the access pattern of a
 * gate that touches every amplitude; src unused).
 * block: threads per workgroup (multiple of 64 in [64, 1024]); unroll: 16-byte
 * vectors per thread per workgroup tile (1, 2, 4 or 8).  bytes must be a
 * positive multiple of 16 and the used pointers 16-byte aligned.
 * Asynchronous on `stream` (NULL = the null stream): time it with events.
 * Errors: SV_ERR_ARG, SV_ERR_HIP. */
sv_status sv_stream_bench(int mode, void* dst, const void* src, size_t bytes, int block, int unroll, void* stream);
const char* sv_last_error(void);
const char* sv_status_string(sv_status s);
int sv_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SV_ABI_H_INCLUDED */
