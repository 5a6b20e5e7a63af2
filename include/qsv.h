/*
 * qsv.h -- C ABI of the MI355X (gfx950) state-vector library libqsv.so.
 *
 * The library applies quantum gates to a 2^n-amplitude state vector held in
 * GPU memory, in place, following eq. (1) of Carrazza, Efthymiou, Lazzarin &
 * Pasquale, "An open-source modular framework for quantum computing" (Sec. 2):
 *
 *     psi'(tau, q) = sum_{tau'} G(tau, tau') psi(tau', q)
 *
 * where tau is the bitstring of the n_tar target qubits and q the bitstring of
 * the other n - n_tar qubits.  Around that core it provides controlled and
 * multi-qubit gates (Sec. 2, index generation for controlled and multi-target
 * gates), fused dense blocks of up to 5 qubits, expectation values of
 * Pauli-sum Hamiltonians (Sec. 3, Hamiltonian primitives), adjoint-method
 * gradients of parametrised rotation circuits (the gradient role Sec. 2
 * gives to automatic differentiation, Sec. 3 variational layers / VQE), a
 * batched mode that evaluates many small circuits in one persistent launch,
 * simulated measurement (marginal probabilities, shot sampling, outcome
 * frequencies; Sec. 3) and Trotterised time evolution of Pauli sums (Sec. 3).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - State layout: 2^n complex amplitudes, interleaved (re, im), amplitude i
 *    at element i.  QSV_C64 = 2 x float (8 bytes), QSV_C128 = 2 x double
 *    (16 bytes).  The pointer must be device memory, 16-byte aligned.
 *  - Qubit j is bit j of the amplitude index (weight 2^j).
 *  - Gate matrices are host arrays of complex128, row-major, interleaved:
 *    G[(row * 2^k + col) * 2 + {0: re, 1: im}].  For targets t[0..k-1] the
 *    FIRST listed target is the MOST significant bit of the row/column index
 *    (numpy kron order).  For QSV_C64 states every component is rounded to
 *    the nearest float before use.
 *  - Controlled gates apply G only to amplitudes whose control bits are all 1.
 *  - Every call validates all arguments on the host before it enqueues
 *    anything.  On error nothing is enqueued, device memory is unchanged and
 *    qsv_last_error() describes the problem.  Validation covers: 1 <= n <=
 *    QSV_MAX_QUBITS, dtype, 1 <= k <= QSV_MAX_TARGETS, c >= 0, k + c <= n,
 *    every qubit in [0, n), all targets and controls distinct, non-NULL
 *    pointers, 16-byte alignment of state pointers.
 *  - Device work is enqueued on `stream` (a hipStream_t passed as void*;
 *    NULL = the null stream) and calls never synchronise the device unless
 *    stated.  Results written to device memory are valid once the stream has
 *    reached them.
 *  - Ownership: every state, workspace and output buffer belongs to the
 *    caller; the library never frees it.  Host arrays are read only during
 *    the call.  Plans belong to the caller and are released with *_destroy.
 *  - Calls on different streams may run concurrently as long as they do not
 *    share buffers.  Library-internal caches are guarded by a mutex.
 *
 * Environment switches (read when a plan is created or a gate is launched;
 * results are the same with any setting, only the kernels differ):
 *    QSV_TUNE_CACHE=<file>      batch autotuner cache (JSON)
 *    QSV_BATCH_SHAPE=m,t[,s]    batch tile qubits, threads, split (skips the cache)
 *    QSV_NO_GRAPH=1             plans enqueue their launches instead of replaying a graph
 *    QSV_NO_MFMA=1              4- and 5-qubit blocks on the vector units
 *    QSV_MFMA_FORM=3m|real      matrix-core blocks as three real products (Gauss)
 *                               or one real-embedded product (default: three
 *                               products)
 *    QSV_MFMA_TPB=1|2|4         consecutive tiles per workgroup of the three-
 *                               product kernel (default: 4 at k = 5; at k = 4
 *                               2 for targets within 8 qubits, else 1)
 *    QSV_NO_DIAG_RUN=1          plans keep consecutive diagonal gates as separate launches
 *    QSV_NO_GATE_FOLD=1         plans keep single-qubit gates next to diagonal runs as
 *                               separate launches instead of applying them in the run's sweep
 *    QSV_NO_SWAP_MERGE=1        plans keep consecutive SWAP gates as separate launches
 *                               instead of qubit permutation passes
 *    QSV_NO_DIAG_DEFER=1        fusion (fuse_k >= 3) closes blocks at diagonal gates that
 *                               do not fit instead of deferring them past gates they
 *                               commute with
 *    QSV_EXPECT_PLAN=reg|span   expectation values through register passes (with
 *                               LDS-tile or span passes for the rest) or span
 *                               passes alone (default: the cheaper plan)
 *    QSV_NO_SPAN_PASS=1         expectation strings no tile holds take one pass
 *                               per x mask instead of span passes
 *    QSV_NO_TILES=1             per-gate adjoint instead of cache-blocked tile programs
 *    QSV_NO_LANE_SWEEP=1        no cross-lane exchange for low single-qubit targets
 *    QSV_SWEEP_NT=0|1           force the nontemporal hint of sweeps off or on
 */
#ifndef QSV_H
#define QSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QSV_MAX_QUBITS 40
#define QSV_MAX_TARGETS 5
#define QSV_MAX_CONTROLS 4 /* per op inside a circuit; qsv_apply_gate takes any count */

typedef enum { QSV_C64 = 1, QSV_C128 = 2 } qsv_dtype;

typedef enum {
    QSV_OK = 0,
    QSV_ERR_ARG = 1,         /* bad pointer, size, dtype or count */
    QSV_ERR_QUBIT = 2,       /* qubit index out of range or repeated */
    QSV_ERR_UNSUPPORTED = 3, /* valid request the library does not implement */
    QSV_ERR_HIP = 4,         /* HIP runtime or launch failure (message has the HIP string) */
    QSV_ERR_NOMEM = 5        /* host or device allocation failed */
} qsv_status;

/* Description of the last error on the calling thread; valid until the next
 * qsv_* call on that thread.  Never NULL. */
const char* qsv_last_error(void);

/* Library version string, e.g. "qsv 0.1 gfx950". */
const char* qsv_version(void);

/* ------------------------------------------------------------------ states */

/* Bytes of a state of n qubits: 2^n * (8 | 16).  The state is 2^n complex
 * numbers (Sec. 1, memory of Schroedinger-style simulation). */
qsv_status qsv_state_bytes(int n, qsv_dtype dt, size_t* bytes);

/* Convenience allocation for C callers (hipMalloc); Python callers pass torch
 * memory instead.  Free with qsv_state_free. */
qsv_status qsv_state_alloc(int n, qsv_dtype dt, void** psi);
qsv_status qsv_state_free(void* psi);

/* psi = |index>: amplitude `index` = 1, every other amplitude = +0.
 * index < 2^n. */
qsv_status qsv_init_basis(void* psi, int n, qsv_dtype dt, uint64_t index, void* stream);

/* Seeded synthetic state used by tests and benchmarks (not from the paper):
 * amplitude i = s * ((u(i,0) - 1/2) + i (u(i,1) - 1/2)), where
 * u(i,j) = (D(2i+j) >> 11) * 2^-53 and D(c) is draw c of the seed's
 * counter-based SplitMix64 stream (Steele, Lea & Flood 2014): with f the
 * generator's output function at a state and gamma = 0x9E3779B97F4A7C15,
 * key = f(seed) and D(c) = f(key + c * gamma) -- the outputs of the
 * generator restarted at its own first output, so nearby seeds give
 * unrelated states -- and s = 1 / sqrt(sum_i |raw_i|^2) (FP64 sum).
 * Values are computed in FP64 and rounded to the state's precision.  `work`
 * is a device buffer of qsv_reduce_workspace_bytes() bytes. */
qsv_status qsv_init_random(void* psi, int n, qsv_dtype dt, uint64_t seed, void* work, void* stream);

/* ------------------------------------------------------ gate application */

/* Apply the k-target gate G (host, complex128, 2^k x 2^k, see conventions),
 * controlled on `controls` (c entries, may be NULL when c == 0), to psi in
 * place: eq. (1) for every bitstring q of the non-target qubits whose control
 * bits are 1 (Sec. 2).  G need not be unitary.  The library recognises exact
 * 0/1 permutation matrices (moved bit-exactly, no arithmetic) and diagonal
 * matrices (only entries != 1 are touched), and uses MFMA matrix cores for
 * uncontrolled k = 4, 5.  k <= 5; c any (k + c <= n).  For k >= 4 the
 * matrix (or its matrix-core fragments) is staged into a small per-stream
 * device ring by a kernel on `stream` whose arguments carry the bytes: the
 * host never waits for the device, and the ring slot is reused in stream
 * order.  The first such call on a stream allocates the ring (256 KiB). */
qsv_status qsv_apply_gate(void* psi, int n, qsv_dtype dt, const int* targets, int k,
                          const int* controls, int c, const double* G, void* stream);

/* One dense block of a fused circuit: eq. (1) with a k-qubit matrix M (host,
 * complex128, conventions above), k <= 5, no controls (fold them into M). */
typedef struct {
    int k;
    int targets[QSV_MAX_TARGETS];
    const double* M;
} qsv_block;

/* Apply nblocks blocks in order.  Block matrices are staged to device memory
 * as for qsv_apply_gate (stream-ordered staging kernels, no host wait) before
 * the kernels that use them.  Not capturable into a HIP graph (use a plan
 * instead). */
qsv_status qsv_apply_fused(void* psi, int n, qsv_dtype dt, const qsv_block* blocks, int nblocks,
                           void* stream);

/* ---------------------------------------------------------- observables */

/* H = sum_j coeff[j] P_j (Sec. 3, Hamiltonian objects), each Pauli string
 * given by masks: qubit q carries X if only bit q of x_mask is set, Z if only
 * bit q of z_mask is set, Y if both, I if neither.  Host arrays, nterms >= 1.
 * Bits at or above n must be 0. */
typedef struct {
    int nterms;
    const uint64_t* x_mask;
    const uint64_t* z_mask;
    const double* coeff;
} qsv_pauli_sum;

/* Size in bytes of the scratch buffer used by reductions
 * (qsv_norm2, qsv_expectation, qsv_inner, qsv_init_random). */
qsv_status qsv_reduce_workspace_bytes(size_t* bytes);

/* out_dev[0] = sum_i |psi_i|^2, accumulated in FP64 in a fixed order
 * (deterministic for a given n).  out_dev: 1 double, device. */
qsv_status qsv_norm2(const void* psi, int n, qsv_dtype dt, double* out_dev, void* work,
                     void* stream);

/* out_dev[0] = Re <psi|H|psi>, out_dev[1] = Im (a rounding diagnostic; 0 in
 * exact arithmetic for real coefficients; terms taken by the register and
 * span passes below add exactly 0 to it), accumulated in FP64 in a fixed
 * order (Sec. 3, expectation values of Hamiltonians given as sums of Pauli
 * strings).  For n >= 12 the strings are read in passes of one state read
 * each, the cheapest of three plans by a cost measured per dtype:
 * register-tile passes (diagonal strings and strings whose x mask is one or
 * two neighbouring qubits of a five-qubit register set, or of qubits 0..4)
 * with 12-qubit LDS-tile passes or span passes for the rest, or span passes
 * alone (any x mask: five masks with a qubit above 5 per pass, strings on
 * qubits 0..5 and diagonal strings spread over them).  The environment
 * variable QSV_EXPECT_PLAN=reg or =span restricts the choice (comparisons);
 * QSV_NO_SPAN_PASS=1 replaces span passes by one pass per x mask.
 * qsv_expectation_launches reports the launch count.  out_dev: 2 doubles,
 * device. */
qsv_status qsv_expectation(const void* psi, int n, qsv_dtype dt, const qsv_pauli_sum* H,
                           double* out_dev, void* work, void* stream);

/* Number of kernel launches qsv_expectation (and qsv_expectation_noalloc)
 * enqueue for H on an n-qubit state: one per pass over the state (each pass
 * reads it once) plus the final reduction.  Host only; nothing is enqueued. */
qsv_status qsv_expectation_launches(const qsv_pauli_sum* H, int n, qsv_dtype dt, int* nlaunches);

/* qsv_expectation without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * qsv_expectation minus `work`: the partial sums live in a static device
 * array of 32 KiB that each GPU holds from the library's first call on it
 * until the process ends; the call allocates nothing and enqueues no memset
 * (the first pass overwrites the slots it needs).  Every call on one GPU
 * shares that array: calls that overlap in time on one GPU (different
 * streams, or host threads) race and must be serialised by the caller.
 * Every n up to QSV_MAX_QUBITS fits (at most 2 x 1024 partial sums);
 * QSV_ERR_UNSUPPORTED would report a state needing more. */
qsv_status qsv_expectation_noalloc(const void* psi, int n, qsv_dtype dt, const qsv_pauli_sum* H,
                                   double* out_dev, void* stream);

/* out_dev[0..1] = <a|b> (re, im) in FP64. */
qsv_status qsv_inner(const void* a, const void* b, int n, qsv_dtype dt, double* out_dev,
                     void* work, void* stream);

/* out = H psi (out and psi distinct device states of the same n and dtype). */
qsv_status qsv_apply_pauli_sum(const void* psi, void* out, int n, qsv_dtype dt,
                               const qsv_pauli_sum* H, void* stream);

/* ---------------------------------------------------------- measurement */

/* Simulated measurement (Sec. 3: measurement outcomes are sampled from the
 * state).  Outcome i has Born weight |psi_i|^2; no normalisation is applied,
 * the state's own norm is the total mass.  Weights and sums are FP64. */

/* Size in bytes of the scratch buffer qsv_probabilities and qsv_sample need
 * for an n-qubit state (about 2^(n-8) doubles, at least 8 MiB; 32 MiB at
 * n = 30). */
qsv_status qsv_measure_workspace_bytes(int n, qsv_dtype dt, size_t* bytes);

/* Marginal distribution of the m distinct qubits qubits[0..m-1] (host array,
 * 1 <= m <= n): out_dev[b] = sum of |psi_i|^2 over every i whose bits at
 * qubits[0..m-1] spell b, qubits[0] being the MOST significant bit of b (the
 * order of gate targets).  out_dev: 2^m doubles, device.  Every entry is
 * summed in a fixed order (deterministic).  Errors: as for gates
 * (QSV_ERR_ARG for m outside [1, n], QSV_ERR_QUBIT for a repeated or
 * out-of-range qubit), NULL out_dev or work. */
qsv_status qsv_probabilities(const void* psi, int n, qsv_dtype dt, const int* qubits, int m,
                             double* out_dev, void* work, void* stream);

/* Whole-register outcomes by inverse-transform sampling.  With the running
 * sums C_i = sum_{j <= i} |psi_j|^2 and T = C_(2^n - 1), shot s takes
 * t = u_dev[s] * T and returns out_dev[s] = the smallest i with C_i > t, or,
 * if there is none (t >= T: rounding, u >= 1 or NaN), the last outcome of
 * nonzero probability (0 for the zero vector); u < 0 counts as 0.  So an
 * outcome of zero probability is never returned.  u_dev: nshots uniforms in
 * [0, 1) (device, FP64, supplied by the caller, which owns the random
 * stream); out_dev: nshots int64, device.  The running sums are formed in a
 * fixed two-level order; an outcome can differ from a sequential running sum
 * only when t lies within rounding of a boundary C_i.  nshots == 0 enqueues
 * nothing; nshots < 0 is QSV_ERR_ARG. */
qsv_status qsv_sample(const void* psi, int n, qsv_dtype dt, const double* u_dev, int64_t nshots,
                      int64_t* out_dev, void* work, void* stream);

/* qsv_sample with the uniforms drawn on the device from the seed's
 * counter-based stream: u[s] = (D(s) >> 11) / 2^53 with D as for
 * qsv_init_random (SplitMix64: Steele, Lea & Flood 2014), so no uniform
 * array is needed. */
qsv_status qsv_sample_seeded(const void* psi, int n, qsv_dtype dt, uint64_t seed, int64_t nshots,
                             int64_t* out_dev, void* work, void* stream);

/* Frequencies of shot outcomes over the m distinct qubits qubits[0..m-1]
 * (host array, 1 <= m <= min(n, 30)): counts_dev[b] = number of shots s whose
 * outcome samples_dev[s] (whole-register indices, e.g. from qsv_sample) has
 * bits qubits[0..m-1] spelling b, qubits[0] the MOST significant bit of b.
 * samples_dev: nshots int64, device; counts_dev: 2^m int64, device, zeroed by
 * the call itself (also for nshots == 0).  Only the measured bits of a sample
 * are read.  Integer counts: the result is exact and deterministic.  Errors:
 * as for qsv_probabilities, QSV_ERR_UNSUPPORTED for m > 30, nshots < 0. */
qsv_status qsv_frequencies(const int64_t* samples_dev, int64_t nshots, int n, const int* qubits, int m,
                           int64_t* counts_dev, void* stream);

/* State after a measurement (Sec. 3: measurements; projective collapse):
 * for the outcome `outcome` of the m distinct qubits qubits[0..m-1]
 * (qubits[0] the MOST significant bit of the outcome), amplitudes whose bits
 * at those qubits spell the outcome are divided by sqrt(prob_dev[0]) and every
 * other amplitude is set to 0, in place.  prob_dev: 1 double, device (e.g. the
 * outcome's entry of qsv_probabilities, so the call needs no host round
 * trip); prob_dev[0] <= 0 leaves the zero vector.  Errors: as for
 * qsv_probabilities, QSV_ERR_ARG for an outcome >= 2^m or a NULL prob_dev. */
qsv_status qsv_collapse(void* psi, int n, qsv_dtype dt, const int* qubits, int m, uint64_t outcome,
                        const double* prob_dev, void* stream);

/* ------------------------------------------------------------- circuits */

/* Gate kinds (Sec. 3: circuits of 1-, 2- and 3-qubit gates).  Rotations are
 * R_P(theta) = exp(-i theta P / 2) with theta = params[param]:
 *   RX = [[c, -i s], [-i s, c]], RY = [[c, -s], [s, c]],
 *   RZ = diag(e^{-i theta/2}, e^{i theta/2}), c = cos(theta/2), s = sin(theta/2).
 * H = [[1,1],[1,-1]]/sqrt 2; X, Y, Z the Pauli matrices; SWAP on 2 targets;
 * MATRIX uses M (k targets).  Any kind may carry controls (CNOT = X with one
 * control, CZ = Z with one control, CRZ = RZ with one control). */
typedef enum {
    QSV_OP_MATRIX = 0,
    QSV_OP_H = 1,
    QSV_OP_X = 2,
    QSV_OP_Y = 3,
    QSV_OP_Z = 4,
    QSV_OP_RX = 5,
    QSV_OP_RY = 6,
    QSV_OP_RZ = 7,
    QSV_OP_SWAP = 8
} qsv_op_kind;

typedef struct {
    int kind;                          /* qsv_op_kind */
    int k;                             /* number of targets */
    int targets[QSV_MAX_TARGETS];
    int c;                             /* number of controls */
    int controls[QSV_MAX_CONTROLS];
    int param;                         /* rotations: index into params; else -1 */
    const double* M;                   /* QSV_OP_MATRIX: host complex128 2^k x 2^k */
} qsv_op;

typedef struct {
    int n;
    int nops;
    const qsv_op* ops;
    int nparams; /* length of the parameter vector */
} qsv_circuit;

typedef struct qsv_plan qsv_plan;

/* Compile a circuit into launches.  Gates are fused into dense blocks of at
 * most fuse_k qubits (1..5; 1 = no fusion) wherever every qubit of the gate,
 * targets and controls, fits the block; gates on disjoint qubits may be
 * reordered.  If params_host is non-NULL, rotation angles are bound now and
 * rotations fuse like any other gate; otherwise rotations stay separate
 * launches that read their angle from params_dev at run time.  Matrices are
 * copied to plan-owned device memory (this call synchronises the device). */
qsv_status qsv_plan_create(const qsv_circuit* circ, qsv_dtype dt, int fuse_k,
                           const double* params_host, qsv_plan** plan);

/* Apply the plan to psi in place.  params_dev (device, nparams doubles) is
 * read only by unbound rotations (may be NULL if there are none).  The first
 * run for a given (psi, params_dev, stream) records the launches into a HIP
 * graph that later runs replay (disable with the environment variable
 * QSV_NO_GRAPH=1).  A plan without launches (empty or all-identity circuit)
 * enqueues nothing. */
qsv_status qsv_plan_run(qsv_plan* plan, void* psi, const double* params_dev, void* stream);

/* Launch count, algorithmic HBM bytes (each touched amplitude read and
 * written once) and algorithmic flops of one run. */
qsv_status qsv_plan_info(const qsv_plan* plan, int* nlaunches, double* bytes, double* flops);

qsv_status qsv_plan_destroy(qsv_plan* plan);

/* Trotterised time evolution (Sec. 3: Hamiltonian objects interfaced with a
 * time-evolution solver through the Trotter decomposition).  Compiles `steps`
 * steps of length tau approximating exp(-i steps tau H), H = sum_j c_j P_j,
 * into a plan (run, info and destroy as for qsv_plan_create).  Each factor
 * exp(-i theta P_j) = cos(theta) I - i sin(theta) P_j is a dense gate on the
 * support of P_j (an identity string is the global phase exp(-i theta)).
 * order 1: per step, terms j = 0..T-1 with theta = tau c_j.  order 2
 * (symmetric): terms 0..T-1 then T-1..0, each with theta = tau c_j / 2, so
 * the step with -tau is the exact inverse of the step with tau.  Factors
 * fuse into blocks of at most fuse_k qubits like circuit gates.  Errors:
 * QSV_ERR_ARG for steps < 0, order not 1 or 2, non-finite tau or a bad Pauli
 * sum; QSV_ERR_UNSUPPORTED for a term on more than QSV_MAX_TARGETS qubits.
 * steps == 0 gives an empty plan. */
qsv_status qsv_trotter_plan_create(const qsv_pauli_sum* H, int n, double tau, int steps, int order,
                                   qsv_dtype dt, int fuse_k, qsv_plan** plan);


/* ------------------------------------------------------------ gradients */

typedef struct qsv_adjoint_plan qsv_adjoint_plan;

/* Prepare E(theta) = <psi(theta)|H|psi(theta)>, psi(theta) = U_N..U_1|0..0>,
 * and its gradient by the adjoint method (Jones & Gacon 2020): one forward
 * sweep, lambda = H psi, then one reverse sweep that uncomputes both vectors
 * with U_k^dagger and reads g_k = Im <lambda_k| P_k |psi_k> for every rotation
 * exp(-i theta P_k / 2) (controlled rotations: restricted to the
 * control-on subspace).  No per-gate checkpoints are kept.  Ops must be
 * unitary; parameters may be shared between ops (their terms add).
 * *work_bytes = size of the device workspace qsv_adjoint_run needs (two
 * states, FP64 partial sums and, for cache-blocked plans, the gate
 * descriptors each run stages from params_dev).  Runs that share one
 * workspace must not overlap in time.  fuse_k as in qsv_plan_create (applies
 * to runs of non-rotation gates). */
qsv_status qsv_adjoint_plan_create(const qsv_circuit* circ, const qsv_pauli_sum* H, qsv_dtype dt,
                                   int fuse_k, qsv_adjoint_plan** plan, size_t* work_bytes);

/* energy_dev[0] = E (FP64), grad_dev[0..nparams-1] = dE/dtheta (FP64),
 * both device.  params_dev: device, nparams doubles.  The states are swept in
 * the plan's dtype; every reduction accumulates in FP64. */
qsv_status qsv_adjoint_run(qsv_adjoint_plan* plan, const double* params_dev, void* work,
                           double* energy_dev, double* grad_dev, void* stream);

/* Forward sweep only: E into energy_dev, the final state into work's first
 * state slot (read it with qsv_adjoint_state). */
qsv_status qsv_adjoint_energy(qsv_adjoint_plan* plan, const double* params_dev, void* work,
                              double* energy_dev, void* stream);

/* Device pointer of the state slot inside work (slot 0 = psi, 1 = lambda). */
qsv_status qsv_adjoint_state(const qsv_adjoint_plan* plan, void* work, int slot, void** psi);

qsv_status qsv_adjoint_plan_destroy(qsv_adjoint_plan* plan);

/* One-shot form of qsv_adjoint_plan_create + qsv_adjoint_run + destroy, with
 * the same arguments and results.  work: device, 256-byte aligned,
 * work_bytes >= the *work_bytes qsv_adjoint_plan_create reports for the same
 * (circ, H, dt, fuse_k); a smaller buffer is QSV_ERR_ARG before anything is
 * enqueued.  The plan's device memory is released at the end of the call, so
 * the call host-synchronises `stream` (unlike every other call) and is not
 * capturable; a failed synchronisation is QSV_ERR_HIP. */
qsv_status qsv_adjoint_gradient(const qsv_circuit* circ, const double* params_dev,
                                const qsv_pauli_sum* H, qsv_dtype dt, int fuse_k, void* work,
                                size_t work_bytes, double* energy_dev, double* grad_dev,
                                void* stream);

/* --------------------------------------------------------------- batches */

typedef struct qsv_batch_plan qsv_batch_plan;

/* Many independent (circuit, Hamiltonian) instances of uneven size
 * (n <= QSV_BATCH_MAX_QUBITS; single-target gates with at most 2 controls;
 * rotations as for the adjoint plan) evaluated together: energies and adjoint
 * gradients of all instances.  Instances below a split size run in one
 * persistent kernel launch, one workgroup per instance, taken from a queue
 * largest first: those whose two state vectors fit the workgroup's LDS tile
 * stay there for the whole evaluation, the others stream cache-blocked tiles
 * of their own workspace region.  Instances at or above the split size (16 or
 * more qubits) run across the whole GPU with the cache-blocked adjoint, on
 * three side streams that the plan owns (created on the device current at
 * plan creation, default priority): qsv_batch_run forks them from `stream`
 * with an event before the persistent launch (which replays through a HIP
 * graph) and joins them back after, so the tiers and the large instances
 * overlap and every result is ready when `stream` reaches the end of the
 * call's work.  Calls with one plan must not overlap in time.  The tile
 * size, workgroup size and split size come
 * from the autotuner (qsv_batch_tune) or its cache.  Parameters and
 * gradients of instance i live at offsets[i] .. offsets[i+1]-1 of the
 * concatenated vectors (qsv_batch_offsets).  *work_bytes = workspace size. */
#define QSV_BATCH_MAX_QUBITS 24  /* and at least 3 qubits per instance */
qsv_status qsv_batch_plan_create(const qsv_circuit* circs, const qsv_pauli_sum* Hs, int ninst,
                                 qsv_dtype dt, qsv_batch_plan** plan, size_t* work_bytes);

/* offsets: ninst + 1 int64 entries (host). */
qsv_status qsv_batch_offsets(const qsv_batch_plan* plan, int64_t* offsets);

/* energies_dev: ninst doubles; grads_dev: offsets[ninst] doubles (device). */
qsv_status qsv_batch_run(qsv_batch_plan* plan, const double* params_dev, void* work,
                         double* energies_dev, double* grads_dev, void* stream);

/* Autotuner: times candidate shapes on this batch with these inputs (tile
 * qubits = the largest instance kept wholly in LDS, workgroup size, then the
 * split size of the large tier), keeps the fastest, and records it in the
 * JSON cache named by QSV_TUNE_CACHE (if set).  Synchronises the stream.
 * chosen (optional, host, 3 ints) receives (tile qubits, threads, split). */
qsv_status qsv_batch_tune(qsv_batch_plan* plan, const double* params_dev, void* work,
                          double* energies_dev, double* grads_dev, void* stream, int* chosen);

qsv_status qsv_batch_plan_destroy(qsv_batch_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* QSV_H */
