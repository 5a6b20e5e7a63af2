// Internal declarations shared by the HIP kernel files and the host API of
// libqsv.so.  Not part of the public ABI (that is include/qsv.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <vector>

namespace qsv {

constexpr int kMaxIns = 40;      // inserted (fixed) bit positions per launch
constexpr int kBlock = 256;      // threads per block for streaming kernels
constexpr int kMaxTermsPerLaunch = 32;

enum Dt : int { C64 = 1, C128 = 2 };

// How a thread reads the amplitudes of one group (c64 only uses W2/INTRA):
//  W1    - one amplitude per load (float2 / double2);
//  W2    - c64, qubit 0 untouched by the gate: a float4 holds amplitudes 2u,
//          2u+1, which belong to two different groups with the same tau;
//  INTRA - c64, qubit 0 is the lowest target: a float4 holds tau' = 2v, 2v+1
//          of the same group.
enum Mode : int { W1 = 0, W2 = 1, INTRA = 2 };

enum LaunchType : int { L_DENSE = 0, L_DIAG = 1, L_PERM = 2, L_MFMA = 3, L_DIAGRUN = 4, L_QPERM = 5 };

constexpr int kMaxRunFactors = 32;  // diagonal gates merged into one L_DIAGRUN sweep
constexpr int kMaxRunEntries = kMaxRunFactors * 32;  // table entries of one run

// Rotation kinds read from a device parameter vector (values follow qsv_op_kind).
enum Rot : int { ROT_NONE = 0, ROT_X = 5, ROT_Y = 6, ROT_Z = 7 };

// Insert zero bits at ascending positions p (low[j] = 2^p - 1) into a group
// index, then OR in `setmask` (controls = 1).  All positions are in "unit"
// index space (amplitude index >> 1 for W2/INTRA).
struct InsertSpec {
    int nins;
    uint64_t setmask;
    uint64_t low[kMaxIns];
};

// A host-side description of one kernel launch on one (or two) states.
struct GateLaunch {
    int type = L_DENSE;
    int dt = C128;
    int n = 0;
    int K = 0;          // dense: #targets; diag: #varying targets; mfma: K; perm: unused
    int mode = W1;
    int lowq = 0;       // lowest qubit the launch touches (targets and controls)
    uint64_t ngroups = 0;
    InsertSpec ins{};
    uint64_t off[32] = {};   // dense: unit offset per tau' (INTRA: per tau'>>1); perm: dst
    uint64_t off2[32] = {};  // perm: src
    int nmoved = 0;
    int tpos[5] = {};        // diag: amplitude-space positions of varying targets (tau bit j)
    std::vector<double> g;   // dense: canonical matrix (complex128, row-major); diag: d[tau]
    const void* gdev = nullptr; // dense K>=4: matrix in state precision; mfma: A fragments
    int rot = ROT_NONE;
    int pidx = -1;
    int dag = 0;
    const double* params = nullptr; // device parameter vector (bound at run time)
    // mfma tile geometry
    int L = 0;
    uint64_t ntiles = 0;
    uint64_t choff[32] = {};
    int tloc[5] = {};
    int floc[6] = {};
    int mfma3 = 1;           // mfma: three-product kernel (0: real-embedding kernel)
    int mfma_tpb = 1;        // mfma: consecutive tiles per workgroup (1, 2 or 4)
    // diagonal run: amplitude i is multiplied by entry tau_f(i) of factor f's
    // table for every factor f with (i & run_fix[f]) == run_val[f]; tau_f bit j
    // = bit run_tpos[f][j] of i (run_nt[f] <= 5 varying bits).  The tables
    // (complex128, concatenated; factor f starts at complex entry run_off[f])
    // are uploaded in state precision and reached through gdev.
    int run_nf = 0;
    uint64_t run_fix[kMaxRunFactors] = {};
    uint64_t run_val[kMaxRunFactors] = {};
    int run_nt[kMaxRunFactors] = {};
    int run_tpos[kMaxRunFactors][5] = {};
    int run_off[kMaxRunFactors] = {};
    std::vector<double> run_tab;
    // a thread's units differ in unit bits run_w..run_w+3 (run_w >= 8); a
    // single-qubit gate on amplitude bit run_gt (one of the thread's varying
    // bits) may be applied in the same sweep, before (run_gate = 1) or after
    // (2) the diagonal, matrix run_g (canonical, complex128, row-major)
    int run_w = 8;
    int run_gate = 0;
    int run_gt = 0;
    double run_g[8] = {};
    // perm: the two qubits of an uncontrolled SWAP (-1: another permutation)
    int swapq[2] = {-1, -1};
    // qubit permutation pass: output amplitude j takes input amplitude i with
    // bit b of i = bit qp_q[b] of j (an involution); tiles of rows of 2^qp_rl
    // amplitudes at the offsets of the qp_hb tile bits qp_hpos (ascending),
    // zeros inserted at the tile bits by `ins`, one tile (or a tile and its
    // image) per workgroup, ngroups tiles; qp_cmap[k] is the tile-local bit of
    // the output that lands on tile-local bit k of the source.
    int qp_rl = 0;
    int qp_hb = 0;
    int qp_hpos[6] = {};
    int qp_cmap[12] = {};
    int qp_q[64] = {};
    int qp_wsrc[64] = {};  // bit p of the tile index = bit qp_wsrc[p] of the workgroup index
    uint64_t qmask = ~0ull;  // every qubit the launch reads or writes (targets and controls)
    // accounting
    double bytes = 0.0;
    double flops = 0.0;
};

// plan.cpp
// Merge runs of diagonal launches (no device parameters, at most two varying
// bits each) into L_DIAGRUN sweeps where a full sweep is cheaper than the
// separate launches' estimated traffic.
void merge_diagonal_runs(std::vector<GateLaunch>& Ls, std::vector<long long>& upload_off, int n, int dt);

// Apply a plain single-qubit gate next to a diagonal run in the run's sweep
// (L_DIAGRUN with run_gate set) where its target fits the run kernel.
void fold_gates_into_runs(std::vector<GateLaunch>& Ls, std::vector<long long>& upload_off, int n, int dt);

// Compose runs of consecutive SWAP launches into qubit permutation passes
// (L_QPERM, one or two per run) where that moves fewer bytes.
void merge_swaps(std::vector<GateLaunch>& Ls, std::vector<long long>& upload_off, int n, int dt);

// Row bits of the qubit permutation tiles: 512-byte rows in both precisions.
constexpr int kQpRowBitsC64 = 6;
constexpr int kQpRowBitsC128 = 5;

// kernels_qperm.hip (L_QPERM launches; psi2 may be NULL)
hipError_t launch_qperm(const GateLaunch& L, void* psi, void* psi2, hipStream_t s);

// kernels_diagrun.hip (L_DIAGRUN launches)
hipError_t launch_diag_run(const GateLaunch& L, void* psi, hipStream_t s);

// kernels_gate.hip
hipError_t launch_gate(const GateLaunch& L, void* psi, void* psi2, hipStream_t s);
hipError_t launch_init_basis(void* psi, int n, int dt, uint64_t index, hipStream_t s);
hipError_t launch_init_random(void* psi, int n, int dt, uint64_t seed, double* work, hipStream_t s);

// kernels_mfma.hip
hipError_t launch_mfma(const GateLaunch& L, void* psi, void* psi2, hipStream_t s);
// Fill the MFMA A-operand fragments of the real embedding of a canonical
// k-qubit complex128 matrix, in state precision (host side).
void mfma_fragments(const double* Gc, int K, int dt, std::vector<unsigned char>& out);
void mfma3_fragments(const double* Gc, int K, int dt, std::vector<unsigned char>& out);

// kernels_reduce.hip
int reduce_blocks(int n, int dt);
struct TermChunk {
    int nt;
    int ylo[kMaxTermsPerLaunch];          // number of Y factors mod 4
    uint64_t z[kMaxTermsPerLaunch];
    double c[kMaxTermsPerLaunch];
};
hipError_t launch_norm2(const void* psi, int n, int dt, double* partials, int accumulate, hipStream_t s);
hipError_t launch_expect_diag(const void* psi, int n, int dt, const TermChunk& t, double* partials,
                              int accumulate, hipStream_t s);
hipError_t launch_expect_pair(const void* psi, int n, int dt, uint64_t x, const TermChunk& t,
                              double* partials, int accumulate, hipStream_t s);
hipError_t launch_inner(const void* a, const void* b, int n, int dt, double* partials2,
                        int accumulate, hipStream_t s);
hipError_t launch_finalize(const double* partials, int nblocks, int ncomp, double* out, hipStream_t s);

// Device scratch of the allocation-free expectation (kernels_reduce.hip): a
// file-scope __device__ array of kStaticScratchBytes per GPU.  static_scratch
// returns the current device's address of it (looked up once per device with
// hipGetSymbolAddress; the array's name is not a device address on the host).
constexpr size_t kStaticScratchBytes = 32768;

// Staging of small host tables into device memory in stream order (a kernel
// whose arguments carry the bytes, kStageChunkBytes per launch); bytes and
// dst must be multiples of 16.
constexpr int kStageChunkBytes = 2048;
hipError_t launch_stage(void* dst, const void* host, size_t bytes, hipStream_t s);
hipError_t static_scratch(double** ptr);
hipError_t launch_hpsi_diag(const void* psi, void* lam, int n, int dt, const TermChunk& t,
                            int accumulate, hipStream_t s);
hipError_t launch_hpsi_pair(const void* psi, void* lam, int n, int dt, uint64_t x,
                            const TermChunk& t, hipStream_t s);
hipError_t launch_fill_zero(double* p, uint64_t count, hipStream_t s);

// kernels_measure.hip
size_t sample_workspace_doubles(int n);
size_t marginal_workspace_doubles();
hipError_t launch_sample(const void* psi, int n, int dt, const double* u, uint64_t seed, int seeded,
                         int64_t nshots, int64_t* out, double* work, hipStream_t s);
hipError_t launch_marginal(const void* psi, int n, int dt, const int* q, int m, double* out, double* work,
                           hipStream_t s);
hipError_t launch_collapse(void* psi, int n, int dt, const int* q, int m, uint64_t outcome,
                           const double* prob, hipStream_t s);
hipError_t launch_frequencies(const int64_t* samples, int64_t nshots, int n, const int* q, int m,
                              int64_t* counts, hipStream_t s);

// kernels_adjoint.hip
// One reverse step of the adjoint sweep for the rotation described by L (a
// dense K=1 launch with rot = ROT_X / ROT_Y, or a diag launch with
// rot = ROT_Z): partials[b] (b < nb) = block sums of Im <lam|P phi>, then
// phi and lam are replaced by U^dagger phi and U^dagger lam.
hipError_t launch_adj_step(const GateLaunch& L, void* phi, void* lam, double* partials, int nb,
                           hipStream_t s);
// grad[p] = sum over slots s with slot_param[s] == p (CSR: pstart/plist) of
// sum_b partials[s * nblocks + b].
hipError_t launch_grad_finalize(const double* partials, int nblocks, const int* pstart,
                                const int* plist, int nparams, double* grad, hipStream_t s);

}  // namespace qsv
