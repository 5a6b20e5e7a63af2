// Batched energies and adjoint gradients of many small rotation circuits in
// one persistent launch.
//
// Workgroups take instances from an atomic queue (largest first) and run each
// instance start to finish; no workgroup ever waits for another, so every
// wave reaches the exit once the queue is empty.
//
// An instance runs as a list of passes.  A pass has a set B of m qubits (the
// tile) and a list of single-target gates whose targets and controls all lie
// in B.  If n <= m the state pair (psi, lambda) lives in LDS for the whole
// instance.  Otherwise psi and lambda live in the instance's region of the
// workspace and each pass streams the 2^(n-m) tiles once: load a tile into
// LDS (chunks of contiguous low qubits, 16-byte accesses), apply every gate
// of the pass to it, store it.  Gates act locally inside a tile because all
// their qubits are tile bits, so a pass replaces one state sweep per gate by
// one sweep per pass (cache blocking).
//
// Inside a tile the pass runs as steps of gates on <= 3 qubits (tile_exec.h):
// each thread holds a step's 8 amplitudes in registers and applies all the
// step's gates before the next barrier.
//
// Forward passes apply U to psi; then lambda = H psi and E = Re <psi|lambda>;
// reverse passes walk the same schedule backwards applying U^dagger to psi
// and lambda and, for rotations exp(-i theta P / 2), add Im <lambda|P psi>
// (taken before the uncompute) to the parameter's gradient.  Per-gate partial
// sums are reduced in a fixed order and flushed once per pass, so results are
// deterministic.
#include "qsv_batch.h"
#include "tile_exec.h"

namespace qsv {
namespace {

using tx::ExecShared;
using tx::LOp;

// native 16-byte vector types (arrays of them stay in registers)
typedef float bv4f __attribute__((ext_vector_type(4)));
typedef double bv2d __attribute__((ext_vector_type(2)));

template <typename R>
struct BVec;
template <>
struct BVec<float> {
    using V = bv4f;  // two amplitudes
    static constexpr int APV = 2;
};
template <>
struct BVec<double> {
    using V = bv2d;  // one amplitude
    static constexpr int APV = 1;
};

struct C2d {
    double re, im;
};

template <typename R>
__device__ __forceinline__ C2d getc(const R* p, uint64_t l)
{
    return C2d{(double)p[2 * l], (double)p[2 * l + 1]};
}

template <typename R>
__device__ __forceinline__ void putc(R* p, uint64_t l, C2d v)
{
    p[2 * l] = (R)v.re;
    p[2 * l + 1] = (R)v.im;
}

// i^(y + 2 popcount(j & z))
__device__ __forceinline__ C2d pauli_phase(uint64_t j, const BTerm& t)
{
    const int e = (t.ylo + 2 * __popcll(j & t.z)) & 3;
    return C2d{e == 0 ? 1.0 : (e == 2 ? -1.0 : 0.0), e == 1 ? 1.0 : (e == 3 ? -1.0 : 0.0)};
}

struct BShared {
    int item;
    int pad;
    ExecShared ex;
    double pacc[kMaxPassOps];  // per-slot sums of a reverse pass
};

template <typename R, bool REV>
__device__ void run_pass(const BatchArgs& a, const BInst& I, const DPass& P, R* phiL, R* lamL,
                         LOp<R>* ops, DStep* steps, BShared& sm, R* phiG, R* lamG, double* grads,
                         int& parity)
{
    using V = typename BVec<R>::V;
    constexpr int APV = BVec<R>::APV;
    tx::stage<R>(P, a.steps, a.ops, a.mats, a.params + I.param_off, REV, ops, steps, sm.pacc);
    __syncthreads();
    // One loop for both tiers (a single inlined copy of the executor): the
    // LDS tier is one tile of n qubits that never leaves LDS.
    const bool lds_tier = I.n <= a.m;
    const int m = lds_tier ? I.n : a.m;
    const uint32_t nvec = lds_tier ? 0u : (1u << m) / APV;
    const uint64_t ntiles = lds_tier ? 1ull : (1ull << (I.n - m));
    V* pg = reinterpret_cast<V*>(phiG);
    V* lg = reinterpret_cast<V*>(lamG);
    V* pl = reinterpret_cast<V*>(phiL);
    V* ll = reinterpret_cast<V*>(lamL);
    // Vector v = threadIdx.x + blockDim.x * r sits at base | deposit(v * APV);
    // the tile bits are disjoint, so the deposit splits into a lane part and a
    // uniform part, and a thread moves its vectors in groups of kMove with
    // every load of a group in flight together.
    constexpr int kMove = 4;
    const uint32_t vpt = nvec / blockDim.x;  // nvec is a multiple of blockDim.x
    const uint64_t glane = lds_tier ? 0 : tx::deposit_mask((uint64_t)threadIdx.x * APV, P.bmask);
    for (uint64_t tile = 0; tile < ntiles; ++tile) {
        const uint64_t base = tx::insert_mask(tile, P.bmask);
        for (uint32_t r0 = 0; r0 < vpt; r0 += kMove) {
            V xp[kMove], xl[kMove];
#pragma unroll
            for (int u = 0; u < kMove; ++u)
                if (r0 + u < vpt) {
                    const uint64_t gi =
                        (base | glane | tx::deposit_mask((uint64_t)blockDim.x * APV * (r0 + u), P.bmask)) / APV;
                    xp[u] = pg[gi];
                    if (REV)
                        xl[u] = lg[gi];
                }
#pragma unroll
            for (int u = 0; u < kMove; ++u)
                if (r0 + u < vpt) {
                    pl[threadIdx.x + blockDim.x * (r0 + u)] = xp[u];
                    if (REV)
                        ll[threadIdx.x + blockDim.x * (r0 + u)] = xl[u];
                }
        }
        __syncthreads();
        // 16 amplitudes per thread need tiles of >= 16 (complex64 shapes only)
        bool wide = false;
        if constexpr (sizeof(R) == 4)
            wide = a.apt == 16 && m >= 4;
        if constexpr (sizeof(R) == 4) {
            if (wide)
                tx::exec_tile<R, REV, 16>(ops, steps, P.nsteps, m, phiL, lamL, sm.ex, sm.pacc, parity);
        }
        if (!wide)
            tx::exec_tile<R, REV, 8>(ops, steps, P.nsteps, m, phiL, lamL, sm.ex, sm.pacc, parity);
        for (uint32_t r = 0; r < vpt; ++r) {
            const uint32_t v = threadIdx.x + blockDim.x * r;
            const uint64_t gi =
                (base | glane | tx::deposit_mask((uint64_t)blockDim.x * APV * r, P.bmask)) / APV;
            pg[gi] = pl[v];
            if (REV)
                lg[gi] = ll[v];
        }
        __syncthreads();
    }
    if (REV) {
        __syncthreads();
        // flush the pass's per-slot sums into the gradient (one add per rotation)
        if (P.shared) {
            if (threadIdx.x == 0)
                for (int j = 0; j < P.nops; ++j) {
                    const DOp d = a.ops[P.op_off + j];
                    if (d.kind != 0)
                        grads[d.param] += sm.pacc[d.slot];
                }
        } else {
            for (int j = threadIdx.x; j < P.nops; j += blockDim.x) {
                const DOp d = a.ops[P.op_off + j];
                if (d.kind != 0)
                    grads[d.param] += sm.pacc[d.slot];
            }
        }
        __syncthreads();
    }
}

// lambda = H psi over the whole instance state, and the thread's share of
// Re <psi|lambda>.  (P psi)[i] = phase(i xor x) psi[i xor x].
template <typename R>
__device__ double hamiltonian_pass(const BatchArgs& a, const BInst& I, const R* phi, R* lam)
{
    const uint64_t N = 1ull << I.n;
    double e = 0.0;
    for (uint64_t i = threadIdx.x; i < N; i += blockDim.x) {
        C2d acc{0.0, 0.0};
        for (int t = 0; t < I.nterm; ++t) {
            const BTerm T = a.terms[I.term_off + t];
            const uint64_t j = i ^ T.x;
            const C2d ph = pauli_phase(j, T);
            const C2d v = getc(phi, j);
            acc.re += T.c * (ph.re * v.re - ph.im * v.im);
            acc.im += T.c * (ph.re * v.im + ph.im * v.re);
        }
        const C2d p = getc(phi, i);
        e += p.re * acc.re + p.im * acc.im;
        putc(lam, i, acc);
    }
    return e;
}

template <typename R>
__device__ void run_instance(const BatchArgs& a, int idx, R* phiL, R* lamL, LOp<R>* ops,
                             DStep* steps, BShared& sm)
{
    const BInst I = a.inst[idx];
    const uint64_t N = 1ull << I.n;
    double* grads = a.grads + I.param_off;
    for (int p = threadIdx.x; p < I.nparam; p += blockDim.x)
        grads[p] = 0.0;
    const bool lds_tier = I.n <= a.m;
    R* phiG = reinterpret_cast<R*>(a.work + I.work_off);
    R* lamG = phiG + 2 * N;
    R* phi = lds_tier ? phiL : phiG;
    R* lam = lds_tier ? lamL : lamG;
    for (uint64_t i = threadIdx.x; i < N; i += blockDim.x)
        putc(phi, i, C2d{i == 0 ? 1.0 : 0.0, 0.0});
    __syncthreads();
    int parity = 0;
    for (int p = 0; p < I.npass; ++p)
        run_pass<R, false>(a, I, a.passes[I.pass_off + p], phiL, lamL, ops, steps, sm, phiG, lamG,
                           grads, parity);
    __syncthreads();
    const double e = tx::wave_sum(hamiltonian_pass<R>(a, I, phi, lam));
    if ((threadIdx.x & 63) == 0)
        sm.ex.red[0][0][threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double E = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
            E += sm.ex.red[0][0][w];
        a.energies[idx] = E;
    }
    __syncthreads();
    parity = 0;
    for (int p = I.npass - 1; p >= 0; --p)
        run_pass<R, true>(a, I, a.passes[I.pass_off + p], phiL, lamL, ops, steps, sm, phiG, lamG,
                          grads, parity);
    __syncthreads();
}

template <typename R>
__global__ void __launch_bounds__(512) k_batch(const BatchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ BShared sm;
    const size_t tile = (size_t)2 * sizeof(R) << a.m;  // one complex tile
    R* phiL = reinterpret_cast<R*>(smem);
    R* lamL = reinterpret_cast<R*>(smem + tile);
    LOp<R>* ops = reinterpret_cast<LOp<R>*>(smem + 2 * tile);
    DStep* steps = reinterpret_cast<DStep*>(smem + 2 * tile + sizeof(LOp<R>) * kMaxPassOps);
    for (;;) {
        if (threadIdx.x == 0)
            sm.item = atomicAdd(a.counter, 1);
        __syncthreads();
        const int item = sm.item;
        __syncthreads();
        if (item >= a.ninst)
            break;
        run_instance<R>(a, a.order[item], phiL, lamL, ops, steps, sm);
    }
}

__global__ void k_zero_counter(int* c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *c = 0;
}

}  // namespace

size_t batch_lds_bytes(int dt, int m)
{
    const size_t R = dt == C64 ? 4 : 8;
    const size_t op = dt == C64 ? sizeof(LOp<float>) : sizeof(LOp<double>);
    return 2 * (2 * R << m) + (op + sizeof(DStep)) * kMaxPassOps;
}

int batch_resident_blocks(int dt, int m, int threads)
{
    int dev = 0, cus = 0, per = 0, maxlds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    const size_t lds = batch_lds_bytes(dt, m);
    if (lds + sizeof(BShared) > (size_t)maxlds)
        return 0;
    const void* fn = dt == C64 ? reinterpret_cast<const void*>(k_batch<float>)
                               : reinterpret_cast<const void*>(k_batch<double>);
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    hipError_t e = dt == C64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch<float>,
                                                                            threads, lds)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch<double>,
                                                                            threads, lds);
    if (e != hipSuccess)
        return 0;
    return per * cus;
}

hipError_t launch_batch(const BatchArgs& a, int dt, int threads, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, a.counter);
    const size_t lds = batch_lds_bytes(dt, a.m);
    if (dt == C64)
        hipLaunchKernelGGL(k_batch<float>, dim3(blocks), dim3(threads), lds, s, a);
    else
        hipLaunchKernelGGL(k_batch<double>, dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

}  // namespace qsv
