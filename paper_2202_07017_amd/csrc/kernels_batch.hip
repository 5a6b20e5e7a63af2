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
// Forward passes apply U to psi; then lambda = H psi and E = Re <psi|lambda>;
// reverse passes walk the same schedule backwards applying U^dagger to psi
// and lambda and, for rotations exp(-i theta P / 2), add Im <lambda|P psi>
// (taken before the uncompute) to the parameter's gradient.  Per-gate partial
// sums are reduced in a fixed order (wave shuffles, then thread 0 over the
// waves) and added by thread 0 only, so results are deterministic.
#include "qsv_batch.h"

namespace qsv {
namespace {

template <typename R>
struct BVec;
template <>
struct BVec<float> {
    using V = float4;
    static constexpr int APV = 2;
};
template <>
struct BVec<double> {
    using V = double2;
    static constexpr int APV = 1;
};

struct C2d {
    double re, im;
};

template <typename R>
struct LOp {                 // one staged gate of the current pass (LDS)
    R m[8];                  // 2x2 matrix, row-major (re, im): U or U^dagger
    uint64_t low[3];         // insertion masks (ascending local positions)
    uint32_t cmask;          // local control mask
    uint32_t tbit;           // local target bit value
    int16_t nins;
    int16_t gen;             // generator of a rotation: 5 = X, 6 = Y, 7 = Z; 0 = none
    int32_t param;           // instance-local parameter index (rotations)
};

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Matrix of a pass gate in FP64 (forward: U; reverse: U^dagger).
__device__ __forceinline__ void gate_matrix(const BPOp& po, const double* mats, const double* params,
                                            bool dag, double* m)
{
    if (po.kind == 0) {
        for (int j = 0; j < 8; ++j)
            m[j] = mats[(size_t)po.mat * 8 + j];
    } else {
        const double th = params[po.param];
        const double c = cos(0.5 * th), s = sin(0.5 * th);
        for (int j = 0; j < 8; ++j)
            m[j] = 0.0;
        m[0] = c;
        m[6] = c;
        if (po.kind == 5) {  // RX = [[c, -is], [-is, c]]
            m[3] = -s;
            m[5] = -s;
        } else if (po.kind == 6) {  // RY = [[c, -s], [s, c]]
            m[2] = -s;
            m[4] = s;
        } else {  // RZ = diag(c - is, c + is)
            m[1] = -s;
            m[7] = s;
        }
    }
    if (dag) {  // conjugate transpose
        double t[8];
        for (int j = 0; j < 8; ++j)
            t[j] = m[j];
        m[0] = t[0];
        m[1] = -t[1];
        m[2] = t[4];
        m[3] = -t[5];
        m[4] = t[2];
        m[5] = -t[3];
        m[6] = t[6];
        m[7] = -t[7];
    }
}

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

template <typename R>
__device__ __forceinline__ void apply2(const R* m, C2d& a, C2d& b)
{
    const C2d x = a, y = b;
    a.re = (double)m[0] * x.re - (double)m[1] * x.im + (double)m[2] * y.re - (double)m[3] * y.im;
    a.im = (double)m[0] * x.im + (double)m[1] * x.re + (double)m[2] * y.im + (double)m[3] * y.re;
    b.re = (double)m[4] * x.re - (double)m[5] * x.im + (double)m[6] * y.re - (double)m[7] * y.im;
    b.im = (double)m[4] * x.im + (double)m[5] * x.re + (double)m[6] * y.im + (double)m[7] * y.re;
}

// Im <lam|P phi> over one pair.
__device__ __forceinline__ double gen_term(int gen, C2d l0, C2d l1, C2d p0, C2d p1)
{
    if (gen == 5)
        return (l0.re * p1.im - l0.im * p1.re) + (l1.re * p0.im - l1.im * p0.re);
    if (gen == 6)
        return -(l0.re * p1.re + l0.im * p1.im) + (l1.re * p0.re + l1.im * p0.im);
    return (l0.re * p0.im - l0.im * p0.re) - (l1.re * p1.im - l1.im * p1.re);
}

// i^(y + 2 popcount(j & z))
__device__ __forceinline__ C2d pauli_phase(uint64_t j, const BTerm& t)
{
    const int e = (t.ylo + 2 * __popcll(j & t.z)) & 3;
    return C2d{e == 0 ? 1.0 : (e == 2 ? -1.0 : 0.0), e == 1 ? 1.0 : (e == 3 ? -1.0 : 0.0)};
}

struct Smem {
    int item;
    int pad;
    double red[2][16];  // per-wave partials, double-buffered by gate parity
};

template <typename R>
__device__ void stage_ops(const BatchArgs& a, const BInst& I, const BPass& P, bool dag, LOp<R>* ops)
{
    const double* params = a.params + I.param_off;
    for (int j = threadIdx.x; j < P.nops; j += blockDim.x) {
        const BPOp po = a.pops[P.op_off + j];
        double m[8];
        gate_matrix(po, a.mats, params, dag, m);
        LOp<R> o;
        for (int q = 0; q < 8; ++q)
            o.m[q] = (R)m[q];
        int pos[3] = {po.tloc, po.c0, po.c1};
        const int cnt = 1 + po.nc;
        for (int x = 0; x < cnt; ++x)  // sort ascending (cnt <= 3)
            for (int y = x + 1; y < cnt; ++y)
                if (pos[y] < pos[x]) {
                    const int t = pos[x];
                    pos[x] = pos[y];
                    pos[y] = t;
                }
        for (int x = 0; x < 3; ++x)
            o.low[x] = x < cnt ? ((1ull << pos[x]) - 1) : 0;
        o.nins = (int16_t)cnt;
        o.cmask = (po.nc > 0 ? 1u << po.c0 : 0u) | (po.nc > 1 ? 1u << po.c1 : 0u);
        o.tbit = 1u << po.tloc;
        o.gen = (int16_t)(po.kind == 0 ? 0 : po.kind);
        o.param = po.param;
        ops[j] = o;
    }
}

// Apply gate j of the staged pass to the LDS state(s) of 2^mb amplitudes.
// Reverse gates also accumulate the rotation's gradient partial.
template <typename R, bool REV>
__device__ void apply_op(const LOp<R>& o, int mb, R* phi, R* lam, int parity, Smem& sm,
                         double* grads)
{
    const uint32_t npairs = 1u << (mb - o.nins);
    const int gen = o.gen, param = o.param;  // read before the barrier below
    double acc = 0.0;
    for (uint32_t g = threadIdx.x; g < npairs; g += blockDim.x) {
        uint64_t l = g;
        for (int x = 0; x < o.nins; ++x)
            l = ((l & ~o.low[x]) << 1) | (l & o.low[x]);
        const uint32_t l0 = (uint32_t)l | o.cmask, l1 = l0 | o.tbit;
        C2d p0 = getc(phi, l0), p1 = getc(phi, l1);
        if constexpr (REV) {
            C2d q0 = getc(lam, l0), q1 = getc(lam, l1);
            if (gen)
                acc += gen_term(gen, q0, q1, p0, p1);
            apply2(o.m, q0, q1);
            putc(lam, l0, q0);
            putc(lam, l1, q1);
        }
        apply2(o.m, p0, p1);
        putc(phi, l0, p0);
        putc(phi, l1, p1);
    }
    if constexpr (REV) {
        if (gen) {
            acc = wave_sum(acc);
            if ((threadIdx.x & 63) == 0)
                sm.red[parity][threadIdx.x >> 6] = acc;
        }
    }
    __syncthreads();
    if constexpr (REV) {
        if (gen && threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
                s += sm.red[parity][w];
            grads[param] += s;
        }
    }
}

// Deposit the bits of l into the positions of mask (ascending).
__device__ __forceinline__ uint64_t deposit_mask(uint64_t l, uint32_t mask)
{
    uint64_t out = 0;
    int b = 0;
    for (uint32_t m = mask; m; m &= m - 1, ++b)
        if ((l >> b) & 1ull)
            out |= (uint64_t)(m & (~m + 1));
    return out;
}

// Insert zero bits at the positions of mask (ascending) into t.
__device__ __forceinline__ uint64_t insert_mask(uint64_t t, uint32_t mask)
{
    for (uint32_t m = mask; m; m &= m - 1) {
        const uint64_t lo = (uint64_t)(m & (~m + 1)) - 1;
        t = ((t & ~lo) << 1) | (t & lo);
    }
    return t;
}

template <typename R, bool REV>
__device__ void run_pass(const BatchArgs& a, const BInst& I, const BPass& P, R* phiL, R* lamL,
                         LOp<R>* ops, Smem& sm, R* phiG, R* lamG, double* grads)
{
    using V = typename BVec<R>::V;
    constexpr int APV = BVec<R>::APV;
    stage_ops<R>(a, I, P, REV, ops);
    __syncthreads();
    const bool lds_tier = I.n <= a.m;
    if (lds_tier) {
        if (!REV)
            for (int j = 0; j < P.nops; ++j)
                apply_op<R, false>(ops[j], I.n, phiL, lamL, j & 1, sm, grads);
        else
            for (int j = P.nops - 1; j >= 0; --j)
                apply_op<R, true>(ops[j], I.n, phiL, lamL, j & 1, sm, grads);
        return;
    }
    const int m = a.m;
    const uint32_t nvec = (1u << m) / APV;
    const uint64_t ntiles = 1ull << (I.n - m);
    V* pg = reinterpret_cast<V*>(phiG);
    V* lg = reinterpret_cast<V*>(lamG);
    V* pl = reinterpret_cast<V*>(phiL);
    V* ll = reinterpret_cast<V*>(lamL);
    for (uint64_t tile = 0; tile < ntiles; ++tile) {
        const uint64_t base = insert_mask(tile, P.bmask);
        for (uint32_t v = threadIdx.x; v < nvec; v += blockDim.x) {
            const uint64_t gi = (base | deposit_mask((uint64_t)v * APV, P.bmask)) / APV;
            pl[v] = pg[gi];
            if (REV)
                ll[v] = lg[gi];
        }
        __syncthreads();
        if (!REV)
            for (int j = 0; j < P.nops; ++j)
                apply_op<R, false>(ops[j], m, phiL, lamL, j & 1, sm, grads);
        else
            for (int j = P.nops - 1; j >= 0; --j)
                apply_op<R, true>(ops[j], m, phiL, lamL, j & 1, sm, grads);
        for (uint32_t v = threadIdx.x; v < nvec; v += blockDim.x) {
            const uint64_t gi = (base | deposit_mask((uint64_t)v * APV, P.bmask)) / APV;
            pg[gi] = pl[v];
            if (REV)
                lg[gi] = ll[v];
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
__device__ void run_instance(const BatchArgs& a, int idx, R* phiL, R* lamL, LOp<R>* ops, Smem& sm)
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
    for (int p = 0; p < I.npass; ++p)
        run_pass<R, false>(a, I, a.passes[I.pass_off + p], phiL, lamL, ops, sm, phiG, lamG, grads);
    __syncthreads();
    double e = wave_sum(hamiltonian_pass<R>(a, I, phi, lam));
    if ((threadIdx.x & 63) == 0)
        sm.red[0][threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double E = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
            E += sm.red[0][w];
        a.energies[idx] = E;
    }
    __syncthreads();
    for (int p = I.npass - 1; p >= 0; --p)
        run_pass<R, true>(a, I, a.passes[I.pass_off + p], phiL, lamL, ops, sm, phiG, lamG, grads);
    __syncthreads();
}

template <typename R>
__global__ void __launch_bounds__(1024) k_batch(const BatchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ Smem sm;
    const size_t tile = (size_t)2 * sizeof(R) << a.m;  // one complex tile
    R* phiL = reinterpret_cast<R*>(smem);
    R* lamL = reinterpret_cast<R*>(smem + tile);
    LOp<R>* ops = reinterpret_cast<LOp<R>*>(smem + 2 * tile);
    for (;;) {
        if (threadIdx.x == 0)
            sm.item = atomicAdd(a.counter, 1);
        __syncthreads();
        const int item = sm.item;
        __syncthreads();
        if (item >= a.ninst)
            break;
        run_instance<R>(a, a.order[item], phiL, lamL, ops, sm);
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
    return 2 * (2 * R << m) + op * kMaxPassOps;
}

int batch_resident_blocks(int dt, int m, int threads)
{
    int dev = 0, cus = 0, per = 0, maxlds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    const size_t lds = batch_lds_bytes(dt, m);
    if (lds + sizeof(Smem) > (size_t)maxlds)
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
    if (dt == C64) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_batch<float>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_batch<float>, dim3(blocks), dim3(threads), lds, s, a);
    } else {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_batch<double>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_batch<double>, dim3(blocks), dim3(threads), lds, s, a);
    }
    return hipGetLastError();
}

}  // namespace qsv
