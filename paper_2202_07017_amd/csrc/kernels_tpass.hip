// One cache-blocked pass of a tile program over a whole state (one launch per
// pass, tiles spread over the grid).
//
// k_tstage turns every gate of the program into its executor descriptor
// (matrix and form; forward U, then reverse U^dagger) once per run; the pass
// kernels read a pass's descriptors and steps from there through scalar
// loads.  Every block takes tiles tile = blockIdx.x, + gridDim.x, ...: loads
// the tile (psi; reverse passes also lambda) into LDS in contiguous chunks of
// 16-byte vectors (all of a thread's vectors in flight together, the next
// tile's while this one is processed), runs the pass's steps on it
// (tile_exec.h) and stores it back.  Reverse passes end by writing the
// block's per-rotation FP64 sums to partials[(slot_base + slot) * nb + block],
// which a finalize kernel adds in block order.
#include "qsv_tpass.h"
#include "tile_exec.h"

namespace qsv {
namespace {

using tx::ExecShared;
using tx::LOp;

typedef float tv4f __attribute__((ext_vector_type(4)));
typedef double tv2d __attribute__((ext_vector_type(2)));

template <typename R>
struct TV;
template <>
struct TV<float> {
    using V = tv4f;  // two amplitudes
    static constexpr int APV = 2;
};
template <>
struct TV<double> {
    using V = tv2d;  // one amplitude
    static constexpr int APV = 1;
};

// Threads per block NT: 8 amplitudes each, so a block holds a tile of
// 8 NT amplitudes (NT = 512, 256, 128 for complex64 tiles of 12, 11, 10
// qubits; 256, 128 for complex128 tiles of 11, 10).  Smaller tiles serve
// states too small to give every CU a tile of the full size.
template <typename R>
constexpr int tpass_max_threads()
{
    return sizeof(R) == 4 ? 512 : 256;
}

int tpass_threads_for(int dt, int m)
{
    const int hi = dt == C64 ? 512 : 256;
    const int nt = m >= 3 ? (1 << (m - 3)) : 1;
    return nt >= hi ? hi : (nt <= 128 ? 128 : nt);
}

// 16-byte vectors per thread per state: 8 amplitudes.
template <typename R>
constexpr int tpass_vpt()
{
    return sizeof(R) == 4 ? 4 : 8;
}

// Waves per SIMD to keep the resident blocks' waves within the register
// file: complex64 reverse passes fit two full-size tiles (or more smaller
// ones) in LDS, i.e. 16 waves per CU; 1 = no constraint.
template <typename R, bool REV>
constexpr int tpass_wpe()
{
    return (sizeof(R) == 4 && REV) ? 4 : 1;
}

template <typename R>
__global__ void __launch_bounds__(256) k_tstage(const DOp* __restrict__ ops, int nops,
                                                const double* __restrict__ mats,
                                                const double* __restrict__ params,
                                                LOp<R>* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 2 * nops)
        out[i] = tx::make_lop<R>(ops[i < nops ? i : i - nops], mats, params, i >= nops);
}

template <typename R, bool REV, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(tpass_wpe<R, REV>())))
    k_tpass(R* __restrict__ psi, R* __restrict__ lam, const LOp<R>* __restrict__ ops,
            const DStep* __restrict__ steps, const TPassArgs a)
{
    using V = typename TV<R>::V;
    constexpr int APV = TV<R>::APV;
    constexpr int NS = REV ? 2 : 1;  // states moved per tile
    constexpr int kTpassThreads = NT;
    constexpr int kVPT = tpass_vpt<R>();
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ ExecShared sh;
    const int m = a.m;
    const size_t tile = (size_t)2 * sizeof(R) << m;
    R* phiL = reinterpret_cast<R*>(smem);
    R* lamL = reinterpret_cast<R*>(smem + tile);
    double* pacc = reinterpret_cast<double*>(smem + 2 * tile);  // reverse passes
    const DPass P = a.pass;
    if (REV)
        for (int j = threadIdx.x; j < P.nrot; j += kTpassThreads)
            pacc[j] = 0.0;
    const uint32_t nvec = (1u << m) / APV;
    const uint64_t ntiles = 1ull << (a.n - m);
    V* const gs[2] = {reinterpret_cast<V*>(psi), reinterpret_cast<V*>(lam)};
    V* const ls[2] = {reinterpret_cast<V*>(phiL), reinterpret_cast<V*>(lamL)};
    // Vector v = threadIdx.x + kTpassThreads * r holds local amplitudes v * APV
    // (+ 1); its global index is base | deposit(v * APV).  The tile bits are
    // disjoint, so the deposit splits into a lane part and a uniform part.
    const uint64_t glane = tx::deposit_mask((uint64_t)threadIdx.x * APV, P.bmask);
    uint64_t greg[kVPT];
#pragma unroll
    for (int r = 0; r < kVPT; ++r)
        greg[r] = tx::deposit_mask((uint64_t)kTpassThreads * APV * r, P.bmask);
    V x[NS][kVPT];
    // (opaque copies of the lane offset keep the compiler from holding every
    // vector's global address in registers across the steps)
    auto load = [&](uint64_t t) {
        const uint64_t base = tx::insert_mask(t, P.bmask);
        uint64_t gl = glane;
        asm volatile("" : "+v"(gl));
#pragma unroll
        for (int r = 0; r < kVPT; ++r)
            if (threadIdx.x + kTpassThreads * r < nvec)
#pragma unroll
                for (int sidx = 0; sidx < NS; ++sidx)
                    x[sidx][r] = __builtin_nontemporal_load(gs[sidx] + (base | gl | greg[r]) / APV);
    };
    auto to_lds = [&]() {
#pragma unroll
        for (int r = 0; r < kVPT; ++r)
            if (threadIdx.x + kTpassThreads * r < nvec)
#pragma unroll
                for (int sidx = 0; sidx < NS; ++sidx)
                    ls[sidx][threadIdx.x + kTpassThreads * r] = x[sidx][r];
    };
    int parity = 0;
    uint64_t t = blockIdx.x;
    // Forward passes prefetch: the next tile's loads are issued before this
    // tile's steps, and its LDS copy is written at the end of the iteration,
    // after this tile's stores (vector memory counters retire in order, so
    // the wait for the loads then need not cover the stores); past the last
    // tile a block reloads its own tile, a copy that is never used.  Reverse
    // passes (two states: the prefetch registers would halve the resident
    // blocks) load each tile at the top of its iteration.
    constexpr bool PF = !REV;
    if (PF && t < ntiles) {
        load(t);
        to_lds();
    }
    for (; t < ntiles; t += gridDim.x) {
        const uint64_t base = tx::insert_mask(t, P.bmask);
        if (!PF) {
            load(t);
            to_lds();
        }
        __syncthreads();
        if (PF)
            load(t + gridDim.x < ntiles ? t + gridDim.x : t);
        tx::exec_tile<R, REV, 8, true>(ops, steps, P.nsteps, m, phiL, lamL, sh, pacc, parity);
        uint64_t gl = glane;
        asm volatile("" : "+v"(gl));
#pragma unroll
        for (int r = 0; r < kVPT; ++r)
            if (threadIdx.x + kTpassThreads * r < nvec)
#pragma unroll
                for (int sidx = 0; sidx < NS; ++sidx)
                    __builtin_nontemporal_store(ls[sidx][threadIdx.x + kTpassThreads * r],
                                                gs[sidx] + (base | gl | greg[r]) / APV);
        __syncthreads();
        if (PF)
            to_lds();
    }
    if (REV)
        for (int j = threadIdx.x; j < P.nrot; j += blockDim.x)
            a.partials[(size_t)(P.slot_base + j) * gridDim.x + blockIdx.x] = pacc[j];
}

template <typename R, bool REV>
const void* tpass_fn(int nt)
{
    if (nt == 512)
        return reinterpret_cast<const void*>(k_tpass<R, REV, (sizeof(R) == 4 ? 512 : 256)>);
    if (nt == 256)
        return reinterpret_cast<const void*>(k_tpass<R, REV, 256>);
    return reinterpret_cast<const void*>(k_tpass<R, REV, 128>);
}

template <typename R, bool REV, int NT>
hipError_t go_nt(const TPassArgs& a, void* psi, void* lam, int blocks, size_t lds, hipStream_t s)
{
    const LOp<R>* ops = static_cast<const LOp<R>*>(a.lops) + (REV ? a.nops_total : 0) + a.pass.op_off;
    hipLaunchKernelGGL((k_tpass<R, REV, NT>), dim3(blocks), dim3(NT), lds, s, static_cast<R*>(psi),
                       static_cast<R*>(lam ? lam : psi), ops, a.steps + a.pass.step_off, a);
    return hipGetLastError();
}

template <typename R, bool REV>
hipError_t go(const TPassArgs& a, void* psi, void* lam, int blocks, hipStream_t s)
{
    const int dt = sizeof(R) == 4 ? C64 : C128;
    const size_t lds = tpass_lds_bytes(dt, a.m, REV);
    const int nt = tpass_threads_for(dt, a.m);
    hipError_t e = hipFuncSetAttribute(tpass_fn<R, REV>(nt), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess)
        return e;
    if (nt == tpass_max_threads<R>())
        return go_nt<R, REV, tpass_max_threads<R>()>(a, psi, lam, blocks, lds, s);
    if (nt == 256)
        return go_nt<R, REV, 256>(a, psi, lam, blocks, lds, s);
    return go_nt<R, REV, 128>(a, psi, lam, blocks, lds, s);
}

}  // namespace

size_t tpass_lds_bytes(int dt, int m, bool rev)
{
    const size_t R = dt == C64 ? 4 : 8;
    return rev ? 2 * (2 * R << m) + sizeof(double) * kMaxTpassOps : (2 * R << m);
}

size_t tpass_lop_bytes(int dt, int nops)
{
    return 2 * (size_t)nops * (dt == C64 ? sizeof(LOp<float>) : sizeof(LOp<double>));
}

hipError_t launch_tstage(const TPassArgs& a, int dt, hipStream_t s)
{
    const int n2 = 2 * a.nops_total;
    if (n2 == 0)
        return hipSuccess;
    const int blocks = (n2 + 255) / 256;
    if (dt == C64)
        hipLaunchKernelGGL(k_tstage<float>, dim3(blocks), dim3(256), 0, s, a.ops, a.nops_total, a.mats,
                           a.params, static_cast<LOp<float>*>(a.lops));
    else
        hipLaunchKernelGGL(k_tstage<double>, dim3(blocks), dim3(256), 0, s, a.ops, a.nops_total, a.mats,
                           a.params, static_cast<LOp<double>*>(a.lops));
    return hipGetLastError();
}

int tpass_resident_blocks(int dt, int m, bool rev)
{
    int dev = 0, cus = 0, per = 0, maxlds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    const size_t lds = tpass_lds_bytes(dt, m, rev);
    if (lds + sizeof(ExecShared) > (size_t)maxlds)
        return 0;
    const int threads = tpass_threads_for(dt, m);
    const void* fn = dt == C64 ? (rev ? tpass_fn<float, true>(threads) : tpass_fn<float, false>(threads))
                               : (rev ? tpass_fn<double, true>(threads) : tpass_fn<double, false>(threads));
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, lds) != hipSuccess)
        return 0;
    return per * cus;
}

hipError_t launch_tpass(const TPassArgs& a, int dt, bool rev, void* psi, void* lam, int blocks,
                        hipStream_t s)
{
    if (dt == C64)
        return rev ? go<float, true>(a, psi, lam, blocks, s) : go<float, false>(a, psi, lam, blocks, s);
    return rev ? go<double, true>(a, psi, lam, blocks, s) : go<double, false>(a, psi, lam, blocks, s);
}

}  // namespace qsv
