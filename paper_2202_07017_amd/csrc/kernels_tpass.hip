// One cache-blocked pass of a tile program over a whole state (one launch per
// pass, tiles spread over the grid).
//
// Every block stages the pass (matrices, steps) in LDS once, then takes tiles
// tile = blockIdx.x, + gridDim.x, ...: loads the tile (psi; reverse passes
// also lambda) into LDS in contiguous chunks of 16-byte vectors, runs the
// pass's steps on it (tile_exec.h) and stores it back.  Reverse passes end by
// writing the block's per-rotation FP64 sums to
// partials[(slot_base + slot) * nb + block], which a finalize kernel adds in
// block order.
#include "qsv_tpass.h"
#include "tile_exec.h"

namespace qsv {
namespace {

using tx::ExecShared;
using tx::LOp;

template <typename R>
struct TV;
template <>
struct TV<float> {
    using V = float4;
    static constexpr int APV = 2;
};
template <>
struct TV<double> {
    using V = double2;
    static constexpr int APV = 1;
};

template <typename R, bool REV>
__global__ void __launch_bounds__(kTpassThreads) k_tpass(R* __restrict__ psi, R* __restrict__ lam,
                                                         const TPassArgs a)
{
    using V = typename TV<R>::V;
    constexpr int APV = TV<R>::APV;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ ExecShared sh;
    const int m = a.m;
    const size_t tile = (size_t)2 * sizeof(R) << m;
    R* phiL = reinterpret_cast<R*>(smem);
    R* lamL = reinterpret_cast<R*>(smem + tile);
    LOp<R>* ops = reinterpret_cast<LOp<R>*>(smem + (REV ? 2 : 1) * tile);
    DStep* steps = reinterpret_cast<DStep*>(reinterpret_cast<unsigned char*>(ops) +
                                            sizeof(LOp<R>) * kMaxPassOps);
    const DPass P = a.pass;
    tx::stage<R>(P, a.steps, a.ops, a.mats, a.params, REV, ops, steps, sh);
    __syncthreads();
    const uint32_t nvec = (1u << m) / APV;
    const uint64_t ntiles = 1ull << (a.n - m);
    V* pg = reinterpret_cast<V*>(psi);
    V* lg = reinterpret_cast<V*>(lam);
    V* pl = reinterpret_cast<V*>(phiL);
    V* ll = reinterpret_cast<V*>(lamL);
    int parity = 0;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint64_t base = tx::insert_mask(t, P.bmask);
        for (uint32_t v = threadIdx.x; v < nvec; v += blockDim.x) {
            const uint64_t gi = (base | tx::deposit_mask((uint64_t)v * APV, P.bmask)) / APV;
            pl[v] = pg[gi];
            if (REV)
                ll[v] = lg[gi];
        }
        __syncthreads();
        tx::exec_tile<R, REV, 8>(ops, steps, P.nsteps, m, phiL, lamL, sh, parity);
        for (uint32_t v = threadIdx.x; v < nvec; v += blockDim.x) {
            const uint64_t gi = (base | tx::deposit_mask((uint64_t)v * APV, P.bmask)) / APV;
            pg[gi] = pl[v];
            if (REV)
                lg[gi] = ll[v];
        }
        __syncthreads();
    }
    if (REV)
        for (int j = threadIdx.x; j < P.nrot; j += blockDim.x)
            a.partials[(size_t)(P.slot_base + j) * gridDim.x + blockIdx.x] = sh.pacc[j];
}

template <typename R, bool REV>
hipError_t go(const TPassArgs& a, void* psi, void* lam, int blocks, hipStream_t s)
{
    const size_t lds = tpass_lds_bytes(sizeof(R) == 4 ? C64 : C128, a.m, REV);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_tpass<R, REV>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_tpass<R, REV>), dim3(blocks), dim3(kTpassThreads), lds, s,
                       static_cast<R*>(psi), static_cast<R*>(lam ? lam : psi), a);
    return hipGetLastError();
}

}  // namespace

size_t tpass_lds_bytes(int dt, int m, bool rev)
{
    const size_t R = dt == C64 ? 4 : 8;
    const size_t op = dt == C64 ? sizeof(LOp<float>) : sizeof(LOp<double>);
    return (rev ? 2 : 1) * (2 * R << m) + (op + sizeof(DStep)) * kMaxPassOps;
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
    const void* fn = dt == C64 ? (rev ? reinterpret_cast<const void*>(k_tpass<float, true>)
                                      : reinterpret_cast<const void*>(k_tpass<float, false>))
                               : (rev ? reinterpret_cast<const void*>(k_tpass<double, true>)
                                      : reinterpret_cast<const void*>(k_tpass<double, false>));
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kTpassThreads, lds) != hipSuccess)
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
