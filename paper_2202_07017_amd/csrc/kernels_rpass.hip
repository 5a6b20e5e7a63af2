// Register-tile Pauli passes: <psi|H|psi> with the tile in registers.
//
// A wave takes a tile of 2^11 amplitudes: its 64 lanes run over 6 lane
// qubits (qubits 0..4 and one more, so every load instruction reads runs of
// 32 consecutive amplitudes) and each lane holds the 32 amplitudes of 5
// register qubits.  The pass evaluates, from registers only, the two kinds
// of terms that dominate the transverse-field and Ising-type Hamiltonians:
//
//  * a single-qubit X on a register qubit pairs amplitude i = (lane, r) with
//    j = (lane, r ^ 2^k); the two contributions conj(psi_i) psi_j and
//    conj(psi_j) psi_i are complex conjugates, so each pair is visited once
//    and adds 2 Re(conj(psi_i) psi_j);
//  * diagonal terms sum (-1)^popcount(i & z) |psi_i|^2.  With the per-lane
//    Walsh-Hadamard transform N(m) = sum_r (-1)^popcount(r & m) |psi_(lane,r)|^2
//    (five butterfly stages), a term costs its two signs (lane part, fixed
//    per lane, and tile part) however many amplitudes the tile holds; terms
//    come grouped by their register mask m, so N(m) is read at a
//    compile-time index;
//  * a single-qubit X on qubits 0..4 (lane bits) is evaluated after an LDS
//    transpose of the wave's tile that makes qubits 0..4 the register
//    qubits.
//
// Every other Pauli string goes to the LDS-tile passes (kernels_expect.hip).
// There is no workgroup barrier in the tile loop: waves stream tiles
// independently (grid-stride over tiles), which keeps the HBM queue full
// (the LDS-tile pass, with a barrier per tile, ran at about 3 TB/s on
// complex64; this form streams at about 7 TB/s with five X terms).  Every
// sum is FP64 with amplitudes widened first; the order is fixed by the
// grid, so results are deterministic.
#include "qsv_rpass.h"

namespace qsv {
namespace {

constexpr int kNR = 1 << kRegQubits;  // 32 amplitudes per lane
constexpr int kWaves = 4;             // waves per block
constexpr int kRow = 64 + 3;          // transpose row: 64 lanes + padding; lanes 32..63 skewed by one

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename R>
struct RV;
template <>
struct RV<float> {
    using A = f32x2;
};
template <>
struct RV<double> {
    using A = f64x2;
};

__device__ __forceinline__ uint64_t insert_tile(uint64_t g, const RegPassK& a)
{
#pragma unroll
    for (int j = 0; j < kRegTileQubits; ++j) {
        const uint64_t lo = a.low[j];
        g = ((g & ~lo) << 1) | (g & lo);
    }
    return g;
}

// sum over the pairs (r, r ^ 2^K), r with bit K clear, of Re(conj(a_r) a_(r ^ 2^K))
// = ar br + ai bi: the value of a single-qubit X on register bit K, halved.
template <int K>
__device__ __forceinline__ double pair_sum(const double (&re)[kNR], const double (&im)[kNR])
{
    double s0 = 0.0, s1 = 0.0;
    int m = 0;
#pragma unroll
    for (int r = 0; r < kNR; ++r) {
        if ((r >> K) & 1)
            continue;
        const int j = r | (1 << K);
        const double d = re[r] * re[j] + im[r] * im[j];
        if (m++ & 1)
            s1 += d;
        else
            s0 += d;
    }
    return s0 + s1;
}

__device__ __forceinline__ double pair_dispatch(uint32_t xr, const double (&re)[kNR], const double (&im)[kNR])
{
    switch (xr) {
    case 1:
        return pair_sum<0>(re, im);
    case 2:
        return pair_sum<1>(re, im);
    case 4:
        return pair_sum<2>(re, im);
    case 8:
        return pair_sum<3>(re, im);
    case 16:
        return pair_sum<4>(re, im);
    default:
        return 0.0;
    }
}

// Terms [k0, k1): single-qubit X on a register qubit of the current roles.
// For Hermitian X the pairs (i, i ^ x) add 2 Re(conj(psi_i) psi_(i ^ x)).
__device__ __forceinline__ double pair_terms(const RegPassK& a, int k0, int k1, const double (&re)[kNR],
                                             const double (&im)[kNR])
{
    double s = 0.0;
    for (int k = k0; k < k1; ++k) {
        const RTerm& T = a.t[k];
        s += 2.0 * T.c * pair_dispatch(T.xr, re, im);
    }
    return s;
}

template <typename R, bool TR>
__global__ void __launch_bounds__(256) k_reg_pass(const R* __restrict__ psi, const RegPassK a,
                                                  double* __restrict__ partials, int pstride, int accumulate)
{
    using A = typename RV<R>::A;
    __shared__ A xt[TR ? kWaves * kNR * kRow : 1];
    __shared__ double red[kWaves];
    const int lane = threadIdx.x & 63;
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint64_t w0 = (uint64_t)blockIdx.x * kWaves + wv;
    const uint64_t nw = (uint64_t)gridDim.x * kWaves;
    uint64_t loff = 0;
#pragma unroll
    for (int b = 0; b < kRegLanes; ++b)
        loff |= (uint64_t)((lane >> b) & 1) << a.lanepos[b];
    // lane part of every diagonal term's sign, once: bit k = parity(lane & zl_k)
    uint64_t lsg = 0;
    for (int k = 0; k < a.nd; ++k)
        lsg |= (uint64_t)(__popc((uint32_t)lane & a.t[k].zl) & 1) << k;
    double acc = 0.0;
    for (uint64_t tl = w0; tl < a.ntiles; tl += nw) {
        const uint64_t base = insert_tile(tl, a);
        const A* p = reinterpret_cast<const A*>(psi) + base;
        A v[kNR];
#pragma unroll
        for (int r = 0; r < kNR; ++r) {
            uint64_t o = 0;
#pragma unroll
            for (int k = 0; k < kRegQubits; ++k)
                if ((r >> k) & 1)
                    o += a.qstride[k];
            v[r] = __builtin_nontemporal_load(p + o + loff);
        }
        A* rows = TR ? xt + wv * (kNR * kRow) : nullptr;
        if (TR && a.nt > a.n1) {
            // transpose through this wave's LDS rows: element (lane l,
            // register r) at row r, column l (+1 for l >= 32: the two
            // half-rows fall on different banks); read back below with
            // register r' = l bits 0..4 and lane L = (l bit 5) | (r << 1)
#pragma unroll
            for (int r = 0; r < kNR; ++r)
                rows[r * kRow + lane + (lane >> 5)] = v[r];
        }
        double s = 0.0;
        if (a.nd > 0) {
            double N[kNR];
#pragma unroll
            for (int r = 0; r < kNR; ++r) {
                const double x = (double)v[r].x, y = (double)v[r].y;
                N[r] = x * x + y * y;
            }
#pragma unroll
            for (int h = 1; h < kNR; h <<= 1)
#pragma unroll
                for (int r = 0; r < kNR; ++r)
                    if (!(r & h)) {
                        const double u = N[r], w = N[r + h];
                        N[r] = u + w;
                        N[r + h] = u - w;
                    }
            // tile part of the signs (uniform), then the terms grouped by
            // their register mask: each group adds (sum of signed
            // coefficients) * N(m) with m known at compile time
            uint64_t bsg = 0;
            for (int k = 0; k < a.nd; ++k)
                bsg |= (uint64_t)(__popcll(base & a.t[k].z) & 1) << k;
            const uint64_t sg = lsg ^ bsg;
#pragma unroll
            for (int m = 0; m < kNR; ++m) {
                const int k0 = a.mofs[m], k1 = a.mofs[m + 1];
                if (k0 == k1)
                    continue;
                double w = 0.0;
                for (int k = k0; k < k1; ++k)
                    w += ((sg >> k) & 1) ? -a.t[k].c : a.t[k].c;
                s += w * N[m];
            }
        }
        double re[kNR], im[kNR];
        if (a.n1 > a.nd) {
#pragma unroll
            for (int r = 0; r < kNR; ++r) {
                re[r] = (double)v[r].x;
                im[r] = (double)v[r].y;
            }
            s += pair_terms(a, a.nd, a.n1, re, im);
        }
        if (TR && a.nt > a.n1) {
            __builtin_amdgcn_wave_barrier();
            const A* src = rows + (lane >> 1) * kRow + ((lane & 1) ? 33 : 0);
#pragma unroll
            for (int r = 0; r < kNR; ++r) {
                const A w = src[r];
                re[r] = (double)w.x;
                im[r] = (double)w.y;
            }
            __builtin_amdgcn_wave_barrier();
            s += pair_terms(a, a.n1, a.nt, re, im);
        }
        acc += s;
    }
    for (int off = 32; off > 0; off >>= 1)
        acc += __shfl_xor(acc, off, 64);
    if (lane == 0)
        red[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kWaves; ++w)
            t += red[w];
        double* pr = partials + blockIdx.x;
        double* pi = partials + pstride + blockIdx.x;
        *pr = accumulate ? *pr + t : t;
        if (!accumulate)
            *pi = 0.0;
    }
    if (!accumulate)  // slots beyond the grid start at zero for later passes
        for (int b = gridDim.x + blockIdx.x * 256 + threadIdx.x; b < pstride; b += gridDim.x * 256) {
            partials[b] = 0.0;
            partials[pstride + b] = 0.0;
        }
}

template <typename R, bool TR>
int reg_grid()
{
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 1024;
    if (cache[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_reg_pass<R, TR>, 256, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            per_cu < 1 || cus < 1)
            return 1024;
        cache[dev] = per_cu * cus;
    }
    return cache[dev];
}

template <typename R, bool TR>
hipError_t go(const RegPassK& a, const void* psi, double* partials, int nslots, int accumulate,
              hipStream_t s)
{
    // every resident block once (capped by the partial slots), each wave
    // streaming tiles
    uint64_t g = (uint64_t)reg_grid<R, TR>();
    if (g > (uint64_t)nslots)
        g = (uint64_t)nslots;
    const uint64_t maxg = (a.ntiles + kWaves - 1) / kWaves;
    if (g > maxg)
        g = maxg;
    if (g < 1)
        g = 1;
    hipLaunchKernelGGL((k_reg_pass<R, TR>), dim3((unsigned)g), dim3(256), 0, s, static_cast<const R*>(psi), a,
                       partials, nslots, accumulate);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_reg_pass(const RegPassK& a, const void* psi, int dt, double* partials, int nslots,
                           int accumulate, hipStream_t s)
{
    if (a.ntiles == 0)
        return hipSuccess;
    const bool tr = a.nt > a.n1;
    if (dt == C64)
        return tr ? go<float, true>(a, psi, partials, nslots, accumulate, s)
                  : go<float, false>(a, psi, partials, nslots, accumulate, s);
    return tr ? go<double, true>(a, psi, partials, nslots, accumulate, s)
              : go<double, false>(a, psi, partials, nslots, accumulate, s);
}

}  // namespace qsv
