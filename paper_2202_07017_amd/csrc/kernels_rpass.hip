// Register-tile Pauli passes: <psi|H|psi> with the tile in registers.
//
// A wave takes a tile of 2^11 amplitudes: its 64 lanes run over 6 lane
// qubits (qubits 0..4 and one more, so every load instruction reads runs of
// 32 consecutive amplitudes) and each lane holds the 32 amplitudes of 5
// register qubits.  The pass evaluates, from registers only, the kinds of
// terms that make up Ising- and Heisenberg-type Hamiltonians:
//
//  * a single-qubit X on a register qubit pairs amplitude i = (lane, r) with
//    j = (lane, r ^ 2^k); the two contributions conj(psi_i) psi_j and
//    conj(psi_j) psi_i are complex conjugates, so each pair is visited once
//    and adds 2 Re(conj(psi_i) psi_j);
//  * any string whose x mask is one or two register qubits (XX, YY, XY, Y,
//    with Z factors anywhere except on the other register qubits) the same
//    way, with 2 Re or 2 Im of the pair product by its number of Y factors
//    and the sign of its z mask on the pair's first member (register part:
//    that member's lower x bit; lane part fixed per lane; tile part per
//    tile);
//  * diagonal terms sum (-1)^popcount(i & z) |psi_i|^2.  With the per-lane
//    Walsh-Hadamard transform N(m) = sum_r (-1)^popcount(r & m) |psi_(lane,r)|^2
//    (five butterfly stages), a term costs its two signs (lane part, fixed
//    per lane, and tile part) however many amplitudes the tile holds; terms
//    come grouped by their register mask m, so N(m) is read at a
//    compile-time index;
//  * strings whose x mask lies on qubits 0..4 (lane bits) are evaluated after
//    an LDS transpose of the wave's tile that makes qubits 0..4 the register
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
// Diagonal terms of one register mask are taken in chunks of up to kChunk
// consecutive terms; a chunk's 2^g signed coefficient sums (one per sign
// pattern of its g terms) sit in an LDS table, so a lane's weight for the
// chunk is one table read indexed by its g sign bits.  Since 2^g <= 32 g / 5
// for 1 <= g <= 5, the tables of kMaxRegTerms terms need at most
// 32 * kMaxRegTerms / 5 entries.
constexpr int kChunk = 5;
constexpr int kDiagTab = (32 * kMaxRegTerms) / kChunk + 1;

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
        double& t = (m++ & 1) ? s1 : s0;
        t = __builtin_fma(re[r], re[j], t);
        t = __builtin_fma(im[r], im[j], t);
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

// Term data held across the wave: lane k keeps term k's coefficient, z mask
// and register x mask in registers, and the tile loop fetches them with
// readlane (a register read) instead of a scalar memory load per term.
struct LaneTerms {
    double c;
    double c2;
    uint64_t z;
    uint32_t xr;
    int32_t ylo;
    uint32_t xl;
};

__device__ __forceinline__ double lane_double(double v, int k)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double term_coef(const LaneTerms& L, int k) { return lane_double(L.c, k); }

// Terms [k0, k1): single-qubit X on a register qubit of the current roles.
// For Hermitian X the pairs (i, i ^ x) add 2 Re(conj(psi_i) psi_(i ^ x)); the
// factor 2 is in the term's coefficient.
__device__ __forceinline__ double pair_terms(const LaneTerms& L, int k0, int k1, const double (&re)[kNR],
                                             const double (&im)[kNR])
{
    double s = 0.0;
    for (int k = k0; k < k1; ++k) {
        const uint32_t xr = (uint32_t)__builtin_amdgcn_readlane((int)L.xr, k);
        s += term_coef(L, k) * pair_dispatch(xr, re, im);
    }
    return s;
}

// A string P with x mask on register bits XR (one bit or two neighbouring
// ones) and a z mask whose register bits lie inside XR: over the pairs
// (a, b = a ^ x) with a the member whose highest x bit (HB) is 0,
//   <psi|P|psi> = sum_pairs c i^ylo (-1)^(z.a) [w + (-1)^ylo conj(w)],
// w = conj(psi_b) psi_a, i.e. 2 Re w (ylo even) or 2 Im w (ylo odd) times
// (+-1) and (-1)^(z.a).  The register part of (-1)^(z.a) is (-1)^(a_LB) when
// z has the lowest x bit LB (a_HB = 0), so the pairs are summed in two
// halves by a_LB (s0: a_LB = 0, s1: a_LB = 1; for a single x bit the halves
// simply alternate) and the host folds that sign into the coefficient of s1.
struct Halves {
    double s0, s1;
};

template <int XR, bool IM>
__device__ __forceinline__ Halves gen_sum(const double (&re)[kNR], const double (&im)[kNR])
{
    constexpr int HB = (XR & 16) ? 4 : (XR & 8) ? 3 : (XR & 4) ? 2 : (XR & 2) ? 1 : 0;
    constexpr int LB = (XR & 1) ? 0 : (XR & 2) ? 1 : (XR & 4) ? 2 : (XR & 8) ? 3 : 4;
    double s0 = 0.0, s1 = 0.0;
    int m = 0;
#pragma unroll
    for (int r = 0; r < kNR; ++r) {
        if ((r >> HB) & 1)
            continue;
        const int j = r ^ XR;
        double& t = (LB != HB ? ((r >> LB) & 1) : (m++ & 1)) ? s1 : s0;
        if (IM) {
            t = __builtin_fma(im[r], re[j], t);
            t = __builtin_fma(-re[r], im[j], t);
        } else {
            t = __builtin_fma(re[r], re[j], t);
            t = __builtin_fma(im[r], im[j], t);
        }
    }
    return Halves{s0, s1};
}

// x masks of one register bit or two neighbouring ones (each further case
// costs registers: with all ten two-bit masks a complex64 pass no longer fits
// two waves per SIMD); the host sends other masks to the LDS-tile passes
template <bool IM>
__device__ __forceinline__ Halves gen_dispatch(uint32_t xr, const double (&re)[kNR], const double (&im)[kNR])
{
    switch (xr) {
    case 1: return gen_sum<1, IM>(re, im);
    case 2: return gen_sum<2, IM>(re, im);
    case 4: return gen_sum<4, IM>(re, im);
    case 8: return gen_sum<8, IM>(re, im);
    case 16: return gen_sum<16, IM>(re, im);
    case 3: return gen_sum<3, IM>(re, im);
    case 6: return gen_sum<6, IM>(re, im);
    case 12: return gen_sum<12, IM>(re, im);
    case 24: return gen_sum<24, IM>(re, im);
    default: return Halves{0.0, 0.0};
    }
}

// Terms [k0, k1): strings with an x mask of one register bit or two
// neighbouring ones of the current roles (merged as described at RTerm).  sg
// bit k set: the lane and tile parts of the z sign are negative for term k.
__device__ __forceinline__ double gen_terms(const LaneTerms& L, uint64_t sg, int k0, int k1,
                                            const double (&re)[kNR], const double (&im)[kNR])
{
    double s = 0.0;
    for (int k = k0; k < k1; ++k) {
        const uint32_t xr = (uint32_t)__builtin_amdgcn_readlane((int)L.xr, k);
        const int ylo = __builtin_amdgcn_readlane(L.ylo, k);
        const Halves h = (ylo & 1) ? gen_dispatch<true>(xr, re, im) : gen_dispatch<false>(xr, re, im);
        const double v = lane_double(L.c, k) * h.s0 + lane_double(L.c2, k) * h.s1;
        s += ((sg >> k) & 1) ? -v : v;
    }
    return s;
}

// Terms [k0, k1) of the transposed roles: strings whose x mask is register
// bit 4 (qubit 4) and one lane bit (mask xl).  The pair of (lane, r), r < 16,
// is (lane ^ xl, r + 16): the partner's amplitudes come over the cross-lane
// crossbar, and each lane sums its own 16 pairs (r bit 4 clear), so every
// pair is visited once.  The z sign has no register part (z on qubits 0..3
// is excluded and r bit 4 is 0); lane and tile parts come from sg, the
// factor 2 and the sign of i^ylo from the coefficient.
__device__ __forceinline__ double cross_terms(const LaneTerms& L, uint64_t sg, int k0, int k1,
                                              const double (&re)[kNR], const double (&im)[kNR])
{
    double s = 0.0;
    for (int k = k0; k < k1; ++k) {
        const int xl = __builtin_amdgcn_readlane((int)L.xl, k);
        const int ylo = __builtin_amdgcn_readlane(L.ylo, k);
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int r = 0; r < kNR / 2; ++r) {
            const double br = __shfl_xor(re[r + kNR / 2], xl, 64);
            const double bi = __shfl_xor(im[r + kNR / 2], xl, 64);
            double& t = (r & 1) ? s1 : s0;
            if (ylo & 1) {
                t = __builtin_fma(im[r], br, t);
                t = __builtin_fma(-re[r], bi, t);
            } else {
                t = __builtin_fma(re[r], br, t);
                t = __builtin_fma(im[r], bi, t);
            }
        }
        const double v = term_coef(L, k) * (s0 + s1);
        s += ((sg >> k) & 1) ? -v : v;
    }
    return s;
}

template <typename R, bool TR, bool GEN>
__global__ void __launch_bounds__(256) k_reg_pass(const R* __restrict__ psi, const RegPassK a,
                                                  double* __restrict__ partials, int pstride, int accumulate)
{
    using A = typename RV<R>::A;
    __shared__ A xt[TR ? kWaves * kNR * kRow : 1];
    __shared__ double red[kWaves];
    __shared__ double dtab[kDiagTab];
    const int lane = threadIdx.x & 63;
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint64_t w0 = (uint64_t)blockIdx.x * kWaves + wv;
    const uint64_t nw = (uint64_t)gridDim.x * kWaves;
    uint64_t loff = 0;
#pragma unroll
    for (int b = 0; b < kRegLanes; ++b)
        loff |= (uint64_t)((lane >> b) & 1) << a.lanepos[b];
    // lane part of every term's sign, once: bit k = parity(lane & zl_k)
    uint64_t lsg = 0;
    for (int k = 0; k < a.nt; ++k)
        lsg |= (uint64_t)(__popc((uint32_t)lane & a.t[k].zl) & 1) << k;
    // signed coefficient sums of every chunk: entry p of a chunk starting at
    // term k0 with g terms = sum_i (-1)^(bit i of p) c_(k0+i)
    if (a.nd > 0) {
        int off = 0;
        for (int m = 0; m < kNR; ++m) {
            const int k1 = a.mofs[m + 1];
            for (int k0 = a.mofs[m]; k0 < k1; k0 += kChunk) {
                const int g = min(kChunk, k1 - k0);
                for (int q = threadIdx.x; q < (1 << g); q += blockDim.x) {
                    double w = 0.0;
                    for (int i = 0; i < g; ++i)
                        w += ((q >> i) & 1) ? -a.t[k0 + i].c : a.t[k0 + i].c;
                    dtab[off + q] = w;
                }
                off += 1 << g;
            }
        }
        __syncthreads();
    }
    LaneTerms LT{0.0, 0.0, 0, 0, 0, 0};
    if (lane < a.nt) {
        LT.c = a.t[lane].c;
        LT.c2 = a.t[lane].c2;
        LT.z = a.t[lane].z;
        LT.xr = a.t[lane].xr;
        LT.ylo = a.t[lane].ylo;
        LT.xl = a.t[lane].xl;
    }
    double acc = 0.0;
    // Software pipeline (passes without the general string sums): the loads
    // of the wave's next tile are issued as soon as the current tile has been
    // widened to FP64, so every term below runs while they are in flight.
    // The general sums need the registers of that second tile.
    constexpr bool kPrefetch = !GEN;
    A v[kNR];
    const A* const p0 = reinterpret_cast<const A*>(psi) + loff;
    auto load_tile = [&](uint64_t b) {
        const A* p = p0 + b;
#pragma unroll
        for (int r = 0; r < kNR; ++r) {
            uint64_t o = 0;
#pragma unroll
            for (int k = 0; k < kRegQubits; ++k)
                if ((r >> k) & 1)
                    o += a.qstride[k];
            v[r] = __builtin_nontemporal_load(p + o);
        }
    };
    if (kPrefetch && w0 < a.ntiles)
        load_tile(insert_tile(w0, a));
    for (uint64_t tl = w0; tl < a.ntiles; tl += nw) {
        const uint64_t base = insert_tile(tl, a);
        if (!kPrefetch)
            load_tile(base);
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
        double re[kNR], im[kNR];
#pragma unroll
        for (int r = 0; r < kNR; ++r) {
            re[r] = (double)v[r].x;
            im[r] = (double)v[r].y;
        }
        if (kPrefetch && tl + nw < a.ntiles)
            load_tile(insert_tile(tl + nw, a));
        // tile part of every term's sign (uniform: lane k evaluates term k's
        // parity with the tile base and a ballot gathers them)
        const uint64_t sg = lsg ^ __ballot(lane < a.nt && (__popcll(base & LT.z) & 1));
        double s = 0.0;
        s += GEN ? gen_terms(LT, sg, a.nd, a.n1, re, im) : pair_terms(LT, a.nd, a.n1, re, im);
        if (a.nd > 0) {
            // N(m) = sum_r (-1)^popcount(r & m) |psi_(lane,r)|^2, built in
            // place of re (the pair terms are done with it)
#pragma unroll
            for (int r = 0; r < kNR; ++r)
                re[r] = re[r] * re[r] + im[r] * im[r];
#pragma unroll
            for (int h = 1; h < kNR; h <<= 1)
#pragma unroll
                for (int r = 0; r < kNR; ++r)
                    if (!(r & h)) {
                        const double u = re[r], w = re[r + h];
                        re[r] = u + w;
                        re[r + h] = u - w;
                    }
            // per register mask m (known at compile time) its chunks: the
            // lane's sign bits of a chunk index its table of signed
            // coefficient sums
            int off = 0;
#pragma unroll
            for (int m = 0; m < kNR; ++m) {
                const int k1 = a.mofs[m + 1];
                for (int k0 = a.mofs[m]; k0 < k1; k0 += kChunk) {
                    const int g = min(kChunk, k1 - k0);
                    const int q = (int)(sg >> k0) & ((1 << g) - 1);
                    s += dtab[off + q] * re[m];
                    off += 1 << g;
                }
            }
        }
        if (TR && a.nt > a.n1) {
            // the transposed roles
            __builtin_amdgcn_wave_barrier();
            const A* src = rows + (lane >> 1) * kRow + ((lane & 1) ? 33 : 0);
#pragma unroll
            for (int r = 0; r < kNR; ++r) {
                const A w = src[r];
                re[r] = (double)w.x;
                im[r] = (double)w.y;
            }
            __builtin_amdgcn_wave_barrier();
            s += GEN ? gen_terms(LT, sg, a.n1, a.nc, re, im) : pair_terms(LT, a.n1, a.nc, re, im);
            if (GEN)
                s += cross_terms(LT, sg, a.nc, a.nt, re, im);
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

template <typename R, bool TR, bool GEN>
int reg_grid()
{
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 1024;
    if (cache[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_reg_pass<R, TR, GEN>, 256, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            per_cu < 1 || cus < 1)
            return 1024;
        cache[dev] = per_cu * cus;
    }
    return cache[dev];
}

template <typename R, bool TR, bool GEN>
hipError_t go(const RegPassK& a, const void* psi, double* partials, int nslots, int accumulate,
              hipStream_t s)
{
    // every resident block once (capped by the partial slots), each wave
    // streaming tiles
    uint64_t g = (uint64_t)reg_grid<R, TR, GEN>();
    if (g > (uint64_t)nslots)
        g = (uint64_t)nslots;
    const uint64_t maxg = (a.ntiles + kWaves - 1) / kWaves;
    if (g > maxg)
        g = maxg;
    if (g < 1)
        g = 1;
    hipLaunchKernelGGL((k_reg_pass<R, TR, GEN>), dim3((unsigned)g), dim3(256), 0, s, static_cast<const R*>(psi),
                       a, partials, nslots, accumulate);
    return hipGetLastError();
}

// The variant: complex64 or complex128; with the transpose when strings on
// qubits 0..4 are present; with the general string sums only when needed
// (they cost registers, and complex64 passes without them keep two waves
// per SIMD).
template <typename R>
hipError_t pick(const RegPassK& a, const void* psi, double* partials, int nslots, int accumulate,
                hipStream_t s)
{
    const bool tr = a.nt > a.n1;
    const bool gen = a.n1 > a.ns1 || a.nc > a.ns2 || a.nt > a.nc;
    if (tr)
        return gen ? go<R, true, true>(a, psi, partials, nslots, accumulate, s)
                   : go<R, true, false>(a, psi, partials, nslots, accumulate, s);
    return gen ? go<R, false, true>(a, psi, partials, nslots, accumulate, s)
               : go<R, false, false>(a, psi, partials, nslots, accumulate, s);
}

}  // namespace

hipError_t launch_reg_pass(const RegPassK& a, const void* psi, int dt, double* partials, int nslots,
                           int accumulate, hipStream_t s)
{
    if (a.ntiles == 0)
        return hipSuccess;
    // the term tables assume nd <= nt <= kMaxRegTerms and mofs ascending from
    // 0 to nd (the chunk tables then fit in kDiagTab entries)
    if (a.nt > kMaxRegTerms || a.nd < 0 || a.nd > a.ns1 || a.ns1 > a.n1 || a.n1 > a.ns2 || a.ns2 > a.nc ||
        a.nc > a.nt || a.mofs[0] != 0 || a.mofs[1 << kRegQubits] != a.nd)
        return hipErrorInvalidValue;
    for (int m = 0; m < (1 << kRegQubits); ++m)
        if (a.mofs[m + 1] < a.mofs[m])
            return hipErrorInvalidValue;
    return dt == C64 ? pick<float>(a, psi, partials, nslots, accumulate, s)
                     : pick<double>(a, psi, partials, nslots, accumulate, s);
}

}  // namespace qsv
