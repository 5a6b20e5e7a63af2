// Span passes: <psi|H|psi> for Pauli strings with arbitrary x masks, up to
// five x masks with a qubit above 5 per state read, plus any number of
// strings whose x mask lies on qubits 0..5 and of diagonal strings.
//
// A string P = i^ylo X^x Z^z pairs every amplitude with the one whose index
// differs by x; a pass over the state for each x mask reads the state once
// per mask.  Here a pass takes five x masks at once (the directions d_j, see
// qsv_span_plan.h): a wave's tile is the coset base ^ span(qubits 0..5,
// d_0..d_4) of 2^11 amplitudes, lane L and register r holding amplitude
// base ^ L ^ D(r).  The partner of (L, r) under direction j is (L, r ^ 2^j),
// so every pair lies within one lane's registers and the tile needs no LDS
// and no exchange between lanes.  Each register's load reads the 64
// amplitudes of one aligned run of the state (lane order permuted by the low
// six bits of D(r)), so the reads stay coalesced whatever the masks are.
//
// Over the pairs (a, b = a ^ x), a the member with register bit j clear,
//   <psi|P|psi> = sum_pairs i^ylo (-1)^(z.a) [w + (-1)^ylo conj(w)],
// w = conj(psi_b) psi_a (the second member's sign differs by
// (-1)^popcount(x & z) = (-1)^ylo): 2 Re w or 2 Im w by the parity of ylo,
// times the sign of i^ylo (folded into the coefficient by the host) and
// (-1)^(z.a).  The sign splits as z.a = z.base + z.L + z.D(r): a tile part
// (uniform; lane k evaluates it for string k and a ballot gathers the bits),
// a lane part (fixed per lane) and a register part per pair (host table).
// A string with x on qubits 0..5 pairs (L, r) with (L ^ x, r), taken over
// the cross-lane crossbar; each lane sums its own 32 ordered pairs, so every
// unordered pair is counted from both ends and the factor 2 is not needed.
// Diagonal strings use the per-lane Walsh-Hadamard transform of |psi|^2
// over the registers, N(m), with m = the string's register mask.
// Every product and sum is FP64 (amplitudes widened first), in a fixed order.
#include <type_traits>

#include "qsv_span.h"

namespace qsv {
namespace {

constexpr int kNR = 1 << kSpanDirs;  // 32 amplitudes per lane
constexpr int kWaves = 4;            // waves per block
constexpr int kPairs = kNR / 2;

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename R>
struct SV;
template <>
struct SV<float> {
    using A = f32x2;
};
template <>
struct SV<double> {
    using A = f64x2;
};

__device__ __forceinline__ uint64_t insert_tile(uint64_t g, const SpanPassK& a)
{
#pragma unroll
    for (int j = 0; j < kSpanTileQubits; ++j) {
        const uint64_t lo = a.low[j];
        g = ((g & ~lo) << 1) | (g & lo);
    }
    return g;
}

// D(r): XOR of the directions d_j over the set bits j of r (uniform)
__device__ __forceinline__ uint64_t dmask(const SpanPassK& a, int r)
{
    uint64_t o = 0;
#pragma unroll
    for (int j = 0; j < kSpanDirs; ++j)
        if ((r >> j) & 1)
            o ^= a.d[j];
    return o;
}

// sum_i (-1)^(bit i of m) f_i, f_i = Re (IM false) or Im (IM true) of
// conj(psi_b) psi_a for the i-th pair of direction DIR: a = register r_i
// (bit DIR clear), b = r_i ^ 2^DIR.  The sign is a uniform +-1.0 built from
// m, so each pair costs its product and one fused multiply-add.
template <int DIR, bool IM>
__device__ __forceinline__ double string_sum(const double (&re)[kNR], const double (&im)[kNR], uint32_t m)
{
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kPairs; ++i) {
        const int r = ((i >> DIR) << (DIR + 1)) | (i & ((1 << DIR) - 1));
        const int j = r | (1 << DIR);
        const double f = IM ? im[r] * re[j] - re[r] * im[j] : re[r] * re[j] + im[r] * im[j];
        const double sgn = __longlong_as_double((long long)(0x3FF0000000000000ull | ((uint64_t)((m >> i) & 1) << 63)));
        t = __builtin_fma(f, sgn, t);
    }
    return t;
}

// sum_r (-1)^(bit r of m) f_r, f_r = Re (IM false) or Im (IM true) of
// conj(psi_b) psi_a, a = (L, r), b = (L ^ xl, r): the partner amplitudes
// come over the cross-lane crossbar (complex64 ones as their float values,
// which the widened doubles hold exactly).
template <bool IM, typename R>
__device__ __forceinline__ double lane_sum(const double (&re)[kNR], const double (&im)[kNR], int xl, uint32_t m)
{
    double t = 0.0;
#pragma unroll
    for (int r = 0; r < kNR; ++r) {
        const double br = (double)__shfl_xor((R)re[r], xl, 64);
        const double bi = (double)__shfl_xor((R)im[r], xl, 64);
        const double f = IM ? im[r] * br - re[r] * bi : re[r] * br + im[r] * bi;
        const double sgn = __longlong_as_double((long long)(0x3FF0000000000000ull | ((uint64_t)((m >> r) & 1) << 63)));
        t = __builtin_fma(f, sgn, t);
    }
    return t;
}

__device__ __forceinline__ double lane_double(double v, int k)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
    return __hiloint2double(hi, lo);
}

template <typename R>
__global__ void __launch_bounds__(256) k_span_pass(const R* __restrict__ psi, const SpanPassK a,
                                                   double* __restrict__ partials, int pstride, int accumulate)
{
    using A = typename SV<R>::A;
    __shared__ double red[kWaves];
    const int lane = threadIdx.x & 63;
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint64_t w0 = (uint64_t)blockIdx.x * kWaves + wv;
    const uint64_t nw = (uint64_t)gridDim.x * kWaves;
    // term data in lanes (lane k: string k), fetched with readlane in the
    // tile loop; lane part of every string's sign once
    double tc = 0.0;
    uint64_t tz = 0;
    int tsgn = 0, txl = 0;
    uint64_t lsg = 0;
    for (int k = 0; k < a.nt; ++k)
        lsg |= (uint64_t)(__popcll((uint64_t)lane & a.t[k].z) & 1) << k;
    if (lane < a.nt) {
        tc = a.t[lane].c;
        tz = a.t[lane].z;
        tsgn = (int)a.t[lane].sgn;
        txl = (int)a.t[lane].xl;
    }
    const A* const p = reinterpret_cast<const A*>(psi);
    double acc = 0.0;
    for (uint64_t tl = w0; tl < a.ntiles; tl += nw) {
        const uint64_t base = insert_tile(tl, a);
        const uint64_t u = base | (uint64_t)lane;
        A v[kNR];
#pragma unroll
        for (int r = 0; r < kNR; ++r)
            v[r] = __builtin_nontemporal_load(p + (u ^ dmask(a, r)));
        double re[kNR], im[kNR];
#pragma unroll
        for (int r = 0; r < kNR; ++r) {
            re[r] = (double)v[r].x;
            im[r] = (double)v[r].y;
        }
        const uint64_t sg = lsg ^ __ballot(lane < a.nt && (__popcll(base & tz) & 1));
        double s = 0.0;
        // strings grouped by (direction, Re/Im): one loop per group with
        // the pair pattern fixed at compile time
        auto add = [&](int k, double t) {
            const double w = lane_double(tc, k) * t;
            s += ((sg >> k) & 1) ? -w : w;
        };
        auto group = [&](auto key) {
            constexpr int K = decltype(key)::value;
            for (int k = a.koff[K]; k < a.koff[K + 1]; ++k)
                add(k, string_sum<K / 2, (K & 1) != 0>(re, im, (uint32_t)__builtin_amdgcn_readlane(tsgn, k)));
        };
        group(std::integral_constant<int, 0>{});
        group(std::integral_constant<int, 1>{});
        group(std::integral_constant<int, 2>{});
        group(std::integral_constant<int, 3>{});
        group(std::integral_constant<int, 4>{});
        group(std::integral_constant<int, 5>{});
        group(std::integral_constant<int, 6>{});
        group(std::integral_constant<int, 7>{});
        group(std::integral_constant<int, 8>{});
        group(std::integral_constant<int, 9>{});
        // lane strings: the partner is in lane L ^ xl
        for (int k = a.koff[2 * kSpanDirs]; k < a.koff[2 * kSpanDirs + 1]; ++k)
            add(k, lane_sum<false, R>(re, im, __builtin_amdgcn_readlane(txl, k),
                                      (uint32_t)__builtin_amdgcn_readlane(tsgn, k)));
        for (int k = a.koff[2 * kSpanDirs + 1]; k < a.koff[kSpanGroups]; ++k)
            add(k, lane_sum<true, R>(re, im, __builtin_amdgcn_readlane(txl, k),
                                     (uint32_t)__builtin_amdgcn_readlane(tsgn, k)));
        if (a.koff[kSpanGroups] < a.nt) {
            // diagonal strings: N(m) = sum_r (-1)^popcount(r & m) |psi_(L,r)|^2
            // (five butterfly stages in place of re; the other strings are
            // done with it), read at compile-time m per group of strings
#pragma unroll
            for (int r = 0; r < kNR; ++r)
                re[r] = re[r] * re[r] + im[r] * im[r];
#pragma unroll
            for (int h = 1; h < kNR; h <<= 1)
#pragma unroll
                for (int r = 0; r < kNR; ++r)
                    if (!(r & h)) {
                        const double x0 = re[r], x1 = re[r + h];
                        re[r] = x0 + x1;
                        re[r + h] = x0 - x1;
                    }
#pragma unroll
            for (int m = 0; m < kNR; ++m)
                for (int k = a.mofs[m]; k < a.mofs[m + 1]; ++k) {
                    const double w = lane_double(tc, k) * re[m];
                    s += ((sg >> k) & 1) ? -w : w;
                }
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

template <typename R>
int span_grid()
{
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 1024;
    if (cache[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_span_pass<R>, 256, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            per_cu < 1 || cus < 1)
            return 1024;
        cache[dev] = per_cu * cus;
    }
    return cache[dev];
}

template <typename R>
hipError_t go(const SpanPassK& a, const void* psi, double* partials, int nslots, int accumulate, hipStream_t s)
{
    // every resident block once (capped by the partial slots), each wave
    // streaming tiles
    uint64_t g = (uint64_t)span_grid<R>();
    if (g > (uint64_t)nslots)
        g = (uint64_t)nslots;
    const uint64_t maxg = (a.ntiles + kWaves - 1) / kWaves;
    if (g > maxg)
        g = maxg;
    if (g < 1)
        g = 1;
    hipLaunchKernelGGL(k_span_pass<R>, dim3((unsigned)g), dim3(256), 0, s, static_cast<const R*>(psi), a,
                       partials, nslots, accumulate);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_span_pass(const SpanPassK& a, const void* psi, int dt, double* partials, int nslots,
                            int accumulate, hipStream_t s)
{
    if (a.ntiles == 0)
        return hipSuccess;
    if (a.nt < 0 || a.nt > kMaxSpanTerms)
        return hipErrorInvalidValue;
    // group offsets ascending from 0 to nt; direction and lane strings in
    // their groups; diagonal offsets from koff[kSpanGroups] to nt
    if (a.koff[0] != 0 || a.mofs[0] != a.koff[kSpanGroups] || a.mofs[1 << kSpanDirs] != a.nt)
        return hipErrorInvalidValue;
    for (int g = 0; g < kSpanGroups; ++g) {
        if (a.koff[g + 1] < a.koff[g])
            return hipErrorInvalidValue;
        for (int k = a.koff[g]; k < a.koff[g + 1]; ++k) {
            const STerm& t = a.t[k];
            const bool ok = g < 2 * kSpanDirs ? (2 * t.dir + t.im == g)
                                              : (t.dir == -1 && t.im == g - 2 * kSpanDirs && t.xl != 0 && t.xl < 64);
            if (!ok)
                return hipErrorInvalidValue;
        }
    }
    for (int m = 0; m < (1 << kSpanDirs); ++m) {
        if (a.mofs[m + 1] < a.mofs[m])
            return hipErrorInvalidValue;
        for (int k = a.mofs[m]; k < a.mofs[m + 1]; ++k)
            if ((int)a.t[k].zr != m)
                return hipErrorInvalidValue;
    }
    return dt == C64 ? go<float>(a, psi, partials, nslots, accumulate, s)
                     : go<double>(a, psi, partials, nslots, accumulate, s);
}

}  // namespace qsv
