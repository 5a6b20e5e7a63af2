// Diagonal runs: several diagonal gates applied to a state in one streaming
// sweep.  Diagonal matrices commute with each other, so the run's product
// does not depend on the order of its factors; plans build runs from
// consecutive diagonal gates (moving gates on other qubits ahead of them).
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <utility>
#include <vector>
#include <cstdlib>

#include "qsv_internal.h"

namespace qsv {

namespace {

// Block index in XCD-contiguous order (a bijection on [0, gridDim.x)).
__device__ __forceinline__ uint64_t xcd_block()
{
    const uint32_t G = gridDim.x, b = blockIdx.x, per = G >> 3;
    return b < (per << 3) ? (uint64_t)(b & 7u) * per + (b >> 3) : (uint64_t)b;
}

typedef float nv4f __attribute__((ext_vector_type(4)));
typedef double nv2d __attribute__((ext_vector_type(2)));

// 16-byte streaming loads and stores with the nontemporal hint (every line is
// touched once per sweep).
__device__ __forceinline__ float4 ld_nt(const float4* p)
{
    const nv4f v = __builtin_nontemporal_load(reinterpret_cast<const nv4f*>(p));
    return make_float4(v[0], v[1], v[2], v[3]);
}

__device__ __forceinline__ double2 ld_nt(const double2* p)
{
    const nv2d v = __builtin_nontemporal_load(reinterpret_cast<const nv2d*>(p));
    return make_double2(v[0], v[1]);
}

__device__ __forceinline__ void st_nt(float4* p, float4 v)
{
    nv4f w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<nv4f*>(p));
}

__device__ __forceinline__ void st_nt(double2* p, double2 v)
{
    nv2d w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<nv2d*>(p));
}

// A run of diagonal gates applied in one sweep (diagonal matrices commute, so
// the product's order is free): amplitude i is multiplied by d_f[tau_f(i)]
// for every factor f whose fixed bits match.  Factors are ordered by the
// varying bits (below) they read: [0, boff[0]) none, [boff[j], boff[j+1])
// only varying bit j, [boff[NV], nf) two or more.
template <typename R>
struct DiagRunK {
    uint64_t nunits;  // 16-byte units of the state
    int nf;
    int boff[6];
    uint64_t fix[kMaxRunFactors];
    uint64_t val[kMaxRunFactors];
    int tpos[kMaxRunFactors][5];
    int off[kMaxRunFactors];       // first complex entry of the factor's table
    // factors on several varying bits: fixed bits outside the varying bits
    // (matched once per thread), fixed varying bits as a mask over v, and the
    // table index bit that each varying bit sets
    uint64_t fixn[kMaxRunFactors];
    uint64_t valn[kMaxRunFactors];
    int fixv[kMaxRunFactors];
    int valv[kMaxRunFactors];
    int tvb[kMaxRunFactors][5];
    const R* tab;                  // all tables, (re, im), state precision
    int ntab;                      // complex entries in tab
    int w;                         // a thread's units differ in unit bits w..w+3 (w >= 6)
    uint64_t vmask[5];             // amplitude index bit of varying bit j
    int gafter;                    // the gate follows the diagonal (else it precedes it)
    R g[8];                        // its matrix, row-major (re, im); row 0 = target bit 0
};

// Table index of amplitude i in factor f: bit b is bit tpos[f][b] of i.
// Unused positions hold 63 (zero in every index), so the loop has a fixed
// trip count and a factor's descriptor is read in one batch of scalar loads
// rather than one dependent load per bit.
template <typename R>
__device__ __forceinline__ int run_index(const DiagRunK<R>& a, int f, uint64_t i)
{
    int t = 0;
#pragma unroll
    for (int b = 0; b < 5; ++b)
        t |= (int)((i >> a.tpos[f][b]) & 1u) << b;
    return t;
}

// Multiplies (re, im) by factor f's entry for amplitude i, if i's fixed bits
// match; the tables sit in LDS.
template <typename R>
__device__ __forceinline__ void run_factor(const DiagRunK<R>& a, const R* sd, int f, uint64_t i, R& re,
                                           R& im)
{
    if ((i & a.fix[f]) != a.val[f])
        return;
    const int t = run_index(a, f, i);
    const R dr = sd[2 * (a.off[f] + t)], di = sd[2 * (a.off[f] + t) + 1];
    const R r = re * dr - im * di;
    im = re * di + im * dr;
    re = r;
}

// Lanes cover unit bits 0..5, so every load of a wave is 64 consecutive
// units (1 KiB); each thread takes kRunUPT units that differ in the four
// unit bits w..w+3 (w >= 6, chosen by the planner), and the block's four
// waves sit on unit bits 6, 7 (w >= 8; w = 8: units 256 apart) or just above
// the window (w < 8).  So only NV index bits vary
// over its amplitudes: those four and, in complex64, amplitude bit 0 (the
// two amplitudes of a 16-byte unit).  The
// thread builds the run's product for every value v of those bits, a table
// T[v] of 2^NV entries in registers: factors that read no varying bit are
// evaluated once; a factor that reads only varying bit j contributes
// h_j(v_j), evaluated at both values, and the table is built by doubling
// over j; factors that read several varying bits are evaluated per entry.
// The sweep then multiplies each amplitude by its entry.  A long ladder of
// controlled phases on one of the varying bits costs two evaluations per
// factor and thread instead of one per factor and amplitude.
//
// A single-qubit gate whose target is a varying bit pairs amplitudes within
// the thread, so the sweep can also apply a gate that directly precedes or
// follows the run (0 <= GJ < NV, the gate's varying bit): the thread loads
// its units, applies the gate before or after the diagonal, and stores them,
// one sweep for both.  A gate on unit bit b < 6 (GJ = 8 + b) pairs each
// element with the same element of the lane whose id differs in bit b (the
// unit index's bits 0..5 are the lane id), exchanged with a lane shuffle.
constexpr int kRunUPT = 16;

template <typename R>
struct RunVary {
    static constexpr int NV = sizeof(R) == 4 ? 5 : 4;
};

template <typename R, int GJ>
__global__ void __launch_bounds__(kBlock) k_diag_run(R* __restrict__ psi, const DiagRunK<R> a)
{
    constexpr int AS = sizeof(R) == 4 ? 1 : 0;  // amplitude index = unit << AS
    constexpr int NV = RunVary<R>::NV;
    constexpr int NT = 1 << NV;
    using V2 = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
    const uint64_t seglen = (uint64_t)kBlock * kRunUPT;
    const uint64_t nseg = (a.nunits + seglen - 1) / seglen;
    __shared__ __align__(16) R sd[2 * kMaxRunEntries];
    for (int k = threadIdx.x; k < 2 * a.ntab; k += kBlock)
        sd[k] = a.tab[k];
    __syncthreads();
    // zeros inserted at k bit positions from p up
    auto ins = [](uint64_t x, int p, int k) { return ((x >> p) << (p + k)) | (x & ((1ull << p) - 1)); };
    const int wp = a.w >= 8 ? 6 : a.w + 4;  // unit bit of the wave index
    for (uint64_t seg = xcd_block(); seg < nseg; seg += gridDim.x) {
        // unit of element r: u0 | r << w; the segment fills the unit bits
        // that are neither lane, wave nor window bits
        uint64_t x = seg << 6;
        x = a.w >= 8 ? ins(ins(x, 6, 2), a.w, 4) : ins(x, a.w, 6);
        const uint64_t u0 = x | ((uint64_t)(threadIdx.x >> 6) << wp) | (threadIdx.x & 63);
        const uint64_t i0 = u0 << AS;  // varying bits zero
        R tr[NT], ti[NT];
        tr[0] = (R)1;
        ti[0] = (R)0;
        for (int f = 0; f < a.boff[0]; ++f)
            run_factor(a, sd, f, i0, tr[0], ti[0]);
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const uint64_t bj = a.vmask[j];
            R h0r = (R)1, h0i = (R)0, h1r = (R)1, h1i = (R)0;
            for (int f = a.boff[j]; f < a.boff[j + 1]; ++f) {
                run_factor(a, sd, f, i0, h0r, h0i);
                run_factor(a, sd, f, i0 | bj, h1r, h1i);
            }
#pragma unroll
            for (int v = 0; v < (1 << j); ++v) {
                const R xr = tr[v], xi = ti[v];
                tr[v + (1 << j)] = xr * h1r - xi * h1i;
                ti[v + (1 << j)] = xr * h1i + xi * h1r;
                tr[v] = xr * h0r - xi * h0i;
                ti[v] = xr * h0i + xi * h0r;
            }
        }
        for (int f = a.boff[NV]; f < a.nf; ++f) {
            if ((i0 & a.fixn[f]) != a.valn[f])
                continue;
            // table index of every entry, by doubling over the varying bits
            // from the index of the thread's fixed bits (varying bits of i0 are 0)
            const int t0 = run_index(a, f, i0);
            // each varying bit adds a table bit that is clear in tt[v], so + is |
            int tt[NT];
            tt[0] = a.off[f] + t0;
#pragma unroll
            for (int j = 0; j < NV; ++j)
#pragma unroll
                for (int v = 0; v < (1 << j); ++v)
                    tt[v + (1 << j)] = tt[v] + a.tvb[f][j];
            const V2* e = reinterpret_cast<const V2*>(sd);
            if (a.fixv[f] == 0) {
#pragma unroll
                for (int v = 0; v < NT; ++v) {
                    const V2 d = e[tt[v]];
                    const R xr = tr[v], xi = ti[v];
                    tr[v] = xr * d.x - xi * d.y;
                    ti[v] = xr * d.y + xi * d.x;
                }
            } else {
#pragma unroll
                for (int v = 0; v < NT; ++v) {
                    const bool hit = (v & a.fixv[f]) == a.valv[f];
                    const V2 d = e[tt[v]];
                    const R dr = hit ? d.x : (R)1, di = hit ? d.y : (R)0;
                    const R xr = tr[v], xi = ti[v];
                    tr[v] = xr * dr - xi * di;
                    ti[v] = xr * di + xi * dr;
                }
            }
        }
        if constexpr (GJ >= 0) {
            static_assert(GJ < NV || (GJ >= 8 && GJ < 14), "gate bit");
            // the planner folds a gate only where every unit of the window
            // exists (no tail), so pairs never mix loaded and missing units
            constexpr int NE = NT;
            R er[NE], ei[NE];
#pragma unroll
            for (int r = 0; r < kRunUPT; ++r) {
                const uint64_t u = u0 | ((uint64_t)r << a.w);
                if constexpr (sizeof(R) == 4) {
                    const float4 x = u < a.nunits ? ld_nt(&reinterpret_cast<float4*>(psi)[u]) : make_float4(0, 0, 0, 0);
                    er[2 * r] = x.x;
                    ei[2 * r] = x.y;
                    er[2 * r + 1] = x.z;
                    ei[2 * r + 1] = x.w;
                } else {
                    const double2 x = u < a.nunits ? ld_nt(&reinterpret_cast<double2*>(psi)[u]) : make_double2(0, 0);
                    er[r] = x.x;
                    ei[r] = x.y;
                }
            }
            auto gate = [&]() {
                if constexpr (GJ < NV) {
                    // element pairs (e, e | 2^GJ) within the thread
#pragma unroll
                    for (int e = 0; e < NE; ++e)
                        if (!((e >> GJ) & 1)) {
                            const int h = e | (1 << GJ);
                            const R ar = er[e], ai = ei[e], br = er[h], bi = ei[h];
                            er[e] = a.g[0] * ar - a.g[1] * ai + a.g[2] * br - a.g[3] * bi;
                            ei[e] = a.g[0] * ai + a.g[1] * ar + a.g[2] * bi + a.g[3] * br;
                            er[h] = a.g[4] * ar - a.g[5] * ai + a.g[6] * br - a.g[7] * bi;
                            ei[h] = a.g[4] * ai + a.g[5] * ar + a.g[6] * bi + a.g[7] * br;
                        }
                } else {
                    // the same element of lane ^ 2^(GJ - 8): this lane's row of
                    // the matrix (row 0 if its bit is 0) times (mine, other)
                    constexpr int LM = 1 << (GJ - 8);
                    const bool hi = (threadIdx.x & LM) != 0;
                    const R mr0 = hi ? a.g[6] : a.g[0], mi0 = hi ? a.g[7] : a.g[1];
                    const R or0 = hi ? a.g[4] : a.g[2], oi0 = hi ? a.g[5] : a.g[3];
#pragma unroll
                    for (int e = 0; e < NE; ++e) {
                        const R pr = __shfl_xor(er[e], LM), pi = __shfl_xor(ei[e], LM);
                        const R xr = er[e], xi = ei[e];
                        er[e] = mr0 * xr - mi0 * xi + or0 * pr - oi0 * pi;
                        ei[e] = mr0 * xi + mi0 * xr + or0 * pi + oi0 * pr;
                    }
                }
            };
            if (!a.gafter)
                gate();
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const R xr = er[e], xi = ei[e];
                er[e] = tr[e] * xr - ti[e] * xi;
                ei[e] = tr[e] * xi + ti[e] * xr;
            }
            if (a.gafter)
                gate();
#pragma unroll
            for (int r = 0; r < kRunUPT; ++r) {
                const uint64_t u = u0 | ((uint64_t)r << a.w);
                if (u >= a.nunits)
                    continue;
                if constexpr (sizeof(R) == 4)
                    st_nt(&reinterpret_cast<float4*>(psi)[u], make_float4(er[2 * r], ei[2 * r], er[2 * r + 1], ei[2 * r + 1]));
                else
                    st_nt(&reinterpret_cast<double2*>(psi)[u], make_double2(er[r], ei[r]));
            }
        } else {
#pragma unroll
            for (int r = 0; r < kRunUPT; ++r) {
                const uint64_t u = u0 | ((uint64_t)r << a.w);
                if (u >= a.nunits)
                    break;
                if constexpr (sizeof(R) == 4) {
                    float4* p = reinterpret_cast<float4*>(psi);
                    const float4 x = ld_nt(&p[u]);
                    const float ar = tr[2 * r], ai = ti[2 * r], br = tr[2 * r + 1], bi = ti[2 * r + 1];
                    st_nt(&p[u], make_float4(ar * x.x - ai * x.y, ar * x.y + ai * x.x, br * x.z - bi * x.w,
                                               br * x.w + bi * x.z));
                } else {
                    double2* p = reinterpret_cast<double2*>(psi);
                    const double2 x = ld_nt(&p[u]);
                    st_nt(&p[u], make_double2(tr[r] * x.x - ti[r] * x.y, tr[r] * x.y + ti[r] * x.x));
                }
            }
        }
    }
}

inline unsigned run_grid(uint64_t units)
{
    uint64_t b = (units + (uint64_t)kBlock * kRunUPT - 1) / ((uint64_t)kBlock * kRunUPT);
    if (b < 1)
        b = 1;
    if (b > (1u << 23) - 1)
        b = (1u << 23) - 1;
    return (unsigned)b;
}

template <typename R>
hipError_t diag_run_go(const GateLaunch& L, void* p, hipStream_t s)
{
    constexpr int NV = RunVary<R>::NV;
    constexpr int AS = sizeof(R) == 4 ? 1 : 0;
    // the window must lie inside the unit index, and a folded gate needs
    // every unit of it (no tail)
    const int w = L.run_w;
    const uint64_t span = 1ull << (w >= 8 ? w + 4 : w + 6);  // units the thread and wave bits reach
    if (w < 6 || w > 58 || ((w != 8 || L.run_gate) && L.ngroups < span))
        return hipErrorInvalidValue;
    // varying bits: (complex64) amplitude bit 0, then unit bits w..w+3
    uint64_t vmask[NV];
    for (int j = 0; j < NV; ++j)
        vmask[j] = AS ? (j == 0 ? 1ull : 1ull << (w + j)) : 1ull << (w + j);
    // order the factors by the varying bits they read (see DiagRunK)
    std::vector<std::pair<int, int>> order;  // (class, factor)
    for (int f = 0; f < L.run_nf; ++f) {
        uint64_t dep = L.run_fix[f];
        for (int b = 0; b < L.run_nt[f]; ++b)
            dep |= 1ull << L.run_tpos[f][b];
        int cls = 0, nread = 0;
        for (int j = 0; j < NV; ++j)
            if (dep & vmask[j]) {
                cls = j + 1;
                ++nread;
            }
        order.push_back({nread >= 2 ? NV + 1 : cls, f});
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<int, int>& x, const std::pair<int, int>& y) { return x.first < y.first; });
    DiagRunK<R> a{};
    a.nunits = L.ngroups;
    a.nf = L.run_nf;
    for (int k = 0; k < L.run_nf; ++k) {
        const int f = order[k].second;
        a.fix[k] = L.run_fix[f];
        a.val[k] = L.run_val[f];
        a.off[k] = L.run_off[f];
        for (int b = 0; b < 5; ++b)
            a.tpos[k][b] = b < L.run_nt[f] ? L.run_tpos[f][b] : 63;
        uint64_t vall = 0;
        for (int j = 0; j < NV; ++j) {
            vall |= vmask[j];
            if (L.run_fix[f] & vmask[j]) {
                a.fixv[k] |= 1 << j;
                if (L.run_val[f] & vmask[j])
                    a.valv[k] |= 1 << j;
            }
            for (int b = 0; b < L.run_nt[f]; ++b)
                if (L.run_tpos[f][b] == __builtin_ctzll(vmask[j]))
                    a.tvb[k][j] = 1 << b;
        }
        a.fixn[k] = L.run_fix[f] & ~vall;
        a.valn[k] = L.run_val[f] & ~vall;
    }
    for (int j = 0; j <= NV; ++j) {
        int c = 0;
        while (c < L.run_nf && order[c].first <= j)
            ++c;
        a.boff[j] = c;  // factors of class <= j come first
    }
    a.tab = static_cast<const R*>(L.gdev);
    a.ntab = (int)(L.run_tab.size() / 2);
    if (!a.tab || a.ntab > kMaxRunEntries)
        return hipErrorInvalidValue;
    a.w = w;
    for (int j = 0; j < NV; ++j)
        a.vmask[j] = vmask[j];
    int gjt = -1;  // the gate's varying bit, or 8 + its unit bit below 6
    if (L.run_gate) {
        for (int j = 0; j < NV; ++j)
            if (vmask[j] == 1ull << L.run_gt)
                gjt = j;
        const int tb = L.run_gt - AS;  // the target's unit bit
        if (gjt < 0 && tb >= 0 && tb < 6)
            gjt = 8 + tb;
        if (gjt < 0)
            return hipErrorInvalidValue;
        a.gafter = L.run_gate == 2;
        for (int k = 0; k < 8; ++k)
            a.g[k] = (R)L.run_g[k];
    }
    const dim3 grid(run_grid(a.nunits)), block(kBlock);
    R* ps = static_cast<R*>(p);
    switch (gjt) {
    case -1: hipLaunchKernelGGL((k_diag_run<R, -1>), grid, block, 0, s, ps, a); break;
    case 0: hipLaunchKernelGGL((k_diag_run<R, 0>), grid, block, 0, s, ps, a); break;
    case 1: hipLaunchKernelGGL((k_diag_run<R, 1>), grid, block, 0, s, ps, a); break;
    case 2: hipLaunchKernelGGL((k_diag_run<R, 2>), grid, block, 0, s, ps, a); break;
    case 3: hipLaunchKernelGGL((k_diag_run<R, 3>), grid, block, 0, s, ps, a); break;
    case 4: hipLaunchKernelGGL((k_diag_run<R, NV - 1>), grid, block, 0, s, ps, a); break;
    case 8: hipLaunchKernelGGL((k_diag_run<R, 8>), grid, block, 0, s, ps, a); break;
    case 9: hipLaunchKernelGGL((k_diag_run<R, 9>), grid, block, 0, s, ps, a); break;
    case 10: hipLaunchKernelGGL((k_diag_run<R, 10>), grid, block, 0, s, ps, a); break;
    case 11: hipLaunchKernelGGL((k_diag_run<R, 11>), grid, block, 0, s, ps, a); break;
    case 12: hipLaunchKernelGGL((k_diag_run<R, 12>), grid, block, 0, s, ps, a); break;
    case 13: hipLaunchKernelGGL((k_diag_run<R, 13>), grid, block, 0, s, ps, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_diag_run(const GateLaunch& L, void* psi, hipStream_t s)
{
    if (L.ngroups == 0)
        return hipSuccess;
    return L.dt == C64 ? diag_run_go<float>(L, psi, s) : diag_run_go<double>(L, psi, s);
}

}  // namespace qsv
