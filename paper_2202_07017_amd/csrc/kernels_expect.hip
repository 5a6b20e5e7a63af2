// Tiled Pauli-sum passes: <psi|H|psi> partial sums and lambda = H psi.
//
// A pass loads tiles of 2^12 amplitudes into LDS.  A tile is a set B of 12
// qubits: a contiguous run of low qubits [0, L) (L >= 6, so loads are
// >= 512-byte contiguous chunks) plus up to 12 - L higher qubits.  Every Pauli
// term whose x mask lies inside B pairs amplitudes of the same tile, so one
// read of the state serves all of them; the terms of a Hamiltonian are split
// into passes by their x masks on the host.
//
// Phases i^(y + 2 popcount(i & z)) are split into a per-tile part
// (popcount(base & z)) and a local part (popcount(l & zloc), zloc = z
// compressed onto B).  Diagonal terms are folded per tile into two tables
// WA[l mod 64] and WB[l div 64] (terms whose local mask lies in one half) plus
// a short list of terms that straddle both halves, so the diagonal weight of
// an amplitude costs two LDS reads however many diagonal terms there are.
#include "qsv_expect.h"

namespace qsv {
namespace {

constexpr int kM = kTileQubits;   // 12
constexpr int kTA = 1 << kM;      // amplitudes per tile
constexpr int kThreads = 256;

template <typename R>
struct EV;
template <>
struct EV<float> {
    using V = float4;
    static constexpr int APV = 2;
};
template <>
struct EV<double> {
    using V = double2;
    static constexpr int APV = 1;
};

struct C2 {
    double re, im;
};

__device__ __forceinline__ uint64_t insert_bits(uint64_t g, const InsertSpec& s)
{
    for (int j = 0; j < s.nins; ++j) {
        const uint64_t lo = s.low[j];
        g = ((g & ~lo) << 1) | (g & lo);
    }
    return g;
}

// i^e for e in 0..3
__device__ __forceinline__ C2 ipow(int e)
{
    e &= 3;
    return C2{e == 0 ? 1.0 : (e == 2 ? -1.0 : 0.0), e == 1 ? 1.0 : (e == 3 ? -1.0 : 0.0)};
}

__device__ __forceinline__ float vcomp(const float4& v, int c)
{
    return c == 0 ? v.x : (c == 1 ? v.y : (c == 2 ? v.z : v.w));
}
__device__ __forceinline__ double vcomp(const double2& v, int c)
{
    return c == 0 ? v.x : v.y;
}
__device__ __forceinline__ float4 mkv(const float* o)
{
    return make_float4(o[0], o[1], o[2], o[3]);
}
__device__ __forceinline__ double2 mkv(const double* o)
{
    return make_double2(o[0], o[1]);
}

template <typename R>
__device__ __forceinline__ C2 lds_amp(const R* t, uint32_t l)
{
    return C2{(double)t[2 * l], (double)t[2 * l + 1]};
}

// Shared state of a tile pass.
struct TileShared {
    double wa[64];
    double wb[kTA / 64];
    int tphase[kMaxTileTerms];  // per-term tile phase offset: y + 2 popcount(base & z)
    double red[2][kThreads / 64];
};

// Per tile: tile phase offsets for every term and the diagonal tables.
__device__ void tile_prologue(const TileExpK& a, uint64_t base, TileShared& sh)
{
    for (int t = threadIdx.x; t < a.nt; t += blockDim.x)
        sh.tphase[t] = a.t[t].ylo + 2 * __popcll(base & a.t[t].z);
    if (a.ndiag == 0)
        return;
    for (int e = threadIdx.x; e < 64 + kTA / 64; e += blockDim.x) {
        const bool lowhalf = e < 64;
        const uint32_t v = lowhalf ? (uint32_t)e : (uint32_t)(e - 64) << 6;
        double w = 0.0;
        for (int t = a.nstr; t < a.pstart; ++t) {
            const XTerm& T = a.t[t];
            if (T.dpart != (lowhalf ? 1 : 2))
                continue;
            const int par = (__popcll(base & T.z) + __popc(v & T.zloc)) & 1;
            w += par ? -T.c : T.c;
        }
        if (lowhalf)
            sh.wa[e] = w;
        else
            sh.wb[e - 64] = w;
    }
}

// Diagonal weight of local amplitude l (tables + straddling terms).
__device__ __forceinline__ double diag_weight(const TileExpK& a, const TileShared& sh, uint32_t l)
{
    double w = sh.wa[l & 63] + sh.wb[l >> 6];
    for (int t = 0; t < a.nstr; ++t) {
        const XTerm& T = a.t[t];
        w += ((sh.tphase[t] >> 1) + __popc(l & T.zloc)) & 1 ? -T.c : T.c;
    }
    return w;
}

template <typename R, bool HPSI>
__global__ void __launch_bounds__(kThreads) k_tile_pass(const R* __restrict__ psi, R* __restrict__ lam,
                                                        const TileExpK a, double* partials,
                                                        int accumulate)
{
    using V = typename EV<R>::V;
    constexpr int APV = EV<R>::APV;
    constexpr int VPT = kTA / APV / kThreads;
    __shared__ R tile[2 * kTA];
    __shared__ TileShared sh;

    uint64_t goff[VPT];
    uint32_t loc[VPT];
#pragma unroll
    for (int r = 0; r < VPT; ++r) {
        const uint32_t l = (uint32_t)(threadIdx.x + kThreads * r) * APV;
        loc[r] = l;
        goff[r] = a.choff[l >> a.L] + (l & ((1u << a.L) - 1));
    }
    double sr = 0.0, si = 0.0;
    for (uint64_t tl = blockIdx.x; tl < a.ntiles; tl += gridDim.x) {
        const uint64_t base = insert_bits(tl, a.ins);
        V own[VPT];
#pragma unroll
        for (int r = 0; r < VPT; ++r) {
            own[r] = *reinterpret_cast<const V*>(psi + 2 * (base + goff[r]));
            *reinterpret_cast<V*>(tile + 2 * loc[r]) = own[r];
        }
        tile_prologue(a, base, sh);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < VPT; ++r) {
            R outv[2 * APV];
#pragma unroll
            for (int h = 0; h < APV; ++h) {
                const uint32_t l = loc[r] + h;
                const C2 p{(double)vcomp(own[r], 2 * h), (double)vcomp(own[r], 2 * h + 1)};
                C2 lsum{0.0, 0.0};
                if (a.ndiag) {
                    const double w = diag_weight(a, sh, l);
                    if (HPSI) {
                        lsum.re += w * p.re;
                        lsum.im += w * p.im;
                    } else {
                        sr += w * (p.re * p.re + p.im * p.im);
                    }
                }
                for (int t = a.pstart; t < a.nt; ++t) {
                    const XTerm& T = a.t[t];
                    const uint32_t lj = l ^ T.xloc;
                    if (HPSI) {
                        // (P psi)[i] = i^(phase of j) psi[j], j = i xor x
                        const C2 q = lds_amp(tile, lj);
                        if (T.kind == 2) {
                            lsum.re += T.c * q.re;
                            lsum.im += T.c * q.im;
                        } else {
                            const C2 f = ipow(sh.tphase[t] + 2 * __popc(lj & T.zloc));
                            lsum.re += T.c * (f.re * q.re - f.im * q.im);
                            lsum.im += T.c * (f.re * q.im + f.im * q.re);
                        }
                    } else {
                        if (l & T.hloc)
                            continue;  // the pair is counted by its lower member
                        const C2 q = lds_amp(tile, lj);
                        const double wr = q.re * p.re + q.im * p.im;  // conj(q) p
                        const double wi = q.re * p.im - q.im * p.re;
                        if (T.kind == 2) {
                            sr += 2.0 * T.c * wr;
                        } else {
                            const C2 fi = ipow(sh.tphase[t] + 2 * __popc(l & T.zloc));
                            const C2 fj = ipow(sh.tphase[t] + 2 * __popc(lj & T.zloc));
                            const double pr = fi.re + fj.re, pi = fi.im - fj.im;
                            const double qr = fi.re - fj.re, qi = fi.im + fj.im;
                            sr += T.c * (wr * pr - wi * pi);
                            si += T.c * (wr * qi + wi * qr);
                        }
                    }
                }
                if (HPSI) {
                    if (accumulate) {
                        const R* lv = lam + 2 * (base + goff[r] + h);
                        lsum.re += (double)lv[0];
                        lsum.im += (double)lv[1];
                    }
                    outv[2 * h] = (R)lsum.re;
                    outv[2 * h + 1] = (R)lsum.im;
                }
            }
            if (HPSI)
                *reinterpret_cast<V*>(lam + 2 * (base + goff[r])) = mkv(outv);
        }
        __syncthreads();
    }
    if (!HPSI) {
        for (int off = 32; off > 0; off >>= 1) {
            sr += __shfl_xor(sr, off, 64);
            si += __shfl_xor(si, off, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            sh.red[0][threadIdx.x >> 6] = sr;
            sh.red[1][threadIdx.x >> 6] = si;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a0 = 0.0, a1 = 0.0;
            for (int w = 0; w < kThreads / 64; ++w) {
                a0 += sh.red[0][w];
                a1 += sh.red[1][w];
            }
            double* p = partials + blockIdx.x;
            double* q = partials + gridDim.x + blockIdx.x;
            *p = accumulate ? *p + a0 : a0;
            *q = accumulate ? *q + a1 : a1;
        }
    }
}

}  // namespace

hipError_t launch_tile_pass(const TileExpK& a, const void* psi, void* lam, int dt, bool hpsi,
                            double* partials, int nblocks, int accumulate, hipStream_t s)
{
    if (a.ntiles == 0)
        return hipSuccess;
    unsigned blocks = (unsigned)nblocks;
    if (hpsi) {
        const uint64_t b = a.ntiles < 4096 ? a.ntiles : 4096;
        blocks = (unsigned)b;
    }
    if (dt == C64) {
        if (hpsi)
            hipLaunchKernelGGL((k_tile_pass<float, true>), dim3(blocks), dim3(kThreads), 0, s,
                               static_cast<const float*>(psi), static_cast<float*>(lam), a, partials,
                               accumulate);
        else
            hipLaunchKernelGGL((k_tile_pass<float, false>), dim3(blocks), dim3(kThreads), 0, s,
                               static_cast<const float*>(psi), static_cast<float*>(lam), a, partials,
                               accumulate);
    } else {
        if (hpsi)
            hipLaunchKernelGGL((k_tile_pass<double, true>), dim3(blocks), dim3(kThreads), 0, s,
                               static_cast<const double*>(psi), static_cast<double*>(lam), a, partials,
                               accumulate);
        else
            hipLaunchKernelGGL((k_tile_pass<double, false>), dim3(blocks), dim3(kThreads), 0, s,
                               static_cast<const double*>(psi), static_cast<double*>(lam), a, partials,
                               accumulate);
    }
    return hipGetLastError();
}

}  // namespace qsv
