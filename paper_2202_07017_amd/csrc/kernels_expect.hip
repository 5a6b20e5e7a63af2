// Tiled Pauli-sum passes: <psi|H|psi> partial sums and lambda = H psi.
//
// A pass loads tiles of 2^12 amplitudes into LDS.  A tile is a set B of 12
// qubits: a contiguous run of low qubits [0, L) (L >= 6, so loads are
// >= 512-byte contiguous chunks) plus up to 12 - L higher qubits.  Every Pauli
// term whose x mask lies inside B pairs amplitudes of the same tile, so one
// read of the state serves all of them; the terms of a Hamiltonian are split
// into passes by their x masks on the host.
//
// A tile is held in LDS in FP64 (both state precisions), so each term costs
// one 16-byte LDS read and two FMAs per amplitude.
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
constexpr int kThreads = 512;
constexpr int kAPT = kTA / kThreads;  // amplitudes per thread (8)

// native vector types (not HIP's float4 / double2 classes): a loop-carried
// array of them stays in registers
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename R>
struct EV;
template <>
struct EV<float> {
    using V = f32x4;  // two amplitudes
    static constexpr int APV = 2;
};
template <>
struct EV<double> {
    using V = f64x2;  // one amplitude
    static constexpr int APV = 1;
};

struct C2 {
    double re, im;
};

// Tile base index: zeros inserted at the kTileQubits tile positions (a fixed
// count, so the masks stay in scalar registers across the tile loop).
__device__ __forceinline__ uint64_t insert_tile(uint64_t g, const InsertSpec& s)
{
#pragma unroll
    for (int j = 0; j < kTileQubits; ++j) {
        const uint64_t lo = s.low[j];
        g = ((g & ~lo) << 1) | (g & lo);
    }
    return g;
}

// Values read from LDS at a uniform address, moved to scalar registers.
__device__ __forceinline__ uint32_t uni(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ double uni(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    return __builtin_bit_cast(double, lo | (hi << 32));
}

__device__ __forceinline__ C2 lds_amp(const f64x2* t, uint32_t l)
{
    const f64x2 v = t[l];
    return C2{v.x, v.y};
}

// Shared state of a tile pass.  The pass's terms are staged here once per
// block, so the loops over terms read LDS only (a scalar memory load in such
// a loop shares its wait counter with the LDS reads and serialises them).
struct TileShared {
    double wa[64];                 // static diagonal table, local bits 0..5 (per block)
    double wb[kTA / 64];           // static diagonal table, local bits 6..11 (per block)
    double ce[kMaxTileTerms + 1];  // coefficient with its sign for the current tile
    double c[kMaxTileTerms];
    uint64_t z[kMaxTileTerms];
    uint32_t zl[kMaxTileTerms + 1];
    uint32_t xl[kMaxTileTerms + 1];
    int32_t ylo[kMaxTileTerms];
    double wout;                   // diagonal terms wholly outside the tile, this tile
    double red[2][kThreads / 64];
};

// Adds c * i^e * psi_j to h for the amplitudes of a thread, for a pair term
// with uniform swap (e odd) and per-amplitude sign (bit 1 of e).
template <bool SWP>
__device__ __forceinline__ void pair_term(const f64x2* tile, uint32_t A, double c, uint32_t sl,
                                          const uint32_t (&sk)[kAPT], C2 (&hs)[kAPT])
{
#pragma unroll
    for (int j = 0; j < kAPT; ++j) {
        const C2 q = lds_amp(tile, A ^ (uint32_t)(kThreads * j));
        const double cs = ((sl ^ sk[j]) & 1) ? -c : c;
        hs[j].re += cs * (SWP ? -q.im : q.re);
        hs[j].im += cs * (SWP ? q.re : q.im);
    }
}

// One kernel for both products: every amplitude i of a tile gets
// h_i = w_i psi_i + sum_t c_t i^e_t(j) psi_j (j = i xor x_t, the terms of the
// pass), i.e. (H psi)_i restricted to the pass.  HPSI stores (or adds) h;
// otherwise the block sums conj(psi_i) h_i, whose total over all passes is
// <psi|H|psi>.  Terms are the outer loop over the 8 amplitudes of a thread,
// so each term's data is read once and its 8 LDS partner reads are in flight
// together.
//
// Indexing: amplitude j of a thread has local index lt | K_j with lt =
// threadIdx.x and K_j = kThreads * j (consecutive lanes read consecutive LDS
// words: no bank conflicts).  Global offsets, partner indices and phase
// parities are linear in the local bits, so the K_j parts are uniform
// (scalar) and a lane keeps only lt.  The grid is one block per resident
// slot.
//
// Per tile, wave 0 gives every tile-dependent term its sign for this tile
// (from popcount(base & z)) while the tile is written to LDS; everything
// else about the terms is fixed per block.
template <typename R, bool HPSI>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) k_tile_pass(const R* __restrict__ psi, R* __restrict__ lam,
                                                        const TileExpK a, double* partials,
                                                        int pstride, int accumulate)
{
    using V = typename EV<R>::V;
    constexpr int APV = EV<R>::APV;
    constexpr int VPT = kTA / APV / kThreads;  // loaded vectors per thread
    __shared__ f64x2 tile[kTA];
    __shared__ TileShared sh;

    const int tid = threadIdx.x;
    // stage the terms, then fold the static table terms into the tables
    for (int k = tid; k < a.nt; k += kThreads) {
        const XTerm& T = a.t[k];
        sh.c[k] = T.c;
        sh.ce[k] = T.c;
        sh.z[k] = T.z;
        sh.zl[k] = T.zloc;
        sh.xl[k] = T.xloc;
        sh.ylo[k] = T.ylo;
    }
    if (tid == 0) {  // one padding entry: the term loops read one ahead
        sh.ce[a.nt] = 0.0;
        sh.zl[a.nt] = 0;
        sh.xl[a.nt] = 0;
        sh.wout = 0.0;
    }
    __syncthreads();
    if (a.ndiag) {
        for (int e = tid; e < 64 + kTA / 64; e += kThreads) {
            const bool lowhalf = e < 64;
            const uint32_t v = lowhalf ? (uint32_t)e : (uint32_t)(e - 64) << 6;
            double w = 0.0;
            for (int k = a.no; k < a.pstart; ++k) {
                const uint32_t zl = sh.zl[k];
                const bool inlow = (zl & ~63u) == 0;  // includes the identity (zl = 0)
                if (inlow != lowhalf)
                    continue;
                w += (__popc(v & zl) & 1) ? -sh.c[k] : sh.c[k];
            }
            if (lowhalf)
                sh.wa[e] = w;
            else
                sh.wb[e - 64] = w;
        }
    }

    const uint32_t lmask = (1u << a.L) - 1;
    auto goff = [&](uint32_t l) { return a.choff[l >> a.L] + (l & lmask); };
    const uint64_t gv = goff(tid * APV);  // lane part of the load offsets
    const uint64_t gt = goff(tid);        // lane part of the compute offsets
    uint64_t uo[VPT];                     // uniform parts of the load offsets
#pragma unroll
    for (int r = 0; r < VPT; ++r)
        uo[r] = goff(APV * kThreads * r);
    uint64_t us[HPSI ? kAPT : 1];         // uniform parts of the store offsets (H psi)
#pragma unroll
    for (int j = 0; j < (HPSI ? kAPT : 1); ++j)
        us[j] = goff((uint32_t)(kThreads * j));
    double er = 0.0, ei = 0.0;
    // complex64 prefetches the next tile into registers; complex128 (twice
    // the registers per amplitude) loads each tile at the top of its iteration
    constexpr bool PF = APV == 2;
    V nxt[VPT];
    if (PF && blockIdx.x < a.ntiles) {
        const uint64_t b = insert_tile(blockIdx.x, a.ins);
#pragma unroll
        for (int r = 0; r < VPT; ++r)
            nxt[r] = *reinterpret_cast<const V*>(psi + 2 * (b + uo[r] + gv));
    }
    for (uint64_t tl = blockIdx.x; tl < a.ntiles; tl += gridDim.x) {
        const uint64_t base = insert_tile(tl, a.ins);
        if (!PF) {
            uint64_t gvl = gv;
            asm volatile("" : "+v"(gvl));
#pragma unroll
            for (int r = 0; r < VPT; ++r)
                nxt[r] = *reinterpret_cast<const V*>(psi + 2 * (base + uo[r] + gvl));
        }
#pragma unroll
        for (int r = 0; r < VPT; ++r) {
            const uint32_t l = APV * (tid + kThreads * r);
            if (APV == 2) {
                tile[l] = f64x2{(double)nxt[r][0], (double)nxt[r][1]};
                tile[l + 1] = f64x2{(double)nxt[r][2], (double)nxt[r][3]};
            } else {
                tile[l] = f64x2{(double)nxt[r][0], (double)nxt[r][1]};
            }
        }
        if (tid < 64) {
            // this tile's signs: diagonal terms reaching outside the tile and
            // pair terms (phase i^ylo (-1)^popcount(base & z) of their base part)
            const int k = tid;
            double wo = 0.0;
            if (k >= a.nx && k < a.no) {
                const double cs = (__popcll(base & sh.z[k]) & 1) ? -sh.c[k] : sh.c[k];
                if (k < a.nd)
                    sh.ce[k] = cs;
                else
                    wo = cs;
            } else if (k >= a.pstart && k < a.nt) {
                const int e = (sh.ylo[k] >> 1) + __popcll(base & sh.z[k]);
                sh.ce[k] = (e & 1) ? -sh.c[k] : sh.c[k];
            }
            if (a.no > a.nd) {
                for (int off = 32; off > 0; off >>= 1)
                    wo += __shfl_xor(wo, off, 64);
                if (k == 0)
                    sh.wout = wo;
            }
        }
        __syncthreads();
        if (PF) {
            // next tile (the last one reloads itself: no branch around the
            // loads); the opaque lane offset keeps the VPT sums with the
            // uniform parts from being hoisted into registers
            const uint64_t tn = tl + gridDim.x < a.ntiles ? tl + gridDim.x : tl;
            const uint64_t b = insert_tile(tn, a.ins);
            uint64_t gvl = gv;
            asm volatile("" : "+v"(gvl));
#pragma unroll
            for (int r = 0; r < VPT; ++r)
                nxt[r] = *reinterpret_cast<const V*>(psi + 2 * (b + uo[r] + gvl));
        }
        // opaque copy of the lane index: keeps the compiler from hoisting the
        // per-amplitude LDS addresses out of the tile loop into registers
        uint32_t lt = tid;
        asm volatile("" : "+v"(lt));
        C2 hs[kAPT];
        {
            double w[kAPT];
            const double w0 = a.ndiag ? sh.wout : 0.0;
#pragma unroll
            for (int j = 0; j < kAPT; ++j) {
                const uint32_t l = lt | (uint32_t)(kThreads * j);
                w[j] = a.ndiag ? sh.wa[l & 63] + sh.wb[l >> 6] + w0 : 0.0;
            }
            // diagonal terms with a per-amplitude sign that no table holds
            uint32_t zl = uni(sh.zl[0]);
            double c = uni(sh.ce[0]);
#pragma unroll 1
            for (int k = 0; k < a.nd; ++k) {
                const uint32_t zl1 = sh.zl[k + 1];
                const double c1 = sh.ce[k + 1];
                const uint32_t sl = (uint32_t)__popc(lt & zl);
#pragma unroll
                for (int j = 0; j < kAPT; ++j)
                    w[j] += ((sl ^ (uint32_t)__popc((uint32_t)(kThreads * j) & zl)) & 1) ? -c : c;
                zl = uni(zl1);
                c = uni(c1);
            }
            if (a.ndiag) {
#pragma unroll
                for (int j = 0; j < kAPT; ++j) {  // psi_i is re-read at the end: not live across the terms
                    const C2 p = lds_amp(tile, lt | (uint32_t)(kThreads * j));
                    hs[j] = C2{w[j] * p.re, w[j] * p.im};
                }
            } else {
#pragma unroll
                for (int j = 0; j < kAPT; ++j)
                    hs[j] = C2{0.0, 0.0};
            }
        }
        {
            // pure X strings; the next term's data is read ahead
            uint32_t x = uni(sh.xl[a.pstart]);
            double c = uni(sh.ce[a.pstart]);
#pragma unroll 1
            for (int k = a.pstart; k < a.pxend; ++k) {
                const uint32_t x1 = sh.xl[k + 1];
                const double c1 = sh.ce[k + 1];
                const uint32_t A = lt ^ x;  // partner of lt | K_j is A ^ K_j
                if ((x & ~(uint32_t)(kThreads - 1)) == 0) {
                    // x only in lane bits: A ^ K_j = A + K_j, immediate LDS offsets
                    const f64x2* tp = tile + A;
#pragma unroll
                    for (int j = 0; j < kAPT; ++j) {
                        const f64x2 q = tp[kThreads * j];
                        hs[j].re += c * q.x;
                        hs[j].im += c * q.y;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < kAPT; ++j) {
                        const C2 q = lds_amp(tile, A ^ (uint32_t)(kThreads * j));
                        hs[j].re += c * q.re;
                        hs[j].im += c * q.im;
                    }
                }
                x = uni(x1);
                c = uni(c1);
            }
        }
        {
            // (P psi)_i = i^e psi_j, e = y + 2 popcount(j & z): bit 0 of e is
            // uniform, bit 1 is the parity of the tile part (in ce) and of
            // the local part
            uint32_t x = uni(sh.xl[a.pxend]), zl = uni(sh.zl[a.pxend]);
            double c = uni(sh.ce[a.pxend]);
#pragma unroll 1
            for (int k = a.pxend; k < a.nt; ++k) {
                const uint32_t x1 = sh.xl[k + 1], zl1 = sh.zl[k + 1];
                const double c1 = sh.ce[k + 1];
                const bool odd = uni((uint32_t)sh.ylo[k]) & 1;
                const uint32_t A = lt ^ x;
                const uint32_t sl = (uint32_t)__popc(A & zl);
                uint32_t sk[kAPT];
#pragma unroll
                for (int j = 0; j < kAPT; ++j)
                    sk[j] = (uint32_t)__popc((uint32_t)(kThreads * j) & zl);
                if (odd)
                    pair_term<true>(tile, A, c, sl, sk, hs);
                else
                    pair_term<false>(tile, A, c, sl, sk, hs);
                x = uni(x1);
                zl = uni(zl1);
                c = uni(c1);
            }
        }
        if (HPSI) {
#pragma unroll
            for (int j = 0; j < kAPT; ++j) {
                R* dst = lam + 2 * (base + gt + us[HPSI ? j : 0]);
                C2 o = hs[j];
                if (accumulate) {
                    o.re += (double)dst[0];
                    o.im += (double)dst[1];
                }
                dst[0] = (R)o.re;
                dst[1] = (R)o.im;
            }
        } else {
            uint32_t lt2 = lt;  // opaque: a fresh read, not values kept from the start
            asm volatile("" : "+v"(lt2));
#pragma unroll
            for (int j = 0; j < kAPT; ++j) {
                const C2 p = lds_amp(tile, lt2 | (uint32_t)(kThreads * j));
                er += p.re * hs[j].re + p.im * hs[j].im;  // conj(psi_i) h_i
                ei += p.re * hs[j].im - p.im * hs[j].re;
            }
        }
        __syncthreads();
    }
    if (!HPSI) {
        for (int off = 32; off > 0; off >>= 1) {
            er += __shfl_xor(er, off, 64);
            ei += __shfl_xor(ei, off, 64);
        }
        if ((tid & 63) == 0) {
            sh.red[0][tid >> 6] = er;
            sh.red[1][tid >> 6] = ei;
        }
        __syncthreads();
        if (tid == 0) {
            double a0 = 0.0, a1 = 0.0;
            for (int w = 0; w < kThreads / 64; ++w) {
                a0 += sh.red[0][w];
                a1 += sh.red[1][w];
            }
            double* p = partials + blockIdx.x;
            double* q = partials + pstride + blockIdx.x;
            *p = accumulate ? *p + a0 : a0;
            *q = accumulate ? *q + a1 : a1;
        }
        if (!accumulate)  // slots beyond the grid start at zero for later passes
            for (int b = gridDim.x + blockIdx.x * kThreads + tid; b < pstride;
                 b += gridDim.x * kThreads) {
                partials[b] = 0.0;
                partials[pstride + b] = 0.0;
            }
    }
}

}  // namespace

// Blocks of the tile pass resident on the whole device (the grid: one block
// per resident slot, each streaming tiles with the next tile's loads in
// flight).  Cached per device and kernel variant.
template <typename R, bool HPSI>
int resident_grid()
{
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 1024;
    if (cache[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tile_pass<R, HPSI>, kThreads, 0) !=
                hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            per_cu < 1 || cus < 1)
            return 1024;
        cache[dev] = per_cu * cus;
    }
    return cache[dev];
}

hipError_t launch_tile_pass(const TileExpK& a, const void* psi, void* lam, int dt, bool hpsi,
                            double* partials, int nslots, int accumulate, hipStream_t s)
{
    if (a.ntiles == 0)
        return hipSuccess;
    int g = dt == C64 ? (hpsi ? resident_grid<float, true>() : resident_grid<float, false>())
                      : (hpsi ? resident_grid<double, true>() : resident_grid<double, false>());
    if (!hpsi && g > nslots)
        g = nslots;  // partial slots: block b writes slot b, the first pass zeroes the rest
    if ((uint64_t)g > a.ntiles)
        g = (int)a.ntiles;
    const dim3 grid((unsigned)g);
    if (dt == C64) {
        if (hpsi)
            hipLaunchKernelGGL((k_tile_pass<float, true>), grid, dim3(kThreads), 0, s,
                               static_cast<const float*>(psi), static_cast<float*>(lam), a, partials,
                               nslots, accumulate);
        else
            hipLaunchKernelGGL((k_tile_pass<float, false>), grid, dim3(kThreads), 0, s,
                               static_cast<const float*>(psi), static_cast<float*>(lam), a, partials,
                               nslots, accumulate);
    } else {
        if (hpsi)
            hipLaunchKernelGGL((k_tile_pass<double, true>), grid, dim3(kThreads), 0, s,
                               static_cast<const double*>(psi), static_cast<double*>(lam), a, partials,
                               nslots, accumulate);
        else
            hipLaunchKernelGGL((k_tile_pass<double, false>), grid, dim3(kThreads), 0, s,
                               static_cast<const double*>(psi), static_cast<double*>(lam), a, partials,
                               nslots, accumulate);
    }
    return hipGetLastError();
}

}  // namespace qsv
