// Dense k = 4, 5 qubit blocks on the gfx950 matrix cores.
//
// eq. (1) of the paper (Sec. 2) for a block of k targets is, for all groups q
// at once, the product Out = G In of the 2^k x 2^k complex matrix with a
// 2^k x (#groups) matrix of amplitudes.  With interleaved (re, im) storage the
// same product is a real one, Out_r = R(G) In_r, where R(G) is the
// 2^(k+1) x 2^(k+1) real matrix with 2x2 blocks [[Re g, -Im g], [Im g, Re g]].
// That real product runs on v_mfma_f32_16x16x4f32 (complex64 states) or
// v_mfma_f64_16x16x4f64 (complex128 states); R(G) stays in registers as the
// A operand for the whole kernel.  Both shapes take A[i][k] from lane
// i + 16 k and B[k][j] from lane j + 16 k; their results differ: the f32 form
// returns rows 4 (lane / 16) + r, the f64 form rows lane / 16 + 4 r (column
// lane % 16, register r), as measured on gfx950.
//
// A workgroup handles tiles of 2^(k+6) amplitudes: all targets plus the six
// lowest non-target qubits (64 groups).  Because those six bits and every
// target below them form a contiguous run of low bits, a tile is a few
// contiguous chunks of >= 64 amplitudes, loaded with 16-byte accesses.  The
// tile is transposed through LDS into [tau'][group] rows (padded by one
// amplitude against bank conflicts), each of the 4 wavefronts multiplies 16
// groups, writes its results back in place and the tile is stored.  The grid
// is persistent over tiles and the next tile's loads are issued before the
// current tile's matrix products.
#include "qsv_internal.h"

namespace qsv {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <int K>
struct MfmaK {
    uint64_t ntiles;
    InsertSpec ins;
    int L;
    uint64_t choff[32];
    int tloc[5];
    int floc[6];
};

__device__ __forceinline__ uint64_t insert_bits(uint64_t g, const InsertSpec& s)
{
    for (int j = 0; j < s.nins; ++j) {
        const uint64_t lo = s.low[j];
        g = ((g & ~lo) << 1) | (g & lo);
    }
    return g | s.setmask;
}

template <typename R>
struct MfmaT;
template <>
struct MfmaT<float> {
    using Acc = v4f;
    using Vec = float4;                 // 16-byte global vector
    static constexpr int APV = 2;       // amplitudes per vector
    __device__ static Acc mfma(float a, float b, Acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // result register r of lane l holds row 4 (l / 16) + r, column l % 16
    __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct MfmaT<double> {
    using Acc = v4d;
    using Vec = double2;
    static constexpr int APV = 1;
    __device__ static Acc mfma(double a, double b, Acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // result register r of lane l holds row l / 16 + 4 r, column l % 16
    __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

constexpr int kRow = 65;  // LDS row length in amplitudes (64 groups + 1 pad)

template <typename R, int K>
__global__ void __launch_bounds__(256) k_mfma(R* __restrict__ psi0, R* __restrict__ psi1,
                                              const MfmaK<K> a, const R* __restrict__ frag)
{
    using T = MfmaT<R>;
    using Vec = typename T::Vec;
    constexpr int D = 1 << K;           // amplitudes per group
    constexpr int TA = D * 64;          // amplitudes per tile
    constexpr int APV = T::APV;
    constexpr int VPT = TA / APV / 256; // vectors per thread
    constexpr int KS = (2 * D) / 4;     // k-steps of 4 real rows
    constexpr int RB = (2 * D) / 16;    // 16-row output blocks

    __shared__ R lds[D * kRow * 2];

    R* psi = blockIdx.y ? psi1 : psi0;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int grp = wave * 16 + (lane & 15);

    // A operand: R(G) fragments, lane-major, kept in registers.
    R afr[RB][KS];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int kk = 0; kk < KS; ++kk)
            afr[rb][kk] = frag[(rb * KS + kk) * 64 + lane];

    // Per-thread tile geometry (same for every tile).
    uint64_t goff[VPT];
    int pos[VPT][APV];
#pragma unroll
    for (int r = 0; r < VPT; ++r) {
        const int loc = (tid + 256 * r) * APV;
        goff[r] = a.choff[loc >> a.L] + (uint64_t)(loc & ((1 << a.L) - 1));
#pragma unroll
        for (int h = 0; h < APV; ++h) {
            const int l = loc + h;
            int tau = 0, j = 0;
#pragma unroll
            for (int b = 0; b < K; ++b)
                tau |= ((l >> a.tloc[b]) & 1) << b;
#pragma unroll
            for (int b = 0; b < 6; ++b)
                j |= ((l >> a.floc[b]) & 1) << b;
            pos[r][h] = (tau * kRow + j) * 2;
        }
    }

    uint64_t tile = blockIdx.x;
    if (tile >= a.ntiles)
        return;
    Vec in[VPT];
    {
        const uint64_t base = insert_bits(tile, a.ins);
#pragma unroll
        for (int r = 0; r < VPT; ++r)
            in[r] = *reinterpret_cast<const Vec*>(psi + 2 * (base + goff[r]));
    }
    for (; tile < a.ntiles; tile += gridDim.x) {
        const uint64_t base = insert_bits(tile, a.ins);
        // registers -> LDS [tau'][group]
#pragma unroll
        for (int r = 0; r < VPT; ++r) {
            const R* v = reinterpret_cast<const R*>(&in[r]);
#pragma unroll
            for (int h = 0; h < APV; ++h) {
                lds[pos[r][h]] = v[2 * h];
                lds[pos[r][h] + 1] = v[2 * h + 1];
            }
        }
        __syncthreads();
        const uint64_t next = tile + gridDim.x;
        if (next < a.ntiles) {
            const uint64_t nb = insert_bits(next, a.ins);
#pragma unroll
            for (int r = 0; r < VPT; ++r)
                in[r] = *reinterpret_cast<const Vec*>(psi + 2 * (nb + goff[r]));
        }
        // B operand: lane holds real row 4kk + lane/16 of group `grp`.
        R bfr[KS];
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            const int tp = 2 * kk + (lane >> 5);
            bfr[kk] = lds[(tp * kRow + grp) * 2 + ((lane >> 4) & 1)];
        }
        typename T::Acc acc[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
            acc[rb] = typename T::Acc{0, 0, 0, 0};
        // k-steps outermost: the RB accumulators are independent chains that
        // the matrix core can overlap.
#pragma unroll
        for (int kk = 0; kk < KS; ++kk)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                acc[rb] = T::mfma(afr[rb][kk], bfr[kk], acc[rb]);
        // D: register r of each lane holds real row 16 rb + T::row(lane, r) of
        // group `grp`; real row 2 tau + c is component c of amplitude tau.
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rr = 16 * rb + T::row(lane, r);
                lds[((rr >> 1) * kRow + grp) * 2 + (rr & 1)] = acc[rb][r];
            }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < VPT; ++r) {
            Vec o;
            R* v = reinterpret_cast<R*>(&o);
#pragma unroll
            for (int h = 0; h < APV; ++h) {
                v[2 * h] = lds[pos[r][h]];
                v[2 * h + 1] = lds[pos[r][h] + 1];
            }
            *reinterpret_cast<Vec*>(psi + 2 * (base + goff[r])) = o;
        }
        __syncthreads();
    }
}

template <typename R, int K>
hipError_t mfma_go(const GateLaunch& L, void* p0, void* p1, hipStream_t s)
{
    MfmaK<K> a{};
    a.ntiles = L.ntiles;
    a.ins = L.ins;
    a.L = L.L;
    for (int j = 0; j < 32; ++j)
        a.choff[j] = L.choff[j];
    for (int j = 0; j < 5; ++j)
        a.tloc[j] = L.tloc[j];
    for (int j = 0; j < 6; ++j)
        a.floc[j] = L.floc[j];
    uint64_t blocks = L.ntiles < 2048 ? L.ntiles : 2048;
    dim3 grid((unsigned)blocks, p1 ? 2 : 1);
    hipLaunchKernelGGL((k_mfma<R, K>), grid, dim3(256), 0, s, static_cast<R*>(p0),
                       static_cast<R*>(p1 ? p1 : p0), a, static_cast<const R*>(L.gdev));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_mfma(const GateLaunch& L, void* psi, void* psi2, hipStream_t s)
{
    if (L.ntiles == 0)
        return hipSuccess;
    if (L.dt == C64)
        return L.K == 4 ? mfma_go<float, 4>(L, psi, psi2, s) : mfma_go<float, 5>(L, psi, psi2, s);
    return L.K == 4 ? mfma_go<double, 4>(L, psi, psi2, s) : mfma_go<double, 5>(L, psi, psi2, s);
}

void mfma_fragments(const double* Gc, int K, int dt, std::vector<unsigned char>& out)
{
    const int D = 1 << K, KS = 2 * D / 4, RB = 2 * D / 16;
    const size_t count = (size_t)RB * KS * 64;
    out.assign(count * (dt == C64 ? 4 : 8), 0);
    for (int rb = 0; rb < RB; ++rb)
        for (int kk = 0; kk < KS; ++kk)
            for (int lane = 0; lane < 64; ++lane) {
                const int row = 16 * rb + (lane & 15), col = 4 * kk + (lane >> 4);
                const int tau = row >> 1, ra = row & 1, tp = col >> 1, cb = col & 1;
                const double gre = Gc[((size_t)tau * D + tp) * 2];
                const double gim = Gc[((size_t)tau * D + tp) * 2 + 1];
                const double v = (ra == cb) ? gre : (ra == 0 ? -gim : gim);
                const size_t idx = ((size_t)rb * KS + kk) * 64 + lane;
                if (dt == C64)
                    reinterpret_cast<float*>(out.data())[idx] = (float)v;
                else
                    reinterpret_cast<double*>(out.data())[idx] = v;
            }
}

}  // namespace qsv
