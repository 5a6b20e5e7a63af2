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
// A workgroup handles one tile of 2^(k+6) amplitudes: all targets plus the
// six lowest non-target qubits (64 groups).  Because those six bits and every
// target below them form a contiguous run of low bits, a tile is a few
// contiguous chunks of >= 64 amplitudes, loaded with 16-byte nontemporal
// accesses.  The tile is transposed through LDS into [tau'][group] rows
// (padded by one amplitude against bank conflicts).  Work is split by output
// rows: wavefront w computes the real rows of 16-row block(s) w mod RB for
// its share of the 64 group columns, so it keeps only its own A fragments in
// registers (16 per lane for k = 5).  Results go back to LDS and the tile is
// stored in place.  One tile per workgroup, blocks in XCD-contiguous order:
// on MI355X this streams faster than persistent tile loops (measured), and
// the small register footprint keeps several workgroups per CU.  The
// exception is the three-product kernel below for k = 5 (and k = 4 with
// clustered targets): it takes four (two) consecutive tiles per workgroup
// and issues the loads of the next tile as soon as the current one is in
// LDS, so they run under its products.
#include "qsv_internal.h"

namespace qsv {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

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
    using NV = v4f;                     // 16-byte global vector (two amplitudes)
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
    using NV = v2d;                     // one amplitude
    static constexpr int APV = 1;
    __device__ static Acc mfma(double a, double b, Acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // result register r of lane l holds row l / 16 + 4 r, column l % 16
    __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

constexpr int kRow = 65;  // LDS row length in amplitudes (64 groups + 1 pad)

// Complex amplitude as one LDS access (8 bytes for float, 16 for double).
template <typename R>
struct Pair2;
template <>
struct Pair2<float> {
    using T = float2;
};
template <>
struct Pair2<double> {
    using T = double2;
};

// Block index in XCD-contiguous order (a bijection on [0, gridDim.x)).
__device__ __forceinline__ uint64_t xcd_block()
{
    const uint32_t G = gridDim.x, b = blockIdx.x, per = G >> 3;
    return b < (per << 3) ? (uint64_t)(b & 7u) * per + (b >> 3) : (uint64_t)b;
}

// Waves per SIMD the register allocation must allow (1 = no constraint):
// 8 for complex64 k = 4 (fits in 64 VGPRs), 4 for complex128 k = 5 (with the
// B reads two k-steps ahead it fits in 128); measured 3-5% faster each.
// complex64 k = 5 keeps its 72 VGPRs: capping it spills, and 8-wave
// workgroups with half the columns per wave ran slower.
template <typename R, int K>
constexpr int mfma_wpe()
{
    return (sizeof(R) == 4 && K == 4) ? 8 : ((sizeof(R) == 8 && K == 5) ? 4 : 1);
}

template <typename R, int K>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(mfma_wpe<R, K>()))) k_mfma(R* __restrict__ psi0, R* __restrict__ psi1,
                                              const MfmaK<K> a, const R* __restrict__ frag)
{
    using T = MfmaT<R>;
    using NV = typename T::NV;
    using P2 = typename Pair2<R>::T;
    constexpr int D = 1 << K;           // amplitudes per group
    constexpr int TA = D * 64;          // amplitudes per tile
    constexpr int APV = T::APV;
    constexpr int VPT = TA / APV / 256; // vectors per thread
    constexpr int KS = (2 * D) / 4;     // k-steps of 4 real rows
    constexpr int RB = (2 * D) / 16;    // 16-row output blocks (4 for k = 5, 2 for k = 4)
    // Wave w takes row block w % RB and CBW = RB of the 4 16-column blocks,
    // starting at (w / RB) * RB: for k = 5 every wave covers all 64 groups of
    // its row block; for k = 4 waves 0, 1 take groups 0..31, waves 2, 3 the rest.
    constexpr int CBW = RB;
    static_assert(RB == 2 || RB == 4, "tile split");

    __shared__ __align__(16) R lds[D * kRow * 2];

    R* psi = blockIdx.y ? psi1 : psi0;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int rb = wave % RB;
    const int cb0 = (wave / RB) * CBW;

    const uint64_t tile = xcd_block();
    if (tile >= a.ntiles)
        return;
    const uint64_t base = insert_bits(tile, a.ins);

    // Tile loads first (their latency covers the set-up below).
    uint64_t goff[VPT];
    NV in[VPT];
#pragma unroll
    for (int r = 0; r < VPT; ++r) {
        const int loc = (tid + 256 * r) * APV;
        goff[r] = a.choff[loc >> a.L] + (uint64_t)(loc & ((1 << a.L) - 1));
        in[r] = __builtin_nontemporal_load(reinterpret_cast<const NV*>(psi + 2 * (base + goff[r])));
    }
    // A operand: this wave's row block of R(G), KS values per lane,
    // contiguous in the fragment table ([rb][lane][kk]).
    R afr[KS];
#pragma unroll
    for (int kk = 0; kk < KS; ++kk)
        afr[kk] = frag[((size_t)rb * 64 + lane) * KS + kk];
    int pos[VPT][APV];
#pragma unroll
    for (int r = 0; r < VPT; ++r) {
        const int loc = (tid + 256 * r) * APV;
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
    // registers -> LDS [tau'][group]
#pragma unroll
    for (int r = 0; r < VPT; ++r)
#pragma unroll
        for (int h = 0; h < APV; ++h)
            *reinterpret_cast<P2*>(&lds[pos[r][h]]) = P2{in[r][2 * h], in[r][2 * h + 1]};
    __syncthreads();

    // B operand: lane holds real row 4kk + lane/16 of group (cb0 + c) * 16 +
    // lane % 16.  k-steps outermost: the CBW accumulators are independent
    // chains that the matrix core overlaps.
    typename T::Acc acc[CBW];
#pragma unroll
    for (int c = 0; c < CBW; ++c)
        acc[c] = typename T::Acc{0, 0, 0, 0};
    const int bofs = ((lane >> 5) * kRow + cb0 * 16 + (lane & 15)) * 2 + ((lane >> 4) & 1);
    // B reads in groups of KG k-steps, one group ahead of its products
    // (the scheduling barriers keep the reads of group g + 1 issued before
    // the products of group g).
    constexpr int KG = (sizeof(R) == 8 && K == 5) ? 2 : 4;
    R bfr[KS][CBW];
#pragma unroll
    for (int kk = 0; kk < KG; ++kk)
#pragma unroll
        for (int c = 0; c < CBW; ++c)
            bfr[kk][c] = lds[bofs + (2 * kk * kRow + 16 * c) * 2];
#pragma unroll
    for (int g = 0; g < KS / KG; ++g) {
        if (g + 1 < KS / KG) {
#pragma unroll
            for (int kk = (g + 1) * KG; kk < (g + 2) * KG; ++kk)
#pragma unroll
                for (int c = 0; c < CBW; ++c)
                    bfr[kk][c] = lds[bofs + (2 * kk * kRow + 16 * c) * 2];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int kk = g * KG; kk < (g + 1) * KG; ++kk)
#pragma unroll
            for (int c = 0; c < CBW; ++c)
                acc[c] = T::mfma(afr[kk], bfr[kk][c], acc[c]);
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();  // every wave has read its B operands (all rows)
    // D: register r of each lane holds real row 16 rb + T::row(lane, r) of
    // group (cb0 + c) * 16 + lane % 16; real row 2 tau + c' is component c'
    // of amplitude tau.
#pragma unroll
    for (int c = 0; c < CBW; ++c) {
        const int grp = (cb0 + c) * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rr = 16 * rb + T::row(lane, r);
            lds[((rr >> 1) * kRow + grp) * 2 + (rr & 1)] = acc[c][r];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < VPT; ++r) {
        NV o;
#pragma unroll
        for (int h = 0; h < APV; ++h) {
            const P2 w = *reinterpret_cast<const P2*>(&lds[pos[r][h]]);
            o[2 * h] = w.x;
            o[2 * h + 1] = w.y;
        }
        __builtin_nontemporal_store(o, reinterpret_cast<NV*>(psi + 2 * (base + goff[r])));
    }
}

// Gauss's three-product form of the same complex product (3M): with
// G = Gr + i Gi and In = Xr + i Xi,
//     P1 = Gr Xr,  P2 = Gi Xi,  P3 = (Gr + Gi)(Xr + Xi),
//     Out = (P1 - P2) + i (P3 - P1 - P2),
// three real 2^k x 2^k products instead of one 2^(k+1) x 2^(k+1) one: 3/4 of
// the matrix-core work (the k = 5 block is bound by it at ~57% of the f32 /
// f64 matrix peak for 70% of HBM).  The A operands Gr, Gi and Gr + Gi are
// formed on the host in FP64 and rounded once; Xr + Xi is one VALU add per
// B value.  The tile layout in LDS is the same [tau'][group] as above, and
// every B value is one complex LDS read.  Work split: the 2^k / 16 row blocks
// of complex rows take 4 / RB waves each, each wave 4 / WPR of the four
// 16-column group blocks.
// Waves per SIMD the three-product kernel's register allocation must allow:
// complex64 k = 4 fits 8; the others take what they need (complex128 k = 5
// would spill under a 128-register cap).
template <typename R, int K>
constexpr int mfma3_wpe()
{
    return (sizeof(R) == 4 && K == 4) ? 8 : 1;
}

// The products of one tile, between the barrier after the tile is in LDS
// and the barrier before it is read back: B operands from LDS (lane holds
// complex row 4 kk + lane / 16 of group (cb0 + c) * 16 + lane % 16, read in
// groups of KG k-steps one group ahead of the products; scheduling barriers
// keep the order), the three accumulators, and the complex results written
// back over the tile in LDS.
template <typename R, int K>
__device__ __forceinline__ void mfma3_multiply(R* lds, const R (&afr)[3][(1 << K) / 4], int lane, int rb,
                                               int cb0)
{
    using T = MfmaT<R>;
    using P2 = typename Pair2<R>::T;
    constexpr int D = 1 << K;
    constexpr int KS = D / 4;
    constexpr int RB = D / 16;
    constexpr int CBW = 4 / (4 / RB);
    typename T::Acc acc[3][CBW];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int c = 0; c < CBW; ++c)
            acc[p][c] = typename T::Acc{0, 0, 0, 0};
    const int bofs = ((lane >> 4) * kRow + cb0 * 16 + (lane & 15)) * 2;
    constexpr int KG = K == 5 ? 2 : 4;  // k = 5: two k-steps per group keeps the registers in bounds
    P2 bfr[KS][CBW];
#pragma unroll
    for (int kk = 0; kk < KG; ++kk)
#pragma unroll
        for (int c = 0; c < CBW; ++c)
            bfr[kk][c] = *reinterpret_cast<const P2*>(&lds[bofs + (4 * kk * kRow + 16 * c) * 2]);
#pragma unroll
    for (int g = 0; g < KS / KG; ++g) {
        if (g + 1 < KS / KG) {
#pragma unroll
            for (int kk = (g + 1) * KG; kk < (g + 2) * KG; ++kk)
#pragma unroll
                for (int c = 0; c < CBW; ++c)
                    bfr[kk][c] = *reinterpret_cast<const P2*>(&lds[bofs + (4 * kk * kRow + 16 * c) * 2]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int kk = g * KG; kk < (g + 1) * KG; ++kk)
#pragma unroll
            for (int c = 0; c < CBW; ++c) {
                const R xr = bfr[kk][c].x, xi = bfr[kk][c].y;
                acc[0][c] = T::mfma(afr[0][kk], xr, acc[0][c]);
                acc[1][c] = T::mfma(afr[1][kk], xi, acc[1][c]);
                acc[2][c] = T::mfma(afr[2][kk], xr + xi, acc[2][c]);
            }
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();  // every wave has read its B operands
    // register r of each lane holds complex row 16 rb + T::row(lane, r) of
    // group (cb0 + c) * 16 + lane % 16
#pragma unroll
    for (int c = 0; c < CBW; ++c) {
        const int grp = (cb0 + c) * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int tau = 16 * rb + T::row(lane, r);
            const R p1 = acc[0][c][r], p2 = acc[1][c][r], p3 = acc[2][c][r];
            *reinterpret_cast<P2*>(&lds[(tau * kRow + grp) * 2]) = P2{p1 - p2, p3 - p1 - p2};
        }
    }
}

// TPB consecutive tiles per workgroup (TPB divides ntiles; 1, 2 or 4).  With
// more than one, the loads of the next tile are issued as soon as the current
// one is in LDS (the load registers are free again), so they run under its
// products.
template <typename R, int K, int TPB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(mfma3_wpe<R, K>()))) k_mfma3(R* __restrict__ psi0, R* __restrict__ psi1,
                                               const MfmaK<K> a, const R* __restrict__ frag)
{
    using T = MfmaT<R>;
    using NV = typename T::NV;
    using P2 = typename Pair2<R>::T;
    constexpr int D = 1 << K;           // complex rows (amplitudes per group)
    constexpr int TA = D * 64;          // amplitudes per tile
    constexpr int APV = T::APV;
    constexpr int VPT = TA / APV / 256; // vectors per thread
    constexpr int KS = D / 4;           // k-steps of 4 complex rows
    constexpr int RB = D / 16;          // 16-row output blocks (2 for k = 5, 1 for k = 4)
    constexpr int WPR = 4 / RB;         // waves per row block
    constexpr int CBW = 4 / WPR;        // 16-column blocks per wave
    static_assert(RB == 1 || RB == 2, "tile split");
    static_assert(TPB == 1 || TPB == 2 || TPB == 4, "tiles per workgroup");

    __shared__ __align__(16) R lds[D * kRow * 2];

    R* psi = blockIdx.y ? psi1 : psi0;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int rb = wave % RB;
    const int cb0 = (wave / RB) * CBW;

    const uint64_t tile = xcd_block() * TPB;
    if (tile >= a.ntiles)
        return;
    const uint64_t base = insert_bits(tile, a.ins);

    uint64_t goff[VPT];
    NV in[VPT];
#pragma unroll
    for (int r = 0; r < VPT; ++r) {
        const int loc = (tid + 256 * r) * APV;
        goff[r] = a.choff[loc >> a.L] + (uint64_t)(loc & ((1 << a.L) - 1));
        in[r] = __builtin_nontemporal_load(reinterpret_cast<const NV*>(psi + 2 * (base + goff[r])));
    }
    // A operands of this wave's row block: Gr, Gi, Gr + Gi, KS values each
    // per lane, contiguous in the table ([rb][product][lane][kk]).
    R afr[3][KS];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int kk = 0; kk < KS; ++kk)
            afr[p][kk] = frag[(((size_t)rb * 3 + p) * 64 + lane) * KS + kk];
    int pos[VPT][APV];
#pragma unroll
    for (int r = 0; r < VPT; ++r) {
        const int loc = (tid + 256 * r) * APV;
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
    auto to_lds = [&]() {
#pragma unroll
        for (int r = 0; r < VPT; ++r)
#pragma unroll
            for (int h = 0; h < APV; ++h)
                *reinterpret_cast<P2*>(&lds[pos[r][h]]) = P2{in[r][2 * h], in[r][2 * h + 1]};
    };
    auto store = [&](uint64_t b) {
#pragma unroll
        for (int r = 0; r < VPT; ++r) {
            NV o;
#pragma unroll
            for (int h = 0; h < APV; ++h) {
                const P2 w = *reinterpret_cast<const P2*>(&lds[pos[r][h]]);
                o[2 * h] = w.x;
                o[2 * h + 1] = w.y;
            }
            __builtin_nontemporal_store(o, reinterpret_cast<NV*>(psi + 2 * (b + goff[r])));
        }
    };
    if constexpr (TPB > 1) {
#pragma unroll
        for (int it = 0; it < TPB; ++it) {
            to_lds();
            __syncthreads();
            if (it + 1 < TPB) {
                const uint64_t b1 = insert_bits(tile + it + 1, a.ins);
#pragma unroll
                for (int r = 0; r < VPT; ++r)
                    in[r] = __builtin_nontemporal_load(reinterpret_cast<const NV*>(psi + 2 * (b1 + goff[r])));
            }
            mfma3_multiply<R, K>(lds, afr, lane, rb, cb0);
            __syncthreads();
            store(insert_bits(tile + it, a.ins));
            __syncthreads();  // every wave has read the tile back before the next one is written
        }
    } else {
        to_lds();
        __syncthreads();
        mfma3_multiply<R, K>(lds, afr, lane, rb, cb0);
        __syncthreads();
        store(base);
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
    if (L.ntiles > (1ull << 31))
        return hipErrorInvalidValue;
    // consecutive tiles per workgroup as the host chose them by the target
    // layout (GateLaunch::mfma_tpb; the real-embedding kernel takes one)
    const int tpb = L.mfma_tpb;
    if (L.mfma3 && (tpb == 2 || tpb == 4) && L.ntiles >= (uint64_t)tpb) {
        const dim3 g((unsigned)(L.ntiles / tpb), p1 ? 2 : 1);
        if (tpb == 2)
            hipLaunchKernelGGL((k_mfma3<R, K, 2>), g, dim3(256), 0, s, static_cast<R*>(p0),
                               static_cast<R*>(p1 ? p1 : p0), a, static_cast<const R*>(L.gdev));
        else
            hipLaunchKernelGGL((k_mfma3<R, K, 4>), g, dim3(256), 0, s, static_cast<R*>(p0),
                               static_cast<R*>(p1 ? p1 : p0), a, static_cast<const R*>(L.gdev));
        return hipGetLastError();
    }
    dim3 grid((unsigned)L.ntiles, p1 ? 2 : 1);
    if (L.mfma3)
        hipLaunchKernelGGL((k_mfma3<R, K, 1>), grid, dim3(256), 0, s, static_cast<R*>(p0),
                           static_cast<R*>(p1 ? p1 : p0), a, static_cast<const R*>(L.gdev));
    else
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

// A operands of the three-product kernel: [rb][product][lane][kk] with
// lane holding row 16 rb + lane % 16, column 4 kk + lane / 16 of Gr, Gi and
// Gr + Gi (the sum formed in FP64, then rounded once).
void mfma3_fragments(const double* Gc, int K, int dt, std::vector<unsigned char>& out)
{
    const int D = 1 << K, KS = D / 4, RB = D / 16;
    const size_t count = (size_t)RB * 3 * 64 * KS;
    out.assign(count * (dt == C64 ? 4 : 8), 0);
    for (int rb = 0; rb < RB; ++rb)
        for (int p = 0; p < 3; ++p)
            for (int lane = 0; lane < 64; ++lane)
                for (int kk = 0; kk < KS; ++kk) {
                    const int row = 16 * rb + (lane & 15), col = 4 * kk + (lane >> 4);
                    const double gre = Gc[((size_t)row * D + col) * 2];
                    const double gim = Gc[((size_t)row * D + col) * 2 + 1];
                    const double v = p == 0 ? gre : (p == 1 ? gim : gre + gim);
                    const size_t idx = (((size_t)rb * 3 + p) * 64 + lane) * KS + kk;
                    if (dt == C64)
                        reinterpret_cast<float*>(out.data())[idx] = (float)v;
                    else
                        reinterpret_cast<double*>(out.data())[idx] = v;
                }
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
                const size_t idx = ((size_t)rb * 64 + lane) * KS + kk;
                if (dt == C64)
                    reinterpret_cast<float*>(out.data())[idx] = (float)v;
                else
                    reinterpret_cast<double*>(out.data())[idx] = v;
            }
}

}  // namespace qsv
