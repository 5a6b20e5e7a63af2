// Qubit permutation passes (L_QPERM): a run of SWAP gates permutes the bits
// of every amplitude index; one pass applies a bit permutation that is an
// involution, in place, as pure moves of raw bits (signed zeros and NaN
// payloads survive).  The planner (qperm_plan.cpp) composes the swaps and
// splits other permutations into two involutions.
//
// A tile is 2^(RL + hb) amplitudes: rows of 2^RL consecutive amplitudes
// (512 bytes) at the 2^hb offsets of the tile's upper bits, which include the
// images of the row bits, so the image of a tile is one tile and both its
// reads and its writes are whole rows.  A workgroup takes a tile and its
// image (or a tile that is its own image), loads them into LDS, and writes
// each into the other's place, reading the LDS in permuted order.  The
// workgroup index maps to the tile index through a bit permutation chosen by
// the planner, so that consecutive workgroups step through adjacent rows of
// both their tiles and the images (DRAM page locality on both sides).  LDS rows
// are XOR-swizzled by row index so that reading a column (the transpose that
// bit reversal makes of the row bits) spreads over the banks.
#include "qsv_internal.h"

namespace qsv {

namespace {

typedef unsigned int nv2u __attribute__((ext_vector_type(2)));  // one complex64 amplitude
typedef unsigned int nv4u __attribute__((ext_vector_type(4)));  // one complex128 amplitude

struct QPermK {
    uint64_t ntiles;
    InsertSpec ins;  // zeros inserted at the tile bits
    int n;
    int hb;
    int hpos[6];
    int cmap[12];
    unsigned int qw[16];  // q[b] (b < 64) in byte b % 4 of qw[b / 4]
    unsigned int ww[16];  // wsrc[p] likewise: bit p of the tile index = bit wsrc[p] of the workgroup index
    int nouter;           // n - RL - hb
};

// The loops below run to fixed bounds without branches (the launcher pads
// the descriptor so that unused entries contribute nothing), so that its
// arrays are read once into scalar registers instead of one dependent load
// per iteration (a workgroup moves one tile, so such a chain would not be
// hidden).  Index arithmetic that is the same for a whole wave
// is spread over its lanes and read back with readlane: the scalar unit is
// shared by every wave of a compute unit, and per-wave scalar loops over the
// index bits were what limited this kernel.

// Zeros inserted at the (at most 12) tile bits; unused masks are all ones.
__device__ __forceinline__ uint64_t insert_bits(uint64_t g, const InsertSpec& s)
{
#pragma unroll
    for (int j = 0; j < 12; ++j) {
        const uint64_t lo = s.low[j];
        g = ((g & ~lo) << 1) | (g & lo);
    }
    return g | s.setmask;
}

// Block index in XCD-contiguous order (a bijection on [0, gridDim.x)).
__device__ __forceinline__ uint64_t xcd_block()
{
    const uint32_t G = gridDim.x, b = blockIdx.x, per = G >> 3;
    return b < (per << 3) ? (uint64_t)(b & 7u) * per + (b >> 3) : (uint64_t)b;
}

// Global offset of tile row t < 2^hb (its bits deposited at the upper tile
// bits; bits of t at and above hb are zero).
__device__ __forceinline__ uint64_t row_offset(const QPermK& a, int t)
{
    uint64_t o = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k)
        o |= (uint64_t)((t >> k) & 1) << a.hpos[k];
    return o;
}

// Source tile-local index of the output tile-local index l (linear in the
// bits of l: bit k of the result is bit cmap[k] of l; unused entries point at
// bit 31, which is zero in every tile-local index).
__device__ __forceinline__ int source_local(const QPermK& a, int l)
{
    int s = 0;
#pragma unroll
    for (int k = 0; k < 12; ++k)
        s |= ((l >> a.cmap[k]) & 1) << k;
    return s;
}

template <typename V, int RL, int NT>
__global__ void __launch_bounds__(NT) k_qperm(V* __restrict__ psi0, V* __restrict__ psi1, const QPermK a)
{
    constexpr int ROW = 1 << RL;
    constexpr int TMAX = ROW * ROW;    // hb <= RL
    constexpr int EPT = TMAX / NT;     // elements per thread of a full tile
    constexpr int NW = NT / 64;        // waves per workgroup
    static_assert(EPT >= 1 && ROW <= 64, "tile shape");
    __shared__ V lds[2][TMAX];

    V* p = blockIdx.y ? psi1 : psi0;
    const uint64_t widx = xcd_block();
    if (widx >= a.ntiles)
        return;
    const int lane = threadIdx.x & 63;
    // the workgroup's tile: lane p supplies bit p = bit wsrc[p] of widx
    unsigned int wword = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if ((lane >> 2) == j)
            wword = a.ww[j];
    const int wb = (wword >> ((lane & 3) * 8)) & 63;
    const uint64_t tile = __ballot(lane < a.nouter && ((widx >> wb) & 1ull));
    const uint64_t ba = insert_bits(tile, a.ins);
    // the image tile: lane b supplies bit b = bit q[b] of ba
    unsigned int qword = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if ((lane >> 2) == j)
            qword = a.qw[j];
    const int qb = (qword >> ((lane & 3) * 8)) & 63;
    const uint64_t bb = __ballot(lane < a.n && ((ba >> qb) & 1ull));
    if (bb < ba)
        return;  // the workgroup of the image's tile moves both
    const bool pair = bb != ba;
    // A wave instruction covers RPW whole rows: the rows of element r are
    // t = (wave + NW r) RPW + tl, so the row part of every address is uniform
    // across the wave except tl (complex128 only).  Both maps below are
    // linear in the bits, and the bits of (wave + NW r) RPW, tl and the
    // column are disjoint (so | and + agree on them).
    constexpr int RPW = 64 / ROW;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = lane & (ROW - 1);
    const int tl = lane >> RL;
    const int rows = 1 << a.hb;
    const uint64_t lane_off = row_offset(a, tl) | (uint64_t)c;
    const int lane_src = source_local(a, (tl << RL) | c);
    // lane r (< EPT) holds the row part of element r: its global offset and
    // its source tile-local bits
    const int ur = (wave + NW * (lane & (EPT - 1))) * RPW;
    const uint64_t ro_lane = row_offset(a, ur);
    const int sr_lane = source_local(a, ur << RL);
    auto row_off = [&](int r) {
        return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(ro_lane >> 32), r) << 32) |
               (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)ro_lane, r);
    };

    V x0[EPT], x1[EPT];
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
        const int u = (wave + NW * r) * RPW;
        if (u + tl < rows) {
            const uint64_t ro = row_off(r);
            x0[r] = __builtin_nontemporal_load(p + ba + ro + lane_off);
            if (pair)
                x1[r] = __builtin_nontemporal_load(p + bb + ro + lane_off);
        }
    }
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
        const int t = (wave + NW * r) * RPW + tl;
        if (t < rows) {
            lds[0][t * ROW + (c ^ t)] = x0[r];
            if (pair)
                lds[1][t * ROW + (c ^ t)] = x1[r];
        }
    }
    __syncthreads();
    // output tile ba takes its amplitudes from the image tile bb and the other
    // way round; a tile that is its own image takes them from itself
    const V* from_b = pair ? lds[1] : lds[0];
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
        const int u = (wave + NW * r) * RPW;
        if (u + tl < rows) {
            const int s = __builtin_amdgcn_readlane(sr_lane, r) | lane_src;
            const int st = s >> RL, sc = s & (ROW - 1);
            const int si = st * ROW + (sc ^ st);
            const uint64_t ro = row_off(r);
            __builtin_nontemporal_store(from_b[si], p + ba + ro + lane_off);
            if (pair)
                __builtin_nontemporal_store(lds[0][si], p + bb + ro + lane_off);
        }
    }
}

template <typename V, int RL, int NT>
hipError_t qperm_go(const GateLaunch& L, void* p0, void* p1, hipStream_t s)
{
    if (L.qp_rl != RL || L.qp_hb < 0 || L.qp_hb > RL || L.n < 2 * RL || L.n > 64 ||
        L.ngroups != (1ull << (L.n - RL - L.qp_hb)) || L.ngroups > 0x7fffffffull)
        return hipErrorInvalidValue;
    if (L.ins.nins != RL + L.qp_hb || L.ins.setmask != 0)
        return hipErrorInvalidValue;
    QPermK a{};
    a.ntiles = L.ngroups;
    a.ins = L.ins;
    for (int j = L.ins.nins; j < 12; ++j)
        a.ins.low[j] = ~0ull;
    a.n = L.n;
    a.hb = L.qp_hb;
    for (int k = 0; k < L.qp_hb; ++k)
        a.hpos[k] = L.qp_hpos[k];
    for (int k = 0; k < 12; ++k)
        a.cmap[k] = k < RL + L.qp_hb ? L.qp_cmap[k] : 31;
    for (int b = 0; b < L.n; ++b)
        a.qw[b / 4] |= (unsigned int)(L.qp_q[b] & 63) << (8 * (b % 4));
    a.nouter = L.n - RL - L.qp_hb;
    for (int b = 0; b < a.nouter; ++b)
        a.ww[b / 4] |= (unsigned int)(L.qp_wsrc[b] & 63) << (8 * (b % 4));
    const dim3 grid((unsigned)L.ngroups, p1 ? 2 : 1);
    hipLaunchKernelGGL((k_qperm<V, RL, NT>), grid, dim3(NT), 0, s, static_cast<V*>(p0),
                       static_cast<V*>(p1 ? p1 : p0), a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_qperm(const GateLaunch& L, void* psi, void* psi2, hipStream_t s)
{
    return L.dt == C64 ? qperm_go<nv2u, kQpRowBitsC64, 512>(L, psi, psi2, s)
                       : qperm_go<nv4u, kQpRowBitsC128, 256>(L, psi, psi2, s);
}

}  // namespace qsv
