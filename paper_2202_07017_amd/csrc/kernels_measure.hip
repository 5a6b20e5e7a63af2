// Simulated measurement (Sec. 3: measurements are simulated by sampling
// kernels): marginal Born probabilities of a qubit subset, and whole-register
// outcomes drawn by inverse-transform sampling from caller-supplied uniforms.
// Probabilities |psi_i|^2 are formed and summed in FP64 (amplitudes widened
// first); every sum has a fixed order, so results are deterministic.
//
// Sampling keeps no probability vector.  One streaming pass writes a sum
// tree into the workspace: level 0 holds the sums of chunks of 2^cb
// consecutive amplitudes (cb = min(n, 8)), level L + 1 the sums of 64
// consecutive level-L entries, up to a top level of at most 64 entries.
// A shot descends the tree one wave-wide 64-way choice per level and
// resolves the outcome inside one chunk (one 2 or 4 KiB read).
#include "qsv_internal.h"

namespace qsv {

namespace {

constexpr int kWave = 64;
constexpr int kPrepThreads = 1024;       // 16 waves per group block
constexpr int kChunkLog = 8;             // log2(amplitudes per sampling leaf chunk)
constexpr int kMargItemsLog = 16;        // log2(wave items targeted by the marginal pass)
constexpr int kMargPartLog = 20;         // log2(doubles of per-slice partial sums)

template <typename R>
struct A2;
template <>
struct A2<float> {
    using T = float2;
};
template <>
struct A2<double> {
    using T = double2;
};

template <typename R>
__device__ __forceinline__ double prob(const R* psi, uint64_t i)
{
    const typename A2<R>::T a = reinterpret_cast<const typename A2<R>::T*>(psi)[i];
    const double re = (double)a.x, im = (double)a.y;
    return re * re + im * im;
}

// Sum of |psi|^2 over one 16-byte vector: two complex64 or one complex128 amplitude.
__device__ __forceinline__ double prob16(const float* psi, uint64_t v)
{
    const float4 f = reinterpret_cast<const float4*>(psi)[v];
    const double a = (double)f.x, b = (double)f.y, c = (double)f.z, d = (double)f.w;
    return (a * a + b * b) + (c * c + d * d);
}

__device__ __forceinline__ double prob16(const double* psi, uint64_t v)
{
    const double2 f = reinterpret_cast<const double2*>(psi)[v];
    return f.x * f.x + f.y * f.y;
}

// SplitMix64 output function (Steele, Lea & Flood 2014) at state x.  Seeded
// sampling draws u_s = top 53 bits / 2^53 of the output at key + s * golden
// gamma, key = the output at state `seed` (the generator restarted at its own
// first output, so nearby seeds give unrelated streams).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Butterfly sum over the 64 lanes; every lane ends with the same value.
__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = kWave / 2; off > 0; off >>= 1)
        v += __shfl_xor(v, off, kWave);
    return v;
}

// Inclusive prefix over the 64 lanes (lane order).
__device__ __forceinline__ double wave_incl_scan(double v, int lane)
{
    for (int off = 1; off < kWave; off <<= 1) {
        const double y = __shfl_up(v, off, kWave);
        if (lane >= off)
            v += y;
    }
    return v;
}

// Descent step over up to 64 children with masses m (0 for lanes past the
// end): picks the first child whose running mass exceeds t among children of
// nonzero mass, else the last child of nonzero mass (t beyond the node's
// mass: rounding, u >= 1 or NaN), else child 0 (a node of zero mass).  t is
// then made relative to the chosen child.  Only children of nonzero mass are
// taken, so an outcome of zero probability is never reached, whatever the
// rounding of the sums.
__device__ __forceinline__ int descend(double m, double& t, int lane)
{
    const double incl = wave_incl_scan(m, lane);
    const uint64_t c = __ballot(incl > t && m > 0.0);
    int L;
    if (c) {
        L = __builtin_ctzll(c);
    } else {
        const uint64_t nz = __ballot(m > 0.0);
        L = nz ? 63 - __builtin_clzll(nz) : 0;
    }
    t -= __shfl(incl - m, L, kWave);
    return L;
}

// One block per group of 2^gb chunks: wave w sums chunks w, w + 16, ...
// (coalesced 16-byte loads) into level 0; wave 0 adds the group's chunk sums
// into level 1 when the tree has a level above the chunks (lev1 != NULL).
template <typename R>
__global__ void __launch_bounds__(kPrepThreads) k_sample_prep(const R* __restrict__ psi, int cb, int gb,
                                                             double* __restrict__ lev0,
                                                             double* __restrict__ lev1)
{
    __shared__ double csum[kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int G = 1 << gb;
    const uint64_t nvec = sizeof(R) == 4 ? (1ull << cb) / 2 : (1ull << cb);
    const uint64_t grp = blockIdx.x;
    // a wave's chunks (at most four: G <= 64 chunks over 16 waves) are read
    // side by side, so all of their loads are in flight together; each
    // chunk's sum keeps its index order
    constexpr int NW = kPrepThreads / kWave;
    static_assert(NW * 4 >= kWave, "four chunks per wave cover a group of 64");
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint64_t v = lane; v < nvec; v += kWave)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = wave + j * NW;
            if (c < G)
                s[j] += prob16(psi, ((grp << gb) + (uint64_t)c) * nvec + v);
        }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int c = wave + j * NW;
        const double t = wave_sum(s[j]);
        if (c < G && lane == 0)
            csum[c] = t;
    }
    __syncthreads();
    if (wave == 0) {
        const double x = lane < G ? csum[lane] : 0.0;
        if (lane < G)
            lev0[(grp << gb) + lane] = x;
        const double g = wave_sum(x);
        if (lev1 && lane == 0)
            lev1[grp] = g;
    }
}

// out[i] = sum of in[64 i .. 64 i + 63] (entries past nin count as 0); one
// wave per output entry.
__global__ void __launch_bounds__(256) k_tree_up(const double* __restrict__ in, uint64_t nin,
                                                 double* __restrict__ out, uint64_t nout)
{
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t i = (uint64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
    if (i >= nout)
        return;
    const uint64_t j = i * kWave + (uint64_t)lane;
    const double s = wave_sum(j < nin ? in[j] : 0.0);
    if (lane == 0)
        out[i] = s;
}

constexpr int kMaxLevels = 8;

// Sum tree over the state: level 0 holds the chunk sums, level L + 1 the sums
// of 64 consecutive level-L entries, up to a top level of <= 64 entries.
struct SampleTree {
    int cb;                        // log2(chunk length)
    int nlev;
    uint64_t count[kMaxLevels];
    uint64_t off[kMaxLevels];      // offsets (in doubles) into the workspace
};

// One wave per shot (grid-stride over shots): descend the tree, then resolve
// the outcome inside the chosen chunk, where lane l owns amplitudes
// [l E, l E + E), E = max(2^cb / 64, 1).
template <typename R>
__global__ void __launch_bounds__(256) k_sample(const R* __restrict__ psi, SampleTree tr,
                                                const double* __restrict__ work,
                                                const double* __restrict__ u, uint64_t seed, int seeded,
                                                int64_t nshots, int64_t* __restrict__ out)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wid = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (256 / kWave) + threadIdx.x / kWave));
    const int64_t nw = (int64_t)gridDim.x * (256 / kWave);
    const uint64_t csize = 1ull << tr.cb;
    const int E = tr.cb >= 6 ? (int)(csize >> 6) : 1;
    const int cnt = (uint64_t)lane * E < csize ? E : 0;
    const int top = tr.nlev - 1;
    const double* topv = work + tr.off[top];
    const double T = wave_sum((uint64_t)lane < tr.count[top] ? topv[lane] : 0.0);
    const uint64_t key = splitmix64(seed);
    for (int64_t s = wid; s < nshots; s += nw) {
        double us;
        if (seeded)
            us = (double)(splitmix64(key + (uint64_t)s * 0x9E3779B97F4A7C15ull) >> 11) * 0x1.0p-53;
        else
            us = u[s];
        double t = us * T;
        if (t < 0.0)
            t = 0.0;
        uint64_t node = 0;
        for (int L = top; L >= 0; --L) {
            const uint64_t idx = node * kWave + (uint64_t)lane;
            const double m = idx < tr.count[L] ? work[tr.off[L] + idx] : 0.0;
            node = node * kWave + (uint64_t)descend(m, t, lane);
        }
        const uint64_t a0 = (node << tr.cb) + (uint64_t)lane * E;
        double p[16];
        double ls = 0.0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            p[j] = j < cnt ? prob(psi, a0 + j) : 0.0;
            ls += p[j];
        }
        const int L = descend(ls, t, lane);
        if (lane == L) {
            int jsel = -1, jlast = 0;
            double run = 0.0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                run += p[j];
                if (p[j] > 0.0) {
                    jlast = j;
                    if (jsel < 0 && run > t)
                        jsel = j;
                }
            }
            out[s] = (int64_t)(a0 + (uint64_t)(jsel >= 0 ? jsel : jlast));
        }
    }
}

// Deposit the low bits of v into the set bit positions of mask, in order.
__device__ __forceinline__ uint64_t deposit(uint64_t v, uint64_t mask)
{
    uint64_t r = 0;
    while (mask) {
        const uint64_t low = mask & (~mask + 1);
        if (v & 1)
            r |= low;
        v >>= 1;
        mask ^= low;
    }
    return r;
}

// Next index in the enumeration of the positions of mask: adds the deposited
// step d, carrying through the positions outside mask.
__device__ __forceinline__ uint64_t masked_add(uint64_t x, uint64_t d, uint64_t mask)
{
    return ((x | ~mask) + d) & mask;
}

struct MeasSpec {
    int m;
    int q[kMaxIns];      // measured qubits, q[0] = most significant outcome bit
    uint64_t umask;      // unmeasured positions of the state index
};

// The outcome b of state index i: bit (m - 1 - j) of b is bit q[j] of i.
__device__ __forceinline__ uint64_t outcome_index(uint64_t i, const MeasSpec& M)
{
    uint64_t b = 0;
    for (int j = 0; j < M.m; ++j)
        b |= ((i >> M.q[j]) & 1ull) << (M.m - 1 - j);
    return b;
}

// Lanes read 64 consecutive amplitudes (address bits 0..5 = lane bits), so
// every load is coalesced whatever qubits are measured.  A wave item fixes
// the measured address bits above bit 5 (h) and a slice s of the unmeasured
// address bits above bit 5, which the wave walks in order (four independent
// partial sums, combined in a fixed order).  The lanes then add over their
// unmeasured lane bits (xor butterfly on those bits only), and each lane whose
// unmeasured lane bits are 0 holds the sum of one outcome b: written to
// out[b] (one slice) or part[s * 2^m + b].
struct MargLanes {
    uint64_t mhi;        // measured positions >= 6
    uint64_t uhi;        // unmeasured positions >= 6 (below n)
    int lane_umask;      // lane bits whose position is unmeasured or >= n
    int mhi_bits;        // popcount(mhi)
    int iters_log;       // log2(unmeasured steps per item)
    uint64_t nstate;     // 2^n
};

template <typename R>
__global__ void __launch_bounds__(256) k_marginal_lanes(const R* __restrict__ psi, MeasSpec M, MargLanes G,
                                                        uint64_t nitems, double* __restrict__ dst)
{
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t d = deposit(1, G.uhi);
    const uint64_t iters = 1ull << G.iters_log;
    const uint64_t stride = (uint64_t)gridDim.x * (256 / kWave);
    const bool live = (uint64_t)lane < G.nstate;
    for (uint64_t w = (uint64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave; w < nitems; w += stride) {
        const uint64_t h = w & ((1ull << G.mhi_bits) - 1);
        const uint64_t s = w >> G.mhi_bits;
        const uint64_t base = deposit(h, G.mhi) | (uint64_t)lane;
        uint64_t x = deposit(s << G.iters_log, G.uhi);
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        uint64_t j = 0;
        if (live) {
            // four steps per round; the next round's four loads are issued
            // before this round's squares are added (software pipeline), the
            // additions keep the same order
            using T = typename A2<R>::T;
            const T* p = reinterpret_cast<const T*>(psi);
            auto sq = [](const T& a) {
                const double re = (double)a.x, im = (double)a.y;
                return re * re + im * im;
            };
            if (iters >= 4) {
                T c[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    c[u] = p[base | x];
                    x = masked_add(x, d, G.uhi);
                }
                for (j = 4; j + 4 <= iters; j += 4) {
                    T nx[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        nx[u] = p[base | x];
                        x = masked_add(x, d, G.uhi);
                    }
                    a0 += sq(c[0]);
                    a1 += sq(c[1]);
                    a2 += sq(c[2]);
                    a3 += sq(c[3]);
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        c[u] = nx[u];
                }
                a0 += sq(c[0]);
                a1 += sq(c[1]);
                a2 += sq(c[2]);
                a3 += sq(c[3]);
            }
            for (; j < iters; ++j) {
                a0 += sq(p[base | x]);
                x = masked_add(x, d, G.uhi);
            }
        }
        double acc = (a0 + a1) + (a2 + a3);
        for (int k = 0; k < 6; ++k)
            if ((G.lane_umask >> k) & 1)
                acc += __shfl_xor(acc, 1 << k, kWave);
        if ((lane & G.lane_umask) == 0) {
            const uint64_t b = outcome_index(base, M);
            dst[(s << M.m) + b] = acc;
        }
    }
}

// out[b] = sum over s < nslices of part[s * nb + b]: one wave per outcome,
// lane l adding slices l, l + 64, ... in order, then a butterfly.
__global__ void __launch_bounds__(256) k_marginal_finalize(const double* __restrict__ part, uint64_t nb,
                                                           uint64_t nslices, double* __restrict__ out)
{
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t b = (uint64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
    if (b >= nb)
        return;
    double acc = 0.0;
    for (uint64_t s = lane; s < nslices; s += kWave)
        acc += part[s * nb + b];
    acc = wave_sum(acc);
    if (lane == 0)
        out[b] = acc;
}

// counts[b] += 1 for every shot whose outcome bits spell b.  Small outcome
// spaces (2^m <= 4096) count per block in LDS first, then add each nonzero
// bin once; larger ones add straight into device memory.  Integer sums, so
// the result does not depend on the order of the atomics.
constexpr int kFreqLds = 4096;

template <bool LDSH>
__global__ void __launch_bounds__(256) k_frequencies(const int64_t* __restrict__ samples, int64_t nshots,
                                                     MeasSpec M, unsigned long long* __restrict__ counts)
{
    __shared__ unsigned int h[LDSH ? kFreqLds : 1];
    const uint64_t nb = 1ull << M.m;
    if (LDSH) {
        for (uint64_t k = threadIdx.x; k < nb; k += 256)
            h[k] = 0u;
        __syncthreads();
    }
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < nshots; s += stride) {
        const uint64_t b = outcome_index((uint64_t)samples[s], M);
        if (LDSH)
            atomicAdd(&h[b], 1u);
        else
            atomicAdd(&counts[b], 1ull);
    }
    if (LDSH) {
        __syncthreads();
        for (uint64_t k = threadIdx.x; k < nb; k += 256)
            if (h[k])
                atomicAdd(&counts[k], (unsigned long long)h[k]);
    }
}

__global__ void __launch_bounds__(256) k_zero_counts(unsigned long long* p, uint64_t count)
{
    const uint64_t step = (uint64_t)gridDim.x * 256;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += step)
        p[i] = 0ull;
}

// Projective collapse: amplitudes whose measured bits (mask) differ from want
// become +0, the others are scaled by 1 / sqrt(p), p read from device memory
// (p <= 0: the zero vector).  One read+write sweep of 16-byte units with the
// nontemporal hint (every line is touched once).
typedef float nv4f __attribute__((ext_vector_type(4)));
typedef double nv2d __attribute__((ext_vector_type(2)));

template <typename R>
__global__ void __launch_bounds__(256) k_collapse(R* __restrict__ psi, uint64_t nunits, uint64_t mask,
                                                  uint64_t want, const double* __restrict__ prob)
{
    const double p = *prob;
    const double sd = p > 0.0 ? 1.0 / sqrt(p) : 0.0;
    const R sc = (R)sd;
    const uint64_t step = (uint64_t)gridDim.x * 256;
    for (uint64_t u = (uint64_t)blockIdx.x * 256 + threadIdx.x; u < nunits; u += step) {
        if constexpr (sizeof(R) == 4) {
            nv4f* q = reinterpret_cast<nv4f*>(psi);
            const nv4f x = __builtin_nontemporal_load(&q[u]);
            const bool k0 = ((u << 1) & mask) == want, k1 = (((u << 1) | 1u) & mask) == want;
            nv4f y;
            y[0] = k0 ? x[0] * sc : 0.0f;
            y[1] = k0 ? x[1] * sc : 0.0f;
            y[2] = k1 ? x[2] * sc : 0.0f;
            y[3] = k1 ? x[3] * sc : 0.0f;
            __builtin_nontemporal_store(y, &q[u]);
        } else {
            nv2d* q = reinterpret_cast<nv2d*>(psi);
            const nv2d x = __builtin_nontemporal_load(&q[u]);
            const bool k0 = (u & mask) == want;
            nv2d y;
            y[0] = k0 ? x[0] * sc : 0.0;
            y[1] = k0 ? x[1] * sc : 0.0;
            __builtin_nontemporal_store(y, &q[u]);
        }
    }
}

SampleTree sample_tree(int n)
{
    SampleTree tr{};
    tr.cb = n < kChunkLog ? n : kChunkLog;
    uint64_t c = 1ull << (n - tr.cb);
    uint64_t off = 0;
    for (;;) {
        tr.count[tr.nlev] = c;
        tr.off[tr.nlev] = off;
        off += c;
        ++tr.nlev;
        if (c <= (uint64_t)kWave)
            break;
        c = (c + kWave - 1) / kWave;
    }
    return tr;
}

}  // namespace

size_t sample_workspace_doubles(int n)
{
    const SampleTree tr = sample_tree(n);
    return (size_t)(tr.off[tr.nlev - 1] + tr.count[tr.nlev - 1]);
}

size_t marginal_workspace_doubles()
{
    return (size_t)1 << kMargPartLog;
}


hipError_t launch_sample(const void* psi, int n, int dt, const double* u, uint64_t seed, int seeded,
                         int64_t nshots, int64_t* out, double* work, hipStream_t s)
{
    const SampleTree tr = sample_tree(n);
    const int gb = n - tr.cb < 6 ? n - tr.cb : 6;
    const unsigned ngroups = (unsigned)(1ull << (n - tr.cb - gb));
    double* lev1 = tr.nlev > 1 ? work + tr.off[1] : nullptr;
    if (dt == C64)
        hipLaunchKernelGGL(k_sample_prep<float>, dim3(ngroups), dim3(kPrepThreads), 0, s,
                           static_cast<const float*>(psi), tr.cb, gb, work, lev1);
    else
        hipLaunchKernelGGL(k_sample_prep<double>, dim3(ngroups), dim3(kPrepThreads), 0, s,
                           static_cast<const double*>(psi), tr.cb, gb, work, lev1);
    hipError_t e = hipGetLastError();
    for (int L = 2; L < tr.nlev && e == hipSuccess; ++L) {
        const unsigned grid = (unsigned)((tr.count[L] + 3) / 4);
        hipLaunchKernelGGL(k_tree_up, dim3(grid), dim3(256), 0, s, (const double*)(work + tr.off[L - 1]),
                           tr.count[L - 1], work + tr.off[L], tr.count[L]);
        e = hipGetLastError();
    }
    if (e != hipSuccess || nshots == 0)
        return e;
    const int64_t waves = nshots < (int64_t)(1 << 20) ? nshots : (int64_t)(1 << 20);
    const unsigned grid = (unsigned)((waves + 3) / 4);
    if (dt == C64)
        hipLaunchKernelGGL(k_sample<float>, dim3(grid), dim3(256), 0, s, static_cast<const float*>(psi), tr,
                           (const double*)work, u, seed, seeded, nshots, out);
    else
        hipLaunchKernelGGL(k_sample<double>, dim3(grid), dim3(256), 0, s, static_cast<const double*>(psi), tr,
                           (const double*)work, u, seed, seeded, nshots, out);
    return hipGetLastError();
}

hipError_t launch_marginal(const void* psi, int n, int dt, const int* q, int m, double* out, double* work,
                           hipStream_t s)
{
    MeasSpec M{};
    M.m = m;
    uint64_t mm = 0;
    for (int j = 0; j < m; ++j) {
        M.q[j] = q[j];
        mm |= 1ull << q[j];
    }
    const uint64_t all = (1ull << n) - 1;
    M.umask = all & ~mm;
    MargLanes G{};
    G.mhi = mm & ~63ull;
    G.uhi = M.umask & ~63ull;
    G.lane_umask = (int)(~mm & 63ull);
    G.mhi_bits = __builtin_popcountll(G.mhi);
    G.nstate = 1ull << n;
    const int ubits = __builtin_popcountll(G.uhi);
    // slices: as many as keep the item count near 2^kMargItemsLog and the
    // partial sums within the workspace
    int ls = 0;
    while (ls < ubits && G.mhi_bits + ls + 1 <= kMargItemsLog && m + ls + 1 <= kMargPartLog)
        ++ls;
    G.iters_log = ubits - ls;
    const uint64_t nitems = 1ull << (G.mhi_bits + ls);
    double* dst = ls ? work : out;
    const uint64_t blocks = (nitems + 3) / 4;
    const unsigned grid = (unsigned)(blocks < (1ull << 20) ? blocks : (1ull << 20));
    if (dt == C64)
        hipLaunchKernelGGL(k_marginal_lanes<float>, dim3(grid), dim3(256), 0, s,
                           static_cast<const float*>(psi), M, G, nitems, dst);
    else
        hipLaunchKernelGGL(k_marginal_lanes<double>, dim3(grid), dim3(256), 0, s,
                           static_cast<const double*>(psi), M, G, nitems, dst);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || ls == 0)
        return e;
    const uint64_t nb = 1ull << m;
    hipLaunchKernelGGL(k_marginal_finalize, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0, s,
                       (const double*)work, nb, 1ull << ls, out);
    return hipGetLastError();
}

hipError_t launch_frequencies(const int64_t* samples, int64_t nshots, int n, const int* q, int m,
                              int64_t* counts, hipStream_t s)
{
    MeasSpec M{};
    M.m = m;
    uint64_t mm = 0;
    for (int j = 0; j < m; ++j) {
        M.q[j] = q[j];
        mm |= 1ull << q[j];
    }
    M.umask = ((1ull << n) - 1) & ~mm;
    const uint64_t nb = 1ull << m;
    unsigned long long* c = reinterpret_cast<unsigned long long*>(counts);
    const uint64_t zb = (nb + 255) / 256;
    hipLaunchKernelGGL(k_zero_counts, dim3((unsigned)(zb < 65536 ? zb : 65536)), dim3(256), 0, s, c, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nshots == 0)
        return e;
    const int64_t blocks = (nshots + 255) / 256;
    const unsigned grid = (unsigned)(blocks < 4096 ? blocks : 4096);
    if (nb <= (uint64_t)kFreqLds)
        hipLaunchKernelGGL(k_frequencies<true>, dim3(grid), dim3(256), 0, s, samples, nshots, M, c);
    else
        hipLaunchKernelGGL(k_frequencies<false>, dim3(grid), dim3(256), 0, s, samples, nshots, M, c);
    return hipGetLastError();
}

hipError_t launch_collapse(void* psi, int n, int dt, const int* q, int m, uint64_t outcome,
                           const double* prob, hipStream_t s)
{
    uint64_t mask = 0, want = 0;
    for (int j = 0; j < m; ++j) {
        mask |= 1ull << q[j];
        want |= ((outcome >> (m - 1 - j)) & 1ull) << q[j];
    }
    const uint64_t nunits = dt == C64 ? (1ull << n) / 2 : (1ull << n);
    const uint64_t blocks = (nunits + 1023) / 1024;
    const unsigned grid = (unsigned)(blocks < (1ull << 20) ? (blocks ? blocks : 1) : (1ull << 20));
    if (dt == C64)
        hipLaunchKernelGGL(k_collapse<float>, dim3(grid), dim3(256), 0, s, static_cast<float*>(psi), nunits,
                           mask, want, prob);
    else
        hipLaunchKernelGGL(k_collapse<double>, dim3(grid), dim3(256), 0, s, static_cast<double*>(psi), nunits,
                           mask, want, prob);
    return hipGetLastError();
}

}  // namespace qsv
