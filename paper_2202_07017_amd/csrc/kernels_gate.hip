// Gate-application kernels for gfx950: eq. (1) of the paper (Sec. 2) as an
// in-place, HBM-streaming sweep over groups of 2^k amplitudes.
//
// A group is one bitstring q of the non-target qubits.  Its base index is
// made by inserting zero bits at every target/control position of the group
// counter and OR-ing the control mask in (the "index generation by fast
// binary operations" of Sec. 2); its 2^k amplitudes sit at base + off[tau'].
// Consecutive threads take consecutive groups, so every load and store of a
// wavefront is a contiguous run whenever the lowest touched qubit is >= 1.
// For complex64 states two adjacent amplitudes are moved as one 16-byte
// float4 (modes W2 / INTRA), which keeps 16-byte accesses for every target
// position including qubit 0.
//
// Launch shape (measured on MI355X at n = 30): one group per thread, blocks
// visited in XCD-contiguous order (the hardware deals blocks round-robin to
// the 8 XCDs; remapping block b to (b mod 8) * G/8 + b / 8 hands each XCD one
// contiguous eighth of the state), nontemporal loads and stores once the
// contiguous runs are >= 128 bytes, and a lane-exchange kernel for
// uncontrolled single-qubit gates whose partner sits within 64 units.
#include <cstdlib>

#include "qsv_internal.h"

namespace qsv {
namespace {

template <typename R>
struct Amp;
template <>
struct Amp<float> {
    using T = float2;
    using Pair = float4;
};
template <>
struct Amp<double> {
    using T = double2;
    using Pair = double4;  // unused
};

__device__ __forceinline__ uint64_t insert_bits(uint64_t g, const InsertSpec& s)
{
    for (int j = 0; j < s.nins; ++j) {
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

template <typename R>
struct Cx {
    R re, im;
};

typedef float nv4f __attribute__((ext_vector_type(4)));
typedef double nv2d __attribute__((ext_vector_type(2)));

// 16-byte loads and stores, optionally with the nontemporal hint (streaming
// sweeps touch every line once).
template <bool NT>
__device__ __forceinline__ float4 ldv(const float4* p)
{
    if constexpr (NT) {
        const nv4f v = __builtin_nontemporal_load(reinterpret_cast<const nv4f*>(p));
        return make_float4(v[0], v[1], v[2], v[3]);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ double2 ldv(const double2* p)
{
    if constexpr (NT) {
        const nv2d v = __builtin_nontemporal_load(reinterpret_cast<const nv2d*>(p));
        return make_double2(v[0], v[1]);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ float2 ldv(const float2* p)
{
    return *p;
}
template <bool NT>
__device__ __forceinline__ void stv(float4* p, float4 v)
{
    if constexpr (NT) {
        nv4f w = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(w, reinterpret_cast<nv4f*>(p));
    } else {
        *p = v;
    }
}
template <bool NT>
__device__ __forceinline__ void stv(double2* p, double2 v)
{
    if constexpr (NT) {
        nv2d w = {v.x, v.y};
        __builtin_nontemporal_store(w, reinterpret_cast<nv2d*>(p));
    } else {
        *p = v;
    }
}
template <bool NT>
__device__ __forceinline__ void stv(float2* p, float2 v)
{
    *p = v;
}

// Raw 8- and 16-byte units (permutations), optionally nontemporal.
typedef unsigned int nv2u __attribute__((ext_vector_type(2)));
typedef unsigned int nv4u __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ __forceinline__ uint4 ldu(const uint4* p)
{
    if constexpr (NT) {
        const nv4u v = __builtin_nontemporal_load(reinterpret_cast<const nv4u*>(p));
        return make_uint4(v[0], v[1], v[2], v[3]);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ uint2 ldu(const uint2* p)
{
    if constexpr (NT) {
        const nv2u v = __builtin_nontemporal_load(reinterpret_cast<const nv2u*>(p));
        return make_uint2(v[0], v[1]);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ void stu(uint4* p, uint4 v)
{
    if constexpr (NT) {
        nv4u w = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(w, reinterpret_cast<nv4u*>(p));
    } else {
        *p = v;
    }
}
template <bool NT>
__device__ __forceinline__ void stu(uint2* p, uint2 v)
{
    if constexpr (NT) {
        nv2u w = {v.x, v.y};
        __builtin_nontemporal_store(w, reinterpret_cast<nv2u*>(p));
    } else {
        *p = v;
    }
}

template <typename R>
__device__ __forceinline__ void cmac(Cx<R>& acc, R gr, R gi, R xr, R xi)
{
    acc.re = fma(gr, xr, fma(-gi, xi, acc.re));
    acc.im = fma(gr, xi, fma(gi, xr, acc.im));
}

// ------------------------------------------------------------------ dense

template <typename R, int K>
struct DenseK {
    uint64_t ngroups;
    InsertSpec ins;
    uint64_t off[1 << K];
    R g[(K <= 3) ? (2 << (2 * K)) : 2];  // canonical, row-major, (re, im)
    const R* gdev;                       // K >= 4
    const double* params;
    int pidx;
    int rot;
    int dag;
};

// Rotation exp(-i theta P / 2) (theta negated for the dagger), row-major (re, im).
template <typename R>
__device__ __forceinline__ void rotation_matrix(int rot, double theta, R* m)
{
    const double c = cos(0.5 * theta), s = sin(0.5 * theta);
    double v[8] = {c, 0, 0, 0, 0, 0, c, 0};
    if (rot == ROT_X) {
        v[3] = -s;
        v[5] = -s;
    } else if (rot == ROT_Y) {
        v[2] = -s;
        v[4] = s;
    } else {  // ROT_Z
        v[1] = -s;
        v[7] = s;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
        m[j] = (R)v[j];
}

template <typename R, int K, int MODE, bool ROT, int UNR, bool NT>
__global__ void __launch_bounds__(kBlock) k_dense(R* __restrict__ psi0, R* __restrict__ psi1,
                                                  const DenseK<R, K> a)
{
    constexpr int D = 1 << K;
    constexpr int NU = (MODE == INTRA) ? D / 2 : D;  // loads per group
    using A = typename Amp<R>::T;
    R* psi = blockIdx.y ? psi1 : psi0;

    R rm[8];
    if constexpr (ROT) {
        const double th = a.params[a.pidx];
        rotation_matrix<R>(a.rot, a.dag ? -th : th, rm);
    }
    auto gre = [&](int r, int c) -> R {
        if constexpr (ROT)
            return rm[(r * 2 + c) * 2];
        else if constexpr (K <= 3)
            return a.g[(r * D + c) * 2];
        else
            return a.gdev[(r * D + c) * 2];
    };
    auto gim = [&](int r, int c) -> R {
        if constexpr (ROT)
            return rm[(r * 2 + c) * 2 + 1];
        else if constexpr (K <= 3)
            return a.g[(r * D + c) * 2 + 1];
        else
            return a.gdev[(r * D + c) * 2 + 1];
    };

    const uint64_t step = (uint64_t)gridDim.x * kBlock * UNR;
    for (uint64_t g0 = xcd_block() * kBlock * UNR + threadIdx.x; g0 < a.ngroups; g0 += step) {
        uint64_t base[UNR];
        bool ok[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const uint64_t g = g0 + (uint64_t)u * kBlock;
            ok[u] = g < a.ngroups;
            base[u] = insert_bits(ok[u] ? g : 0, a.ins);
        }
        if constexpr (MODE == W1) {
            A* p = reinterpret_cast<A*>(psi);
            A x[UNR][NU];
#pragma unroll
            for (int u = 0; u < UNR; ++u)
#pragma unroll
                for (int v = 0; v < NU; ++v)
                    if (ok[u])
                        x[u][v] = ldv<NT>(&p[base[u] + a.off[v]]);
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                if (!ok[u])
                    continue;
#pragma unroll
                for (int r = 0; r < D; ++r) {
                    Cx<R> acc{0, 0};
#pragma unroll
                    for (int c = 0; c < D; ++c)
                        cmac(acc, gre(r, c), gim(r, c), x[u][c].x, x[u][c].y);
                    A o;
                    o.x = acc.re;
                    o.y = acc.im;
                    stv<NT>(&p[base[u] + a.off[r]], o);
                }
            }
        } else {
            // complex64 only: float4 units of two adjacent amplitudes
            float4* p = reinterpret_cast<float4*>(psi);
            float4 x[UNR][NU];
#pragma unroll
            for (int u = 0; u < UNR; ++u)
#pragma unroll
                for (int v = 0; v < NU; ++v)
                    if (ok[u])
                        x[u][v] = ldv<NT>(&p[base[u] + a.off[v]]);
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                if (!ok[u])
                    continue;
                if constexpr (MODE == W2) {
#pragma unroll
                    for (int r = 0; r < D; ++r) {
                        Cx<R> a0{0, 0}, a1{0, 0};
#pragma unroll
                        for (int c = 0; c < D; ++c) {
                            const R gr = gre(r, c), gi = gim(r, c);
                            cmac(a0, gr, gi, x[u][c].x, x[u][c].y);
                            cmac(a1, gr, gi, x[u][c].z, x[u][c].w);
                        }
                        stv<NT>(&p[base[u] + a.off[r]], make_float4(a0.re, a0.im, a1.re, a1.im));
                    }
                } else {  // INTRA: x[u][v] holds tau' = 2v (xy) and 2v+1 (zw)
#pragma unroll
                    for (int rv = 0; rv < NU; ++rv) {
                        Cx<R> o[2];
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int r = 2 * rv + h;
                            o[h] = Cx<R>{0, 0};
#pragma unroll
                            for (int cv = 0; cv < NU; ++cv) {
                                cmac(o[h], gre(r, 2 * cv), gim(r, 2 * cv), x[u][cv].x, x[u][cv].y);
                                cmac(o[h], gre(r, 2 * cv + 1), gim(r, 2 * cv + 1), x[u][cv].z,
                                     x[u][cv].w);
                            }
                        }
                        if constexpr (NU == 1)  // keeps -O3 from dropping the store's nontemporal hint
                            asm volatile("" ::: "memory");
                        stv<NT>(&p[base[u] + a.off[rv]], make_float4(o[0].re, o[0].im, o[1].re, o[1].im));
                    }
                }
            }
        }
    }
}

// Uncontrolled single-qubit gate whose target is unit bit tb < 6 (complex64:
// qubit tb + 1, the two amplitudes of a float4 share the target bit;
// complex128: qubit tb).  One 16-byte unit per thread: the partner unit
// (target bit flipped) sits in lane xor 2^tb of the same wavefront, so every
// load and store of a wavefront is one contiguous 1 KB run and the pair is
// exchanged across lanes.  nunits is a multiple of kBlock, so every lane of
// a block runs the same iterations.
template <typename R, bool ROT>
__global__ void __launch_bounds__(kBlock) k_dense_lane(R* __restrict__ psi0, R* __restrict__ psi1,
                                                       const DenseK<R, 1> a, uint64_t nunits, int tb)
{
    R* psi = blockIdx.y ? psi1 : psi0;
    R m[8];
    if constexpr (ROT) {
        const double th = a.params[a.pidx];
        rotation_matrix<R>(a.rot, a.dag ? -th : th, m);
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j)
            m[j] = a.g[j];
    }
    const int mask = 1 << tb;
    const uint64_t step = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = xcd_block() * kBlock + threadIdx.x; i < nunits; i += step) {
        const bool hi = ((i >> tb) & 1u) != 0;
        // row `hi` of the gate: out = g[hi][0] * (bit-0 unit) + g[hi][1] * (bit-1 unit)
        const R ar = hi ? m[4] : m[0], ai = hi ? m[5] : m[1];
        const R br = hi ? m[6] : m[2], bi = hi ? m[7] : m[3];
        if constexpr (sizeof(R) == 4) {
            float4* p = reinterpret_cast<float4*>(psi);
            const float4 x = p[i];
            float4 y;
            y.x = __shfl_xor(x.x, mask, 64);
            y.y = __shfl_xor(x.y, mask, 64);
            y.z = __shfl_xor(x.z, mask, 64);
            y.w = __shfl_xor(x.w, mask, 64);
            const float4 u0 = hi ? y : x, u1 = hi ? x : y;
            float4 o;
            o.x = ar * u0.x - ai * u0.y + br * u1.x - bi * u1.y;
            o.y = ar * u0.y + ai * u0.x + br * u1.y + bi * u1.x;
            o.z = ar * u0.z - ai * u0.w + br * u1.z - bi * u1.w;
            o.w = ar * u0.w + ai * u0.z + br * u1.w + bi * u1.z;
            p[i] = o;
        } else {
            double2* p = reinterpret_cast<double2*>(psi);
            const double2 x = p[i];
            double2 y;
            y.x = __shfl_xor(x.x, mask, 64);
            y.y = __shfl_xor(x.y, mask, 64);
            const double2 u0 = hi ? y : x, u1 = hi ? x : y;
            double2 o;
            o.x = ar * u0.x - ai * u0.y + br * u1.x - bi * u1.y;
            o.y = ar * u0.y + ai * u0.x + br * u1.y + bi * u1.x;
            p[i] = o;
        }
    }
}

// --------------------------------------------------------------- diagonal

template <typename R>
struct DiagK {
    uint64_t ngroups;
    InsertSpec ins;
    int nt;
    int tpos[5];
    R d[64];  // d[tau] (re, im)
    const double* params;
    int pidx;
    int dag;
};

template <typename R, int MODE, bool ROT, int UNR, bool NT>
__global__ void __launch_bounds__(kBlock) k_diag(R* __restrict__ psi0, R* __restrict__ psi1,
                                                 const DiagK<R> a)
{
    using A = typename Amp<R>::T;
    R* psi = blockIdx.y ? psi1 : psi0;
    __shared__ R dl[64];
    if constexpr (ROT) {
        if (threadIdx.x == 0) {
            const double th = a.dag ? -a.params[a.pidx] : a.params[a.pidx];
            const double c = cos(0.5 * th), s = sin(0.5 * th);
            dl[0] = (R)c;
            dl[1] = (R)(-s);
            dl[2] = (R)c;
            dl[3] = (R)s;
        }
    } else {
        if (threadIdx.x < (2u << a.nt))
            dl[threadIdx.x] = a.d[threadIdx.x];
    }
    __syncthreads();
    auto tau_of = [&](uint64_t i) -> int {
        int t = 0;
        for (int j = 0; j < a.nt; ++j)
            t |= (int)((i >> a.tpos[j]) & 1u) << j;
        return t;
    };
    const uint64_t step = (uint64_t)gridDim.x * kBlock * UNR;
    for (uint64_t g0 = xcd_block() * kBlock * UNR + threadIdx.x; g0 < a.ngroups; g0 += step) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const uint64_t g = g0 + (uint64_t)u * kBlock;
            if (g >= a.ngroups)
                continue;
            const uint64_t idx = insert_bits(g, a.ins);
            if constexpr (MODE == W1) {
                A* p = reinterpret_cast<A*>(psi);
                A x = ldv<NT>(&p[idx]);
                const int t = tau_of(idx);
                const R dr = dl[2 * t], di = dl[2 * t + 1];
                A o;
                o.x = dr * x.x - di * x.y;
                o.y = dr * x.y + di * x.x;
                stv<NT>(&p[idx], o);
            } else {
                float4* p = reinterpret_cast<float4*>(psi);
                float4 x = ldv<NT>(&p[idx]);
                const int t0 = tau_of(idx << 1), t1 = tau_of((idx << 1) | 1u);
                const float d0r = dl[2 * t0], d0i = dl[2 * t0 + 1];
                const float d1r = dl[2 * t1], d1i = dl[2 * t1 + 1];
                stv<NT>(&p[idx], make_float4(d0r * x.x - d0i * x.y, d0r * x.y + d0i * x.x,
                                             d1r * x.z - d1i * x.w, d1r * x.w + d1i * x.z));
            }
        }
    }
}

// ------------------------------------------------------------ permutation

struct PermK {
    uint64_t ngroups;
    InsertSpec ins;
    int nmoved;
    uint64_t dst[32];
    uint64_t src[32];
};

// Pure moves of raw bits (no arithmetic, so signed zeros and NaN payloads
// survive).  UT is the raw unit type (uint2 = one c64 amplitude, uint4 = one
// c128 amplitude or two adjacent c64 amplitudes).
template <typename UT, int NM, int UNR, bool NT>
__global__ void __launch_bounds__(kBlock) k_perm(UT* __restrict__ psi0, UT* __restrict__ psi1,
                                                 const PermK a)
{
    UT* p = blockIdx.y ? psi1 : psi0;
    const uint64_t step = (uint64_t)gridDim.x * kBlock * UNR;
    for (uint64_t g0 = xcd_block() * kBlock * UNR + threadIdx.x; g0 < a.ngroups; g0 += step) {
        UT x[UNR][NM];
        uint64_t base[UNR];
        bool ok[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const uint64_t g = g0 + (uint64_t)u * kBlock;
            ok[u] = g < a.ngroups;
            base[u] = insert_bits(ok[u] ? g : 0, a.ins);
#pragma unroll
            for (int j = 0; j < NM; ++j)
                if (ok[u] && j < a.nmoved)
                    x[u][j] = ldu<NT>(&p[base[u] + a.src[j]]);
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
            for (int j = 0; j < NM; ++j)
                if (ok[u] && j < a.nmoved)
                    stu<NT>(&p[base[u] + a.dst[j]], x[u][j]);
    }
}

// ------------------------------------------------------------------- init

template <typename R>
__global__ void __launch_bounds__(kBlock) k_init_basis(R* __restrict__ psi, uint64_t nvec,
                                                       uint64_t index)
{
    // 16-byte vectors: c64 holds amplitudes 2v, 2v+1; c128 holds amplitude v.
    constexpr int per = sizeof(R) == 4 ? 2 : 1;
    const uint64_t step = (uint64_t)gridDim.x * kBlock;
    for (uint64_t v = (uint64_t)blockIdx.x * kBlock + threadIdx.x; v < nvec; v += step) {
        R w[4] = {0, 0, 0, 0};
        if (index / per == v)
            w[(index % per) * 2] = (R)1;
        if constexpr (sizeof(R) == 4)
            reinterpret_cast<float4*>(psi)[v] = make_float4(w[0], w[1], w[2], w[3]);
        else
            reinterpret_cast<double2*>(psi)[v] = make_double2(w[0], w[1]);
    }
}

// SplitMix64 output function (Steele, Lea & Flood 2014) at state x.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Draw `ctr` of a seed's counter-based stream, shifted to [-1/2, 1/2): the
// key is the generator's first output from state `seed` (so nearby seeds get
// unrelated keys), and the draw is the output after ctr + 1 steps from the
// key, i.e. the output function at key + ctr * golden gamma.
__device__ __forceinline__ double unit_draw(uint64_t key, uint64_t ctr)
{
    return (double)(splitmix64(key + ctr * 0x9E3779B97F4A7C15ull) >> 11) * 0x1.0p-53 - 0.5;
}

// partial[b] = sum over this block's amplitudes of |raw|^2 (fixed order).
__global__ void __launch_bounds__(kBlock) k_rand_norm(uint64_t N, uint64_t seed, double* partial)
{
    const uint64_t key = splitmix64(seed);
    double s = 0.0;
    const uint64_t step = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += step) {
        const double re = unit_draw(key, 2 * i), im = unit_draw(key, 2 * i + 1);
        s += re * re + im * im;
    }
    __shared__ double red[kBlock];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        partial[blockIdx.x] = red[0];
}

// scale = 1/sqrt(sum partial) (fixed order), written to *scale.
__global__ void __launch_bounds__(kBlock) k_rand_scale(const double* partial, int nb, double* scale)
{
    __shared__ double red[kBlock];
    double s = 0.0;
    for (int j = threadIdx.x; j < nb; j += kBlock)
        s += partial[j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *scale = 1.0 / sqrt(red[0]);
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_rand_fill(R* __restrict__ psi, uint64_t N, uint64_t seed,
                                                      const double* scale)
{
    const double s = *scale;
    const uint64_t key = splitmix64(seed);
    const uint64_t step = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += step) {
        psi[2 * i] = (R)(unit_draw(key, 2 * i) * s);
        psi[2 * i + 1] = (R)(unit_draw(key, 2 * i + 1) * s);
    }
}

// ------------------------------------------------------------- launching

// Blocks for `items` work items: one item per thread (sweeps are fastest
// without grid-stride loops), up to 2^23 - 1 blocks (a grid of < 2^31 work
// items, so a 32-qubit complex64 sweep still takes one item per thread);
// larger jobs loop.
inline unsigned grid_for(uint64_t items, int per_thread)
{
    uint64_t b = (items + (uint64_t)kBlock * per_thread - 1) / ((uint64_t)kBlock * per_thread);
    if (b < 1)
        b = 1;
    if (b > (1u << 23) - 1)
        b = (1u << 23) - 1;
    return (unsigned)b;
}

template <typename R, int K>
DenseK<R, K> dense_args(const GateLaunch& L)
{
    DenseK<R, K> a{};
    a.ngroups = L.ngroups;
    a.ins = L.ins;
    for (int j = 0; j < (1 << K); ++j)
        a.off[j] = L.off[j];
    if constexpr (K <= 3) {
        if (L.rot == ROT_NONE)
            for (int j = 0; j < (2 << (2 * K)); ++j)
                a.g[j] = (R)L.g[j];
    }
    a.gdev = static_cast<const R*>(L.gdev);
    a.params = L.params;
    a.pidx = L.pidx;
    a.rot = L.rot;
    a.dag = L.dag;
    return a;
}

// Nontemporal hint: on once the contiguous runs of a launch (2^p units, p the
// lowest inserted unit bit) are >= 128 bytes; below that it loses on MI355X.
// QSV_SWEEP_NT (0/1) overrides the choice.
bool use_nt(const InsertSpec& ins, int unit_bytes)
{
    if (const char* e = getenv("QSV_SWEEP_NT"))
        return e[0] == '1';
    const int p = ins.nins ? __builtin_ctzll(ins.low[0] + 1) : 63;
    return p >= 16 || ((uint64_t)unit_bytes << p) >= 128;
}

template <typename R, int K, int MODE, bool ROT, bool NT>
hipError_t dense_launch(const GateLaunch& L, void* p0, void* p1, hipStream_t s)
{
    dim3 grid(grid_for(L.ngroups, 1), p1 ? 2 : 1);
    hipLaunchKernelGGL((k_dense<R, K, MODE, ROT, 1, NT>), grid, dim3(kBlock), 0, s,
                       static_cast<R*>(p0), static_cast<R*>(p1 ? p1 : p0), dense_args<R, K>(L));
    return hipGetLastError();
}

template <typename R, int K, int MODE, bool ROT>
hipError_t dense_go(const GateLaunch& L, void* p0, void* p1, hipStream_t s)
{
    const int unit = (MODE == W1) ? (int)(2 * sizeof(R)) : 16;
    return use_nt(L.ins, unit) ? dense_launch<R, K, MODE, ROT, true>(L, p0, p1, s)
                               : dense_launch<R, K, MODE, ROT, false>(L, p0, p1, s);
}

// Uncontrolled single-qubit gate on unit bit < 6 with at least one block of
// units: the lane-exchange kernel.  Returns false when it does not apply.
template <typename R>
bool lane_launch(const GateLaunch& L, void* p0, void* p1, hipStream_t s, hipError_t& err)
{
    if (L.K != 1 || L.ins.nins != 1 || L.ins.setmask != 0)
        return false;
    if (!(sizeof(R) == 4 ? L.mode == W2 : L.mode == W1))
        return false;
    const int tb = L.lowq - (L.mode == W2 ? 1 : 0);  // target as a unit bit
    const uint64_t nunits = L.ngroups * 2;
    if (tb < 0 || tb >= 6 || nunits < (uint64_t)kBlock || nunits % kBlock)
        return false;
    if (const char* e = getenv("QSV_NO_LANE_SWEEP"))
        if (e[0] == '1')
            return false;
    dim3 grid(grid_for(nunits, 1), p1 ? 2 : 1);
    R* q0 = static_cast<R*>(p0);
    R* q1 = static_cast<R*>(p1 ? p1 : p0);
    if (L.rot != ROT_NONE)
        hipLaunchKernelGGL((k_dense_lane<R, true>), grid, dim3(kBlock), 0, s, q0, q1, dense_args<R, 1>(L),
                           nunits, tb);
    else
        hipLaunchKernelGGL((k_dense_lane<R, false>), grid, dim3(kBlock), 0, s, q0, q1, dense_args<R, 1>(L),
                           nunits, tb);
    err = hipGetLastError();
    return true;
}

template <typename R, int K>
hipError_t dense_mode(const GateLaunch& L, void* p0, void* p1, hipStream_t s)
{
    if constexpr (K == 1) {
        hipError_t e = hipSuccess;
        if (lane_launch<R>(L, p0, p1, s, e))
            return e;
        if (L.rot != ROT_NONE) {
            if constexpr (sizeof(R) == 4) {
                if (L.mode == W2)
                    return dense_go<R, 1, W2, true>(L, p0, p1, s);
                if (L.mode == INTRA)
                    return dense_go<R, 1, INTRA, true>(L, p0, p1, s);
            }
            return dense_go<R, 1, W1, true>(L, p0, p1, s);
        }
    }
    if constexpr (sizeof(R) == 4) {
        if (L.mode == W2)
            return dense_go<R, K, W2, false>(L, p0, p1, s);
        if (L.mode == INTRA)
            return dense_go<R, K, INTRA, false>(L, p0, p1, s);
    }
    return dense_go<R, K, W1, false>(L, p0, p1, s);
}

template <typename R>
hipError_t dense_k(const GateLaunch& L, void* p0, void* p1, hipStream_t s)
{
    switch (L.K) {
    case 1: return dense_mode<R, 1>(L, p0, p1, s);
    case 2: return dense_mode<R, 2>(L, p0, p1, s);
    case 3: return dense_mode<R, 3>(L, p0, p1, s);
    case 4: return dense_mode<R, 4>(L, p0, p1, s);
    case 5: return dense_mode<R, 5>(L, p0, p1, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename R, int MODE, bool ROT, bool NT>
hipError_t diag_launch(const DiagK<R>& a, const GateLaunch& L, void* p0, void* p1, hipStream_t s)
{
    dim3 grid(grid_for(L.ngroups, 1), p1 ? 2 : 1);
    hipLaunchKernelGGL((k_diag<R, MODE, ROT, 1, NT>), grid, dim3(kBlock), 0, s, static_cast<R*>(p0),
                       static_cast<R*>(p1 ? p1 : p0), a);
    return hipGetLastError();
}

template <typename R>
hipError_t diag_go(const GateLaunch& L, void* p0, void* p1, hipStream_t s)
{
    DiagK<R> a{};
    a.ngroups = L.ngroups;
    a.ins = L.ins;
    a.nt = L.K;
    for (int j = 0; j < 5; ++j)
        a.tpos[j] = L.tpos[j];
    if (L.rot == ROT_NONE)
        for (int j = 0; j < (2 << L.K); ++j)
            a.d[j] = (R)L.g[j];
    a.params = L.params;
    a.pidx = L.pidx;
    a.dag = L.dag;
    const bool w2 = sizeof(R) == 4 && L.mode == W2;
    const bool nt = use_nt(L.ins, w2 ? 16 : (int)(2 * sizeof(R)));
    const bool rot = L.rot != ROT_NONE;
    if (w2)
        return rot ? (nt ? diag_launch<R, W2, true, true>(a, L, p0, p1, s) : diag_launch<R, W2, true, false>(a, L, p0, p1, s))
                   : (nt ? diag_launch<R, W2, false, true>(a, L, p0, p1, s) : diag_launch<R, W2, false, false>(a, L, p0, p1, s));
    return rot ? (nt ? diag_launch<R, W1, true, true>(a, L, p0, p1, s) : diag_launch<R, W1, true, false>(a, L, p0, p1, s))
               : (nt ? diag_launch<R, W1, false, true>(a, L, p0, p1, s) : diag_launch<R, W1, false, false>(a, L, p0, p1, s));
}

template <typename UT, int NM>
hipError_t perm_go2(const GateLaunch& L, const PermK& a, void* p0, void* p1, hipStream_t s)
{
    dim3 grid(grid_for(L.ngroups, 1), p1 ? 2 : 1);
    if (use_nt(L.ins, (int)sizeof(UT)))
        hipLaunchKernelGGL((k_perm<UT, NM, 1, true>), grid, dim3(kBlock), 0, s, static_cast<UT*>(p0),
                           static_cast<UT*>(p1 ? p1 : p0), a);
    else
        hipLaunchKernelGGL((k_perm<UT, NM, 1, false>), grid, dim3(kBlock), 0, s, static_cast<UT*>(p0),
                           static_cast<UT*>(p1 ? p1 : p0), a);
    return hipGetLastError();
}

template <typename UT>
hipError_t perm_go(const GateLaunch& L, void* p0, void* p1, hipStream_t s)
{
    PermK a{};
    a.ngroups = L.ngroups;
    a.ins = L.ins;
    a.nmoved = L.nmoved;
    for (int j = 0; j < 32; ++j) {
        a.dst[j] = L.off[j];
        a.src[j] = L.off2[j];
    }
    if (L.nmoved <= 2)
        return perm_go2<UT, 2>(L, a, p0, p1, s);
    if (L.nmoved <= 4)
        return perm_go2<UT, 4>(L, a, p0, p1, s);
    if (L.nmoved <= 8)
        return perm_go2<UT, 8>(L, a, p0, p1, s);
    if (L.nmoved <= 16)
        return perm_go2<UT, 16>(L, a, p0, p1, s);
    return perm_go2<UT, 32>(L, a, p0, p1, s);
}

}  // namespace

hipError_t launch_gate(const GateLaunch& L, void* psi, void* psi2, hipStream_t s)
{
    if (L.ngroups == 0)
        return hipSuccess;
    switch (L.type) {
    case L_DENSE:
        return L.dt == C64 ? dense_k<float>(L, psi, psi2, s) : dense_k<double>(L, psi, psi2, s);
    case L_DIAG:
        return L.dt == C64 ? diag_go<float>(L, psi, psi2, s) : diag_go<double>(L, psi, psi2, s);
    case L_PERM:
        if (L.dt == C64 && L.mode == W1)
            return perm_go<uint2>(L, psi, psi2, s);
        return perm_go<uint4>(L, psi, psi2, s);
    case L_MFMA:
        return launch_mfma(L, psi, psi2, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_init_basis(void* psi, int n, int dt, uint64_t index, hipStream_t s)
{
    const uint64_t N = 1ull << n;
    if (dt == C64) {
        const uint64_t nvec = (N + 1) / 2;
        hipLaunchKernelGGL(k_init_basis<float>, dim3(grid_for(nvec, 4)), dim3(kBlock), 0, s,
                           static_cast<float*>(psi), nvec, index);
    } else {
        hipLaunchKernelGGL(k_init_basis<double>, dim3(grid_for(N, 4)), dim3(kBlock), 0, s,
                           static_cast<double*>(psi), N, index);
    }
    return hipGetLastError();
}

hipError_t launch_init_random(void* psi, int n, int dt, uint64_t seed, double* work, hipStream_t s)
{
    const uint64_t N = 1ull << n;
    const int nb = (int)grid_for(N, 16) > 1024 ? 1024 : (int)grid_for(N, 16);
    hipLaunchKernelGGL(k_rand_norm, dim3(nb), dim3(kBlock), 0, s, N, seed, work);
    hipLaunchKernelGGL(k_rand_scale, dim3(1), dim3(kBlock), 0, s, work, nb, work + 1024);
    if (dt == C64)
        hipLaunchKernelGGL(k_rand_fill<float>, dim3(grid_for(N, 4)), dim3(kBlock), 0, s,
                           static_cast<float*>(psi), N, seed, work + 1024);
    else
        hipLaunchKernelGGL(k_rand_fill<double>, dim3(grid_for(N, 4)), dim3(kBlock), 0, s,
                           static_cast<double*>(psi), N, seed, work + 1024);
    return hipGetLastError();
}

}  // namespace qsv
