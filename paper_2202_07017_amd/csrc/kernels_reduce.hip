// FP64 reductions over a state: norm, Pauli-sum expectation values
// (Sec. 3, Hamiltonian primitives), inner products, and H psi.
//
// A Pauli string with masks (x, z) and y = #Y factors maps |i> to
// i^y (-1)^popcount(i & z) |i xor x>.  Terms with x = 0 are diagonal and share
// one streaming pass; terms with the same x != 0 share a pass that visits each
// pair (i, i xor x) once, so every amplitude is read once per pass.
//
// Every reduction is deterministic: a fixed grid of reduce_blocks(n) blocks,
// a fixed per-thread visiting order, a fixed in-block tree, per-block FP64
// partials in device memory, and a one-block finalize that adds them in
// index order.  Amplitudes are widened to FP64 before any product.
#include <mutex>

#include "qsv_internal.h"

// Partial sums of qsv_expectation_noalloc.  Each GPU holds its own copy
// until the process ends; every call on a GPU shares it (calls that overlap
// in time on one GPU race on it).
static __device__ __align__(256) double scratch[qsv::kStaticScratchBytes / sizeof(double)];

namespace qsv {

hipError_t static_scratch(double** ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {nullptr};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        addr[dev] = p;
    }
    *ptr = static_cast<double*>(addr[dev]);
    return hipSuccess;
}

int reduce_blocks(int n, int dt)
{
    (void)dt;
    const uint64_t N = 1ull << n;
    uint64_t b = N / (kBlock * 16);
    if (b < 1)
        b = 1;
    if (b > 1024)
        b = 1024;
    return (int)b;
}

namespace {

__device__ __forceinline__ void block_sum_store(double v, double* out)
{
    __shared__ double red[kBlock];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *out = red[0];
    __syncthreads();
}

typedef float nv4f __attribute__((ext_vector_type(4)));
typedef double nv2d __attribute__((ext_vector_type(2)));

// A 16-byte load, streamed past the caches (NT) for states far larger than
// the caches, plain for states that the previous kernel left in L2 / MALL.
template <bool NT, typename V>
__device__ __forceinline__ V ldu(const V* p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <typename R>
struct W;
template <>
struct W<float> {
    using A = float2;
};
template <>
struct W<double> {
    using A = double2;
};

template <typename R>
__device__ __forceinline__ double2 ld(const R* p, uint64_t i)
{
    const typename W<R>::A a = reinterpret_cast<const typename W<R>::A*>(p)[i];
    return make_double2((double)a.x, (double)a.y);
}

template <typename R>
__device__ __forceinline__ void st(R* p, uint64_t i, double2 v)
{
    typename W<R>::A a;
    a.x = (R)v.x;
    a.y = (R)v.y;
    reinterpret_cast<typename W<R>::A*>(p)[i] = a;
}

// Two adjacent complex64 amplitudes (one 16-byte load), widened to FP64.
__device__ __forceinline__ void ld_pair(const float* p, uint64_t v, double2& a0, double2& a1)
{
    const float4 f = reinterpret_cast<const float4*>(p)[v];
    a0 = make_double2((double)f.x, (double)f.y);
    a1 = make_double2((double)f.z, (double)f.w);
}

__device__ __forceinline__ int popc64(uint64_t v)
{
    return __popcll(v);
}

// Block index in XCD-contiguous order (a bijection on [0, gridDim.x)): the
// hardware deals blocks round-robin to the 8 XCDs, so block b reads the
// slice of logical block (b mod 8) * G/8 + b / 8 and each XCD streams one
// contiguous eighth of every round of the grid-stride loop.
__device__ __forceinline__ uint64_t xcd_block()
{
    const uint32_t G = gridDim.x, b = blockIdx.x, per = G >> 3;
    return b < (per << 3) ? (uint64_t)(b & 7u) * per + (b >> 3) : (uint64_t)b;
}

// sum_j c_j (-1)^popcount(i & z_j)
__device__ __forceinline__ double diag_weight(uint64_t i, const TermChunk& t)
{
    double w = 0.0;
    for (int j = 0; j < t.nt; ++j)
        w += (popc64(i & t.z[j]) & 1) ? -t.c[j] : t.c[j];
    return w;
}

// f(i) = sum_j c_j i^(y_j + 2 popcount(i & z_j))
__device__ __forceinline__ double2 phase_sum(uint64_t i, const TermChunk& t)
{
    double re = 0.0, im = 0.0;
    for (int j = 0; j < t.nt; ++j) {
        const int e = (t.ylo[j] + 2 * popc64(i & t.z[j])) & 3;
        const double c = t.c[j];
        re += e == 0 ? c : (e == 2 ? -c : 0.0);
        im += e == 1 ? c : (e == 3 ? -c : 0.0);
    }
    return make_double2(re, im);
}

template <typename R, bool NT>
__global__ void __launch_bounds__(kBlock) k_norm2(const R* __restrict__ psi, uint64_t N,
                                                  double* partials, int accumulate)
{
    (void)accumulate;
    // software pipeline: the next round's U loads are issued before this
    // round's squares are summed; the sums keep the thread's index order
    constexpr int U = 4;
    using A = typename W<R>::A;
    const A* p = reinterpret_cast<const A*>(psi);
    double s = 0.0;
    const uint64_t step = (uint64_t)gridDim.x * kBlock;
    const uint64_t nu = sizeof(R) == 4 ? N / 2 : N;  // 16-byte units
    auto unit = [&](uint64_t v) {
        if constexpr (sizeof(R) == 4) {
            const nv4f f = ldu<NT>(reinterpret_cast<const nv4f*>(p) + v);
            return make_double4((double)f.x, (double)f.y, (double)f.z, (double)f.w);
        } else {
            const nv2d a = ldu<NT>(reinterpret_cast<const nv2d*>(p) + v);
            return make_double4(a.x, a.y, 0.0, 0.0);
        }
    };
    auto sq = [](const double4& d) { return d.x * d.x + d.y * d.y + (d.z * d.z + d.w * d.w); };
    uint64_t v = xcd_block() * kBlock + threadIdx.x;
    if (v + (U - 1) * step < nu) {
        double4 cur[U], nxt[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            cur[u] = unit(v + (uint64_t)u * step);
        for (;;) {
            const uint64_t vn = v + U * step;
            const bool more = vn + (U - 1) * step < nu;
            if (more) {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    nxt[u] = unit(vn + (uint64_t)u * step);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                s += sq(cur[u]);
            v = vn;
            if (!more)
                break;
#pragma unroll
            for (int u = 0; u < U; ++u)
                cur[u] = nxt[u];
        }
    }
    for (; v < nu; v += step)
        s += sq(unit(v));
    if (sizeof(R) == 4 && N == 1 && blockIdx.x == 0 && threadIdx.x == 0) {
        const double2 a = ld(psi, 0);
        s += a.x * a.x + a.y * a.y;
    }
    block_sum_store(s, partials + blockIdx.x);
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_expect_diag(const R* __restrict__ psi, uint64_t N,
                                                        const TermChunk t, double* partials,
                                                        int accumulate)
{
    double s = 0.0;
    const uint64_t step = (uint64_t)gridDim.x * kBlock;
    if constexpr (sizeof(R) == 4) {
        for (uint64_t v = (uint64_t)blockIdx.x * kBlock + threadIdx.x; v < N / 2; v += step) {
            double2 a, b;
            ld_pair(psi, v, a, b);
            s += diag_weight(2 * v, t) * (a.x * a.x + a.y * a.y) +
                 diag_weight(2 * v + 1, t) * (b.x * b.x + b.y * b.y);
        }
        if (N == 1 && blockIdx.x == 0 && threadIdx.x == 0) {
            const double2 a = ld(psi, 0);
            s += diag_weight(0, t) * (a.x * a.x + a.y * a.y);
        }
    } else {
        for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += step) {
            const double2 a = ld(psi, i);
            s += diag_weight(i, t) * (a.x * a.x + a.y * a.y);
        }
    }
    __shared__ double red[kBlock];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* p = partials + blockIdx.x;
        double* q = partials + gridDim.x + blockIdx.x;
        *p = accumulate ? *p + red[0] : red[0];
        if (!accumulate)
            *q = 0.0;
    }
}

// Pairs (i, j = i xor x), bit h (top bit of x) of i clear.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_expect_pair(const R* __restrict__ psi, uint64_t npairs,
                                                        uint64_t x, uint64_t lowmask,
                                                        const TermChunk t, double* partials,
                                                        int accumulate)
{
    double sr = 0.0, si = 0.0;
    const uint64_t step = (uint64_t)gridDim.x * kBlock;
    for (uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x; g < npairs; g += step) {
        const uint64_t i = ((g & ~lowmask) << 1) | (g & lowmask);
        const uint64_t j = i ^ x;
        const double2 a = ld(psi, i), b = ld(psi, j);
        // w = conj(psi_j) psi_i
        const double wr = b.x * a.x + b.y * a.y, wi = b.x * a.y - b.y * a.x;
        const double2 fi = phase_sum(i, t), fj = phase_sum(j, t);
        // Re[w (f(i) + conj f(j))], Im[w (f(i) - conj f(j))]
        const double pr = fi.x + fj.x, pi = fi.y - fj.y;
        const double qr = fi.x - fj.x, qi = fi.y + fj.y;
        sr += wr * pr - wi * pi;
        si += wr * qi + wi * qr;
    }
    __shared__ double red[2][kBlock];
    red[0][threadIdx.x] = sr;
    red[1][threadIdx.x] = si;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* p = partials + blockIdx.x;
        double* q = partials + gridDim.x + blockIdx.x;
        *p = accumulate ? *p + red[0][0] : red[0][0];
        *q = accumulate ? *q + red[1][0] : red[1][0];
    }
}

// One string per launch (the usual case for strings that no tile pass
// holds): its z mask, coefficient and Y count stay in registers, the phase
// of the partner follows from the phase of i (popcount(j & z) = popcount(i
// & z) + popcount(x & z) mod 2), and each thread keeps four pairs' loads in
// flight.  The per-thread order of the sums is that of k_expect_pair.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_expect_pair1(const R* __restrict__ psi, uint64_t npairs,
                                                         uint64_t x, uint64_t lowmask, uint64_t z,
                                                         double c, int ylo, double* partials,
                                                         int accumulate)
{
    const int dx = popc64(x & z) & 1;
    double sr = 0.0, si = 0.0;
    auto add = [&](uint64_t i, double2 a, double2 b) {
        const double wr = b.x * a.x + b.y * a.y, wi = b.x * a.y - b.y * a.x;
        const int p = popc64(i & z) & 1;
        const int ei = (ylo + 2 * p) & 3, ej = (ylo + 2 * (p ^ dx)) & 3;
        const double2 fi = make_double2(ei == 0 ? c : (ei == 2 ? -c : 0.0), ei == 1 ? c : (ei == 3 ? -c : 0.0));
        const double2 fj = make_double2(ej == 0 ? c : (ej == 2 ? -c : 0.0), ej == 1 ? c : (ej == 3 ? -c : 0.0));
        const double pr = fi.x + fj.x, pi = fi.y - fj.y;
        const double qr = fi.x - fj.x, qi = fi.y + fj.y;
        sr += wr * pr - wi * pi;
        si += wr * qi + wi * qr;
    };
    const uint64_t step = (uint64_t)gridDim.x * kBlock;
    uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    for (; g + 3 * step < npairs; g += 4 * step) {
        uint64_t i[4];
        double2 a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t gu = g + (uint64_t)u * step;
            i[u] = ((gu & ~lowmask) << 1) | (gu & lowmask);
            a[u] = ld(psi, i[u]);
            b[u] = ld(psi, i[u] ^ x);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            add(i[u], a[u], b[u]);
    }
    for (; g < npairs; g += step) {
        const uint64_t i = ((g & ~lowmask) << 1) | (g & lowmask);
        add(i, ld(psi, i), ld(psi, i ^ x));
    }
    __shared__ double red[2][kBlock];
    red[0][threadIdx.x] = sr;
    red[1][threadIdx.x] = si;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* p = partials + blockIdx.x;
        double* q = partials + gridDim.x + blockIdx.x;
        *p = accumulate ? *p + red[0][0] : red[0][0];
        *q = accumulate ? *q + red[1][0] : red[1][0];
    }
}

template <typename R, bool NT>
__global__ void __launch_bounds__(kBlock) k_inner(const R* __restrict__ a, const R* __restrict__ b,
                                                  uint64_t N, double* partials, int accumulate)
{
    // software pipeline as in k_norm2: the next round's loads of both
    // vectors are issued before this round's products are summed; the sums
    // keep the thread's index order
    constexpr int U = 2;
    double sr = 0.0, si = 0.0;
    const uint64_t step = (uint64_t)gridDim.x * kBlock;
    const uint64_t nu = sizeof(R) == 4 ? N / 2 : N;  // 16-byte units
    auto unit = [&](const R* q, uint64_t v) {
        if constexpr (sizeof(R) == 4) {
            const nv4f f = ldu<NT>(reinterpret_cast<const nv4f*>(q) + v);
            return make_double4((double)f.x, (double)f.y, (double)f.z, (double)f.w);
        } else {
            const nv2d d = ldu<NT>(reinterpret_cast<const nv2d*>(q) + v);
            return make_double4(d.x, d.y, 0.0, 0.0);
        }
    };
    // conj(u) v summed over the unit's amplitudes (complex128: the zero
    // second half adds exact zeros)
    auto add = [&](const double4& u, const double4& v) {
        sr += (u.x * v.x + u.y * v.y) + (u.z * v.z + u.w * v.w);
        si += (u.x * v.y - u.y * v.x) + (u.z * v.w - u.w * v.z);
    };
    uint64_t v = xcd_block() * kBlock + threadIdx.x;
    if (v + (U - 1) * step < nu) {
        double4 ca[U], cb[U], na[U], nb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ca[u] = unit(a, v + (uint64_t)u * step);
            cb[u] = unit(b, v + (uint64_t)u * step);
        }
        for (;;) {
            const uint64_t vn = v + U * step;
            const bool more = vn + (U - 1) * step < nu;
            if (more) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    na[u] = unit(a, vn + (uint64_t)u * step);
                    nb[u] = unit(b, vn + (uint64_t)u * step);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                add(ca[u], cb[u]);
            v = vn;
            if (!more)
                break;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                ca[u] = na[u];
                cb[u] = nb[u];
            }
        }
    }
    for (; v < nu; v += step)
        add(unit(a, v), unit(b, v));
    if (sizeof(R) == 4 && N == 1 && blockIdx.x == 0 && threadIdx.x == 0) {
        const double2 u = ld(a, 0), w = ld(b, 0);
        sr += u.x * w.x + u.y * w.y;
        si += u.x * w.y - u.y * w.x;
    }
    __shared__ double red[2][kBlock];
    red[0][threadIdx.x] = sr;
    red[1][threadIdx.x] = si;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* p = partials + blockIdx.x;
        double* q = partials + gridDim.x + blockIdx.x;
        *p = accumulate ? *p + red[0][0] : red[0][0];
        *q = accumulate ? *q + red[1][0] : red[1][0];
    }
}

// out[c] = sum_b partials[c * nb + b] in index order, c < ncomp.
__global__ void __launch_bounds__(kBlock) k_finalize(const double* partials, int nb, int ncomp,
                                                     double* out)
{
    __shared__ double red[kBlock];
    for (int c = 0; c < ncomp; ++c) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += kBlock)
            s += partials[c * nb + b];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w)
                red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0)
            out[c] = red[0];
        __syncthreads();
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_hpsi_diag(const R* __restrict__ psi, R* __restrict__ lam,
                                                      uint64_t N, const TermChunk t, int accumulate)
{
    const uint64_t step = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += step) {
        const double2 a = ld(psi, i);
        const double w = diag_weight(i, t);
        double2 o = make_double2(w * a.x, w * a.y);
        if (accumulate) {
            const double2 l = ld(lam, i);
            o.x += l.x;
            o.y += l.y;
        }
        st(lam, i, o);
    }
}

// lam_i += f(j) psi_j, lam_j += f(i) psi_i for the pairs of mask x.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_hpsi_pair(const R* __restrict__ psi, R* __restrict__ lam,
                                                      uint64_t npairs, uint64_t x, uint64_t lowmask,
                                                      const TermChunk t)
{
    const uint64_t step = (uint64_t)gridDim.x * kBlock;
    for (uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x; g < npairs; g += step) {
        const uint64_t i = ((g & ~lowmask) << 1) | (g & lowmask);
        const uint64_t j = i ^ x;
        const double2 a = ld(psi, i), b = ld(psi, j);
        const double2 fi = phase_sum(i, t), fj = phase_sum(j, t);
        double2 li = ld(lam, i), lj = ld(lam, j);
        li.x += fj.x * b.x - fj.y * b.y;
        li.y += fj.x * b.y + fj.y * b.x;
        lj.x += fi.x * a.x - fi.y * a.y;
        lj.y += fi.x * a.y + fi.y * a.x;
        st(lam, i, li);
        st(lam, j, lj);
    }
}

__global__ void k_fill_zero(double* p, uint64_t count)
{
    const uint64_t step = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += step)
        p[i] = 0.0;
}

inline unsigned stream_grid(uint64_t items)
{
    uint64_t b = (items + kBlock * 4 - 1) / (kBlock * 4);
    if (b < 1)
        b = 1;
    if (b > (1u << 20))
        b = 1u << 20;
    return (unsigned)b;
}

// Reads of more than 1 GiB stream past the caches (the 256 MiB of MALL and
// the L2s cannot hold them); smaller ones keep the plain loads, which hit
// whatever the previous kernel left there (adjoint states of 20-24 qubits).
bool streamed(uint64_t bytes) { return bytes > (1ull << 30); }

}  // namespace

hipError_t launch_norm2(const void* psi, int n, int dt, double* partials, int accumulate,
                        hipStream_t s)
{
    const int nb = reduce_blocks(n, dt);
    const uint64_t N = 1ull << n;
    const bool nt = streamed(N * (dt == C64 ? 8 : 16));
    if (dt == C64)
        hipLaunchKernelGGL((nt ? k_norm2<float, true> : k_norm2<float, false>), dim3(nb), dim3(kBlock), 0, s,
                           static_cast<const float*>(psi), N, partials, accumulate);
    else
        hipLaunchKernelGGL((nt ? k_norm2<double, true> : k_norm2<double, false>), dim3(nb), dim3(kBlock), 0, s,
                           static_cast<const double*>(psi), N, partials, accumulate);
    return hipGetLastError();
}

hipError_t launch_expect_diag(const void* psi, int n, int dt, const TermChunk& t, double* partials,
                              int accumulate, hipStream_t s)
{
    const int nb = reduce_blocks(n, dt);
    const uint64_t N = 1ull << n;
    if (dt == C64)
        hipLaunchKernelGGL(k_expect_diag<float>, dim3(nb), dim3(kBlock), 0, s,
                           static_cast<const float*>(psi), N, t, partials, accumulate);
    else
        hipLaunchKernelGGL(k_expect_diag<double>, dim3(nb), dim3(kBlock), 0, s,
                           static_cast<const double*>(psi), N, t, partials, accumulate);
    return hipGetLastError();
}

static uint64_t top_low_mask(uint64_t x)
{
    int h = 63;
    while (h > 0 && !((x >> h) & 1ull))
        --h;
    return (1ull << h) - 1;
}

hipError_t launch_expect_pair(const void* psi, int n, int dt, uint64_t x, const TermChunk& t,
                              double* partials, int accumulate, hipStream_t s)
{
    const int nb = reduce_blocks(n, dt);
    const uint64_t np = 1ull << (n - 1);
    const uint64_t lm = top_low_mask(x);
    if (t.nt == 1) {
        if (dt == C64)
            hipLaunchKernelGGL(k_expect_pair1<float>, dim3(nb), dim3(kBlock), 0, s, static_cast<const float*>(psi),
                               np, x, lm, t.z[0], t.c[0], t.ylo[0], partials, accumulate);
        else
            hipLaunchKernelGGL(k_expect_pair1<double>, dim3(nb), dim3(kBlock), 0, s,
                               static_cast<const double*>(psi), np, x, lm, t.z[0], t.c[0], t.ylo[0], partials,
                               accumulate);
        return hipGetLastError();
    }
    if (dt == C64)
        hipLaunchKernelGGL(k_expect_pair<float>, dim3(nb), dim3(kBlock), 0, s,
                           static_cast<const float*>(psi), np, x, lm, t, partials, accumulate);
    else
        hipLaunchKernelGGL(k_expect_pair<double>, dim3(nb), dim3(kBlock), 0, s,
                           static_cast<const double*>(psi), np, x, lm, t, partials, accumulate);
    return hipGetLastError();
}

hipError_t launch_inner(const void* a, const void* b, int n, int dt, double* partials2,
                        int accumulate, hipStream_t s)
{
    const int nb = reduce_blocks(n, dt);
    const uint64_t N = 1ull << n;
    const bool nt = streamed(2 * N * (dt == C64 ? 8 : 16));
    if (dt == C64)
        hipLaunchKernelGGL((nt ? k_inner<float, true> : k_inner<float, false>), dim3(nb), dim3(kBlock), 0, s,
                           static_cast<const float*>(a), static_cast<const float*>(b), N, partials2, accumulate);
    else
        hipLaunchKernelGGL((nt ? k_inner<double, true> : k_inner<double, false>), dim3(nb), dim3(kBlock), 0, s,
                           static_cast<const double*>(a), static_cast<const double*>(b), N, partials2,
                           accumulate);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, int nblocks, int ncomp, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, partials, nblocks, ncomp, out);
    return hipGetLastError();
}

hipError_t launch_hpsi_diag(const void* psi, void* lam, int n, int dt, const TermChunk& t,
                            int accumulate, hipStream_t s)
{
    const uint64_t N = 1ull << n;
    if (dt == C64)
        hipLaunchKernelGGL(k_hpsi_diag<float>, dim3(stream_grid(N)), dim3(kBlock), 0, s,
                           static_cast<const float*>(psi), static_cast<float*>(lam), N, t, accumulate);
    else
        hipLaunchKernelGGL(k_hpsi_diag<double>, dim3(stream_grid(N)), dim3(kBlock), 0, s,
                           static_cast<const double*>(psi), static_cast<double*>(lam), N, t,
                           accumulate);
    return hipGetLastError();
}

hipError_t launch_hpsi_pair(const void* psi, void* lam, int n, int dt, uint64_t x,
                            const TermChunk& t, hipStream_t s)
{
    const uint64_t np = 1ull << (n - 1);
    const uint64_t lm = top_low_mask(x);
    if (dt == C64)
        hipLaunchKernelGGL(k_hpsi_pair<float>, dim3(stream_grid(np)), dim3(kBlock), 0, s,
                           static_cast<const float*>(psi), static_cast<float*>(lam), np, x, lm, t);
    else
        hipLaunchKernelGGL(k_hpsi_pair<double>, dim3(stream_grid(np)), dim3(kBlock), 0, s,
                           static_cast<const double*>(psi), static_cast<double*>(lam), np, x, lm, t);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double* p, uint64_t count, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill_zero, dim3(stream_grid(count)), dim3(kBlock), 0, s, p, count);
    return hipGetLastError();
}

}  // namespace qsv
