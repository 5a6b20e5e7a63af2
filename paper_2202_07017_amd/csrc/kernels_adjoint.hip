// Reverse-sweep kernels of the adjoint gradient.
//
// For a rotation U = exp(-i theta P / 2) the derivative times the inverse is
// dU/dtheta U^dagger = -(i/2) P, so with phi_k = U_k..U_1|0> and
// lam_k = U_{k+1}^dagger..U_N^dagger H psi_N the gradient entry
// 2 Re <lam_k| dU_k phi_{k-1}> equals Im <lam_k| P |phi_k>: it needs the two
// vectors as they are *before* gate k is uncomputed and no derivative matrix.
// One kernel therefore reads phi and lam once, adds the FP64 block partial of
// Im <lam|P phi> over the pair (or amplitude), applies U^dagger = U(-theta) to
// both and writes them back: 4 state sweeps of traffic per rotation.  For a
// controlled rotation the groups only visit the control-on subspace, which is
// exactly where dU is non-zero.
#include "qsv_internal.h"

namespace qsv {
namespace {

__device__ __forceinline__ uint64_t insert_bits(uint64_t g, const InsertSpec& s)
{
    for (int j = 0; j < s.nins; ++j) {
        const uint64_t lo = s.low[j];
        g = ((g & ~lo) << 1) | (g & lo);
    }
    return g | s.setmask;
}

struct AdjK {
    uint64_t ngroups;
    InsertSpec ins;
    uint64_t off1;  // unit offset of the partner (W1/W2); unused for INTRA
    int tpos;       // amplitude-space target position (RZ)
    const double* params;
    int pidx;
};

struct C2 {
    double re, im;
};

// Im(conj(l) * v)
__device__ __forceinline__ double im_conj_mul(C2 l, C2 v)
{
    return l.re * v.im - l.im * v.re;
}
__device__ __forceinline__ double re_conj_mul(C2 l, C2 v)
{
    return l.re * v.re + l.im * v.im;
}

// Contribution Im(conj(l0) (P v)_0 + conj(l1) (P v)_1) for P = X or Y.
template <int ROTK>
__device__ __forceinline__ double pair_term(C2 l0, C2 l1, C2 v0, C2 v1)
{
    if constexpr (ROTK == ROT_X)  // (P v) = (v1, v0)
        return im_conj_mul(l0, v1) + im_conj_mul(l1, v0);
    else  // Y: (P v) = (-i v1, i v0);  Im(conj(l) (-i v)) = -Re(conj(l) v)
        return -re_conj_mul(l0, v1) + re_conj_mul(l1, v0);
}

// U(-theta) applied to (v0, v1):  m = row-major 2x2 (re, im)
__device__ __forceinline__ void rot2(const double* m, C2& v0, C2& v1)
{
    const C2 a = v0, b = v1;
    v0.re = m[0] * a.re - m[1] * a.im + m[2] * b.re - m[3] * b.im;
    v0.im = m[0] * a.im + m[1] * a.re + m[2] * b.im + m[3] * b.re;
    v1.re = m[4] * a.re - m[5] * a.im + m[6] * b.re - m[7] * b.im;
    v1.im = m[4] * a.im + m[5] * a.re + m[6] * b.im + m[7] * b.re;
}

__device__ __forceinline__ void block_partial(double s, double* partials)
{
    __shared__ double red[kBlock];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        partials[blockIdx.x] = red[0];
}

template <typename R>
struct Ld;
template <>
struct Ld<float> {
    using A = float2;
};
template <>
struct Ld<double> {
    using A = double2;
};

template <typename R>
__device__ __forceinline__ C2 get(const R* p, uint64_t i)
{
    const typename Ld<R>::A a = reinterpret_cast<const typename Ld<R>::A*>(p)[i];
    return C2{(double)a.x, (double)a.y};
}
template <typename R>
__device__ __forceinline__ void put(R* p, uint64_t i, C2 v)
{
    typename Ld<R>::A a;
    a.x = (R)v.re;
    a.y = (R)v.im;
    reinterpret_cast<typename Ld<R>::A*>(p)[i] = a;
}

// RX / RY step.  MODE W1: unit = amplitude; W2 (c64): float4 = two groups;
// INTRA (c64, target 0): float4 = the pair itself.
template <typename R, int MODE, int ROTK>
__global__ void __launch_bounds__(kBlock) k_adj_pair(R* __restrict__ phi, R* __restrict__ lam,
                                                     const AdjK a, double* partials)
{
    const double th = -a.params[a.pidx];
    const double c = cos(0.5 * th), s = sin(0.5 * th);
    double m[8] = {c, 0, 0, 0, 0, 0, c, 0};
    if constexpr (ROTK == ROT_X) {
        m[3] = -s;
        m[5] = -s;
    } else {
        m[2] = -s;
        m[4] = s;
    }
    double acc = 0.0;
    const uint64_t step = (uint64_t)gridDim.x * kBlock;
    for (uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x; g < a.ngroups; g += step) {
        const uint64_t i0 = insert_bits(g, a.ins);
        if constexpr (MODE == W1) {
            const uint64_t i1 = i0 + a.off1;
            C2 p0 = get(phi, i0), p1 = get(phi, i1), l0 = get(lam, i0), l1 = get(lam, i1);
            acc += pair_term<ROTK>(l0, l1, p0, p1);
            rot2(m, p0, p1);
            rot2(m, l0, l1);
            put(phi, i0, p0);
            put(phi, i1, p1);
            put(lam, i0, l0);
            put(lam, i1, l1);
        } else if constexpr (MODE == W2) {
            float4* P = reinterpret_cast<float4*>(phi);
            float4* Lm = reinterpret_cast<float4*>(lam);
            const uint64_t i1 = i0 + a.off1;
            const float4 fp0 = P[i0], fp1 = P[i1], fl0 = Lm[i0], fl1 = Lm[i1];
            C2 pa0{fp0.x, fp0.y}, pa1{fp1.x, fp1.y}, pb0{fp0.z, fp0.w}, pb1{fp1.z, fp1.w};
            C2 la0{fl0.x, fl0.y}, la1{fl1.x, fl1.y}, lb0{fl0.z, fl0.w}, lb1{fl1.z, fl1.w};
            acc += pair_term<ROTK>(la0, la1, pa0, pa1) + pair_term<ROTK>(lb0, lb1, pb0, pb1);
            rot2(m, pa0, pa1);
            rot2(m, pb0, pb1);
            rot2(m, la0, la1);
            rot2(m, lb0, lb1);
            P[i0] = make_float4(pa0.re, pa0.im, pb0.re, pb0.im);
            P[i1] = make_float4(pa1.re, pa1.im, pb1.re, pb1.im);
            Lm[i0] = make_float4(la0.re, la0.im, lb0.re, lb0.im);
            Lm[i1] = make_float4(la1.re, la1.im, lb1.re, lb1.im);
        } else {  // INTRA
            float4* P = reinterpret_cast<float4*>(phi);
            float4* Lm = reinterpret_cast<float4*>(lam);
            const float4 fp = P[i0], fl = Lm[i0];
            C2 p0{fp.x, fp.y}, p1{fp.z, fp.w}, l0{fl.x, fl.y}, l1{fl.z, fl.w};
            acc += pair_term<ROTK>(l0, l1, p0, p1);
            rot2(m, p0, p1);
            rot2(m, l0, l1);
            P[i0] = make_float4(p0.re, p0.im, p1.re, p1.im);
            Lm[i0] = make_float4(l0.re, l0.im, l1.re, l1.im);
        }
    }
    block_partial(acc, partials);
}

// RZ step: per amplitude, s = +1 (target bit 0) / -1 (bit 1);
// partial += s Im(conj(lam) phi); phi, lam *= conj(d_bit).
template <typename R, int MODE>
__global__ void __launch_bounds__(kBlock) k_adj_z(R* __restrict__ phi, R* __restrict__ lam,
                                                  const AdjK a, double* partials)
{
    const double th = a.params[a.pidx];
    const double c = cos(0.5 * th), s = sin(0.5 * th);
    // U^dagger = diag(e^{+i th/2}, e^{-i th/2})
    double acc = 0.0;
    const uint64_t step = (uint64_t)gridDim.x * kBlock;
    for (uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x; g < a.ngroups; g += step) {
        const uint64_t u = insert_bits(g, a.ins);
        if constexpr (MODE == W1) {
            const int b = (int)((u >> a.tpos) & 1u);
            const double si = b ? -s : s;  // e^{i th/2} for bit 0, e^{-i th/2} for bit 1
            C2 p = get(phi, u), l = get(lam, u);
            acc += (b ? -1.0 : 1.0) * im_conj_mul(l, p);
            put(phi, u, C2{c * p.re - si * p.im, c * p.im + si * p.re});
            put(lam, u, C2{c * l.re - si * l.im, c * l.im + si * l.re});
        } else {  // W2: float4 holds amplitudes 2u, 2u+1
            float4* P = reinterpret_cast<float4*>(phi);
            float4* Lm = reinterpret_cast<float4*>(lam);
            const float4 fp = P[u], fl = Lm[u];
            C2 pv[2] = {{fp.x, fp.y}, {fp.z, fp.w}};
            C2 lv[2] = {{fl.x, fl.y}, {fl.z, fl.w}};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int b = (int)((((u << 1) | (uint64_t)h) >> a.tpos) & 1u);
                const double si = b ? -s : s;
                acc += (b ? -1.0 : 1.0) * im_conj_mul(lv[h], pv[h]);
                const C2 p = pv[h], l = lv[h];
                pv[h] = C2{c * p.re - si * p.im, c * p.im + si * p.re};
                lv[h] = C2{c * l.re - si * l.im, c * l.im + si * l.re};
            }
            P[u] = make_float4(pv[0].re, pv[0].im, pv[1].re, pv[1].im);
            Lm[u] = make_float4(lv[0].re, lv[0].im, lv[1].re, lv[1].im);
        }
    }
    block_partial(acc, partials);
}

// grad[p] = sum over the slots of parameter p (in slot order) of the in-order
// sum of that slot's nb partials.
__global__ void __launch_bounds__(kBlock) k_grad_finalize(const double* partials, int nb,
                                                          const int* pstart, const int* plist,
                                                          double* grad)
{
    __shared__ double red[kBlock];
    const int p = blockIdx.x;
    double total = 0.0;
    for (int k = pstart[p]; k < pstart[p + 1]; ++k) {
        const double* src = partials + (size_t)plist[k] * nb;
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += kBlock)
            s += src[b];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w)
                red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        total += red[0];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        grad[p] = total;
}

template <typename R>
hipError_t adj_go(const GateLaunch& L, void* phi, void* lam, double* partials, int nb, hipStream_t s)
{
    AdjK a{};
    a.ngroups = L.ngroups;
    a.ins = L.ins;
    a.off1 = L.off[1];
    a.tpos = L.tpos[0];
    a.params = L.params;
    a.pidx = L.pidx;
    R* p = static_cast<R*>(phi);
    R* l = static_cast<R*>(lam);
    dim3 g(nb), b(kBlock);
    if (L.type == L_DIAG) {
        if (sizeof(R) == 4 && L.mode == W2)
            hipLaunchKernelGGL((k_adj_z<R, W2>), g, b, 0, s, p, l, a, partials);
        else
            hipLaunchKernelGGL((k_adj_z<R, W1>), g, b, 0, s, p, l, a, partials);
        return hipGetLastError();
    }
    const bool x = L.rot == ROT_X;
    if (sizeof(R) == 4 && L.mode == W2) {
        if (x)
            hipLaunchKernelGGL((k_adj_pair<R, W2, ROT_X>), g, b, 0, s, p, l, a, partials);
        else
            hipLaunchKernelGGL((k_adj_pair<R, W2, ROT_Y>), g, b, 0, s, p, l, a, partials);
    } else if (sizeof(R) == 4 && L.mode == INTRA) {
        if (x)
            hipLaunchKernelGGL((k_adj_pair<R, INTRA, ROT_X>), g, b, 0, s, p, l, a, partials);
        else
            hipLaunchKernelGGL((k_adj_pair<R, INTRA, ROT_Y>), g, b, 0, s, p, l, a, partials);
    } else {
        if (x)
            hipLaunchKernelGGL((k_adj_pair<R, W1, ROT_X>), g, b, 0, s, p, l, a, partials);
        else
            hipLaunchKernelGGL((k_adj_pair<R, W1, ROT_Y>), g, b, 0, s, p, l, a, partials);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_adj_step(const GateLaunch& L, void* phi, void* lam, double* partials, int nb,
                           hipStream_t s)
{
    return L.dt == C64 ? adj_go<float>(L, phi, lam, partials, nb, s)
                       : adj_go<double>(L, phi, lam, partials, nb, s);
}

hipError_t launch_grad_finalize(const double* partials, int nblocks, const int* pstart,
                                const int* plist, int nparams, double* grad, hipStream_t s)
{
    if (nparams == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_grad_finalize, dim3(nparams), dim3(kBlock), 0, s, partials, nblocks, pstart,
                       plist, grad);
    return hipGetLastError();
}

}  // namespace qsv
