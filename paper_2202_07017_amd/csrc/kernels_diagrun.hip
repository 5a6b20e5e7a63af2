// Diagonal runs: several diagonal gates applied to a state in one streaming
// sweep.  Diagonal matrices commute with each other, so the run's product
// does not depend on the order of its factors; plans build runs from
// consecutive diagonal gates (moving gates on other qubits ahead of them).
#include <cmath>
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
// for every factor f whose fixed bits match.
template <typename R>
struct DiagRunK {
    uint64_t nunits;  // 16-byte units of the state
    int nf;
    uint64_t fix[kMaxRunFactors];
    uint64_t val[kMaxRunFactors];
    uint64_t dep[kMaxRunFactors];  // every bit the factor reads (fixed and varying)
    int nt[kMaxRunFactors];
    int tpos[kMaxRunFactors][5];
    int off[kMaxRunFactors];       // first complex entry of the factor's table
    const R* tab;                  // all tables, (re, im), state precision
    int ntab;                      // complex entries in tab
};

// Multiplies (re, im) by factor f's entry for amplitude i, if i's fixed bits
// match; the tables sit in LDS.
template <typename R>
__device__ __forceinline__ void run_factor(const DiagRunK<R>& a, const R* sd, int f, uint64_t i, R& re,
                                           R& im)
{
    if ((i & a.fix[f]) != a.val[f])
        return;
    int t = 0;
    for (int b = 0; b < a.nt[f]; ++b)
        t |= (int)((i >> a.tpos[f][b]) & 1u) << b;
    const R dr = sd[2 * (a.off[f] + t)], di = sd[2 * (a.off[f] + t) + 1];
    const R r = re * dr - im * di;
    im = re * di + im * dr;
    re = r;
}

// Each thread takes kRunUPT units kBlock apart (coalesced across the block),
// so only unit bits 8..11 (and, for complex64, amplitude bit 0) vary across a
// thread's amplitudes: factors that depend on none of those bits are
// evaluated once per thread, the others once per amplitude.
constexpr int kRunUPT = 16;

template <typename R>
__global__ void __launch_bounds__(kBlock) k_diag_run(R* __restrict__ psi, const DiagRunK<R> a)
{
    constexpr int AS = sizeof(R) == 4 ? 1 : 0;  // amplitude index = unit << AS
    const uint64_t vary = (sizeof(R) == 4 ? 1ull : 0ull) | ((uint64_t)(kRunUPT - 1) << (8 + AS));
    const uint64_t seglen = (uint64_t)kBlock * kRunUPT;
    const uint64_t nseg = (a.nunits + seglen - 1) / seglen;
    __shared__ R sd[2 * kMaxRunEntries];
    for (int k = threadIdx.x; k < 2 * a.ntab; k += kBlock)
        sd[k] = a.tab[k];
    __syncthreads();
    for (uint64_t seg = xcd_block(); seg < nseg; seg += gridDim.x) {
        const uint64_t u0 = seg * seglen + threadIdx.x;
        R cr = (R)1, ci = (R)0;
        for (int f = 0; f < a.nf; ++f)
            if (!(a.dep[f] & vary))
                run_factor(a, sd, f, u0 << AS, cr, ci);
        for (int r = 0; r < kRunUPT; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            if (u >= a.nunits)
                break;
            if constexpr (sizeof(R) == 4) {
                float4* p = reinterpret_cast<float4*>(psi);
                const float4 x = ld_nt(&p[u]);
                float ar = cr, ai = ci, br = cr, bi = ci;
                for (int f = 0; f < a.nf; ++f)
                    if (a.dep[f] & vary) {
                        run_factor(a, sd, f, u << 1, ar, ai);
                        run_factor(a, sd, f, (u << 1) | 1u, br, bi);
                    }
                st_nt(&p[u], make_float4(ar * x.x - ai * x.y, ar * x.y + ai * x.x, br * x.z - bi * x.w,
                                           br * x.w + bi * x.z));
            } else {
                double2* p = reinterpret_cast<double2*>(psi);
                const double2 x = ld_nt(&p[u]);
                double ar = cr, ai = ci;
                for (int f = 0; f < a.nf; ++f)
                    if (a.dep[f] & vary)
                        run_factor(a, sd, f, u, ar, ai);
                st_nt(&p[u], make_double2(ar * x.x - ai * x.y, ar * x.y + ai * x.x));
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
    DiagRunK<R> a{};
    a.nunits = L.ngroups;
    a.nf = L.run_nf;
    for (int f = 0; f < L.run_nf; ++f) {
        a.fix[f] = L.run_fix[f];
        a.val[f] = L.run_val[f];
        a.nt[f] = L.run_nt[f];
        a.off[f] = L.run_off[f];
        a.dep[f] = L.run_fix[f];
        for (int b = 0; b < L.run_nt[f]; ++b) {
            a.tpos[f][b] = L.run_tpos[f][b];
            a.dep[f] |= 1ull << L.run_tpos[f][b];
        }
    }
    a.tab = static_cast<const R*>(L.gdev);
    a.ntab = (int)(L.run_tab.size() / 2);
    if (!a.tab || a.ntab > kMaxRunEntries)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_diag_run<R>), dim3(run_grid(a.nunits)), dim3(kBlock), 0, s,
                       static_cast<R*>(p), a);
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
