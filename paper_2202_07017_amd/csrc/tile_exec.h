// Device executor of tile programs (qsv_tileprog.h) on LDS-resident tiles.
//
// stage() copies a pass's steps into LDS and turns its gates into 2x2
// matrices (U for forward passes, U^dagger for reverse passes; rotations
// exp(-i theta P/2) read theta from the parameter vector).  exec_tile() runs
// the steps over a tile of 2^mb amplitudes: per step each thread takes a fixed
// number of groups of the tile (fixed values of the non-step qubits), holds
// their amplitudes in registers, applies the step's gates in order (reverse
// passes: reverse order, and before each rotation's uncompute it adds
// Im <lambda|P psi> over its groups to a partial), writes them back, and the
// block meets one barrier per step.  Per-gate partials are reduced in a fixed
// order (wave shuffle tree, then one thread over the waves) into per-slot
// FP64 accumulators in LDS.
#pragma once

#include "qsv_internal.h"
#include "qsv_tileprog.h"

namespace qsv {
namespace tx {

template <typename R>
struct LOp {
    R m[8];       // 2x2 matrix, row-major (re, im)
    uint8_t tq;   // target position in the step
    uint8_t cm;   // control mask over the step's qubits
    int8_t gen;   // rotation generator 5 / 6 / 7 (X / Y / Z); 0 = fixed gate
    int8_t pad;
    int16_t slot; // rotation slot inside the pass
    int16_t pad2;
};

struct ExecShared {
    double red[2][kMaxStepOps][16];  // per-wave partials, double-buffered by step parity
    double pacc[kMaxPassOps];        // per-slot sums over the tiles of the pass
};

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// 2x2 matrix of a gate in FP64 (dag: conjugate transpose).
__device__ __forceinline__ void gate_matrix(const DOp& d, const double* mats, const double* params,
                                            bool dag, double* m)
{
    if (d.kind == 0) {
        for (int j = 0; j < 8; ++j)
            m[j] = mats[(size_t)d.mat * 8 + j];
    } else {
        const double th = params[d.param];
        const double c = cos(0.5 * th), s = sin(0.5 * th);
        for (int j = 0; j < 8; ++j)
            m[j] = 0.0;
        m[0] = c;
        m[6] = c;
        if (d.kind == 5) {  // RX = [[c, -is], [-is, c]]
            m[3] = -s;
            m[5] = -s;
        } else if (d.kind == 6) {  // RY = [[c, -s], [s, c]]
            m[2] = -s;
            m[4] = s;
        } else {  // RZ = diag(c - is, c + is)
            m[1] = -s;
            m[7] = s;
        }
    }
    if (dag) {
        const double t2 = m[2], t3 = m[3];
        m[1] = -m[1];
        m[2] = m[4];
        m[3] = -m[5];
        m[4] = t2;
        m[5] = -t3;
        m[7] = -m[7];
    }
}

template <typename R>
__device__ void stage(const DPass& P, const DStep* steps, const DOp* ops, const double* mats,
                      const double* params, bool dag, LOp<R>* lops, DStep* lsteps, ExecShared& sh)
{
    for (int j = threadIdx.x; j < P.nops; j += blockDim.x) {
        const DOp d = ops[P.op_off + j];
        double m[8];
        gate_matrix(d, mats, params, dag, m);
        LOp<R> o;
        for (int q = 0; q < 8; ++q)
            o.m[q] = (R)m[q];
        o.tq = d.tq;
        o.cm = d.cm;
        o.gen = (int8_t)(d.kind == 0 ? 0 : d.kind);
        o.pad = 0;
        o.slot = (int16_t)d.slot;
        o.pad2 = 0;
        lops[j] = o;
    }
    for (int j = threadIdx.x; j < P.nsteps; j += blockDim.x)
        lsteps[j] = steps[P.step_off + j];
    for (int j = threadIdx.x; j < P.nrot; j += blockDim.x)
        sh.pacc[j] = 0.0;
}

// Im <l|P v> over one pair (l0, l1), (v0, v1) for P = X (5), Y (6), Z (7).
__device__ __forceinline__ double gen_term(int gen, double l0r, double l0i, double l1r, double l1i,
                                           double v0r, double v0i, double v1r, double v1i)
{
    if (gen == 5)
        return (l0r * v1i - l0i * v1r) + (l1r * v0i - l1i * v0r);
    if (gen == 6)
        return -(l0r * v1r + l0i * v1i) + (l1r * v0r + l1i * v0i);
    return (l0r * v0i - l0i * v0r) - (l1r * v1i - l1i * v1r);
}

template <typename R>
__device__ __forceinline__ void apply2(const R* m, R& ar, R& ai, R& br, R& bi)
{
    const R xr = ar, xi = ai, yr = br, yi = bi;
    ar = m[0] * xr - m[1] * xi + m[2] * yr - m[3] * yi;
    ai = m[0] * xi + m[1] * xr + m[2] * yi + m[3] * yr;
    br = m[4] * xr - m[5] * xi + m[6] * yr - m[7] * yi;
    bi = m[4] * xi + m[5] * xr + m[6] * yi + m[7] * yr;
}

// Apply one gate (target at step position TQ, controls cm over the step's
// qubits) to every group a thread holds: GP groups of 2^NQ amplitudes stored
// at [gi * 2^NQ + u].  All register indices are compile-time constants.
template <typename R, bool REV, int NQ, int TQ, int GP>
__device__ __forceinline__ void gate_pairs(const R* m, int cm, int gen, R* pr, R* pi, R* lr, R* li,
                                           double& acc)
{
    constexpr int NA = 1 << NQ;
    constexpr int TB = 1 << TQ;
#pragma unroll
    for (int gi = 0; gi < GP; ++gi)
#pragma unroll
        for (int p = 0; p < NA / 2; ++p) {
            const int u0 = ((p >> TQ) << (TQ + 1)) | (p & (TB - 1));
            const int u1 = u0 | TB;
            if ((u0 & cm) != cm)
                continue;
            const int a = gi * NA + u0, b = gi * NA + u1;
            if (REV) {
                if (gen)
                    acc += gen_term(gen, (double)lr[a], (double)li[a], (double)lr[b], (double)li[b],
                                    (double)pr[a], (double)pi[a], (double)pr[b], (double)pi[b]);
                apply2(m, lr[a], li[a], lr[b], li[b]);
            }
            apply2(m, pr[a], pi[a], pr[b], pi[b]);
        }
}

// One step on NQ qubits: each active thread holds APT amplitudes (APT / 2^NQ
// groups), applies the step's gates in order (reverse: in reverse order), and
// the per-gate gradient partials go straight to LDS after a wave reduction.
template <typename R, bool REV, int NQ, int APT>
__device__ void exec_step(const LOp<R>* ops, int o0, int nop, int q0, int q1, int q2, int mb,
                          R* phi, R* lam, ExecShared& sh, int parity)
{
    constexpr int NA = 1 << NQ;
    constexpr int GP = APT / NA;
    const uint32_t nthr = (1u << mb) / APT;  // threads holding amplitudes
    const bool active = threadIdx.x < nthr;
    const int qp[3] = {q0, q1, q2};
    uint32_t off[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) {
        uint32_t o = 0;
#pragma unroll
        for (int x = 0; x < NQ; ++x)
            o |= ((uint32_t)(j >> x) & 1u) << qp[x];
        off[j] = o;
    }
    R pr[APT], pi[APT], lr[REV ? APT : 1], li[REV ? APT : 1];
    uint32_t base[GP];
    if (active) {
#pragma unroll
        for (int gi = 0; gi < GP; ++gi) {
            uint32_t b = gi * nthr + threadIdx.x;
#pragma unroll
            for (int x = 0; x < NQ; ++x) {
                const uint32_t lo = (1u << qp[x]) - 1;
                b = ((b & ~lo) << 1) | (b & lo);
            }
            base[gi] = b;
#pragma unroll
            for (int j = 0; j < NA; ++j) {
                pr[gi * NA + j] = phi[2 * (b + off[j])];
                pi[gi * NA + j] = phi[2 * (b + off[j]) + 1];
                if (REV) {
                    lr[gi * NA + j] = lam[2 * (b + off[j])];
                    li[gi * NA + j] = lam[2 * (b + off[j]) + 1];
                }
            }
        }
    }
    for (int k = 0; k < nop; ++k) {
        const int kk = REV ? nop - 1 - k : k;
        const LOp<R>& o = ops[o0 + kk];
        const int tq = __builtin_amdgcn_readfirstlane(o.tq);
        const int cm = __builtin_amdgcn_readfirstlane(o.cm);
        const int gen = REV ? __builtin_amdgcn_readfirstlane(o.gen) : 0;
        R m[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            m[q] = o.m[q];
        double acc = 0.0;
        if (active) {
            if (tq == 0)
                gate_pairs<R, REV, NQ, 0, GP>(m, cm, gen, pr, pi, lr, li, acc);
            else if (NQ > 1 && tq == 1)
                gate_pairs<R, REV, NQ, (NQ > 1 ? 1 : 0), GP>(m, cm, gen, pr, pi, lr, li, acc);
            else if (NQ > 2)
                gate_pairs<R, REV, NQ, (NQ > 2 ? 2 : 0), GP>(m, cm, gen, pr, pi, lr, li, acc);
        }
        if (REV && gen) {
            acc = wave_sum(acc);
            if ((threadIdx.x & 63) == 0)
                sh.red[parity][kk][threadIdx.x >> 6] = acc;
        }
    }
    if (active) {
#pragma unroll
        for (int gi = 0; gi < GP; ++gi)
#pragma unroll
            for (int j = 0; j < NA; ++j) {
                const uint32_t b = base[gi];
                phi[2 * (b + off[j])] = pr[gi * NA + j];
                phi[2 * (b + off[j]) + 1] = pi[gi * NA + j];
                if (REV) {
                    lam[2 * (b + off[j])] = lr[gi * NA + j];
                    lam[2 * (b + off[j]) + 1] = li[gi * NA + j];
                }
            }
    }
}

// Run the staged pass over one LDS tile of 2^mb amplitudes (phi; REV: and
// lam).  APT amplitudes per thread: the block needs 2^mb / APT threads
// (mb >= log2(APT)); extra threads only take part in the barriers.
template <typename R, bool REV, int APT>
__device__ void exec_tile(const LOp<R>* ops, const DStep* steps, int nsteps, int mb, R* phi, R* lam,
                          ExecShared& sh, int& parity)
{
    for (int si = 0; si < nsteps; ++si) {
        // Step and gate descriptors are the same for every lane; readfirstlane
        // keeps them in scalar registers.
        const DStep st = steps[REV ? nsteps - 1 - si : si];
        const int nq = __builtin_amdgcn_readfirstlane(st.nq);
        const int o0 = __builtin_amdgcn_readfirstlane(st.o0);
        const int nop = __builtin_amdgcn_readfirstlane(st.o1) - o0;
        const int q0 = __builtin_amdgcn_readfirstlane(st.q[0]);
        const int q1 = __builtin_amdgcn_readfirstlane(st.q[1]);
        const int q2 = __builtin_amdgcn_readfirstlane(st.q[2]);
        if (nq == 1)
            exec_step<R, REV, 1, APT>(ops, o0, nop, q0, q1, q2, mb, phi, lam, sh, parity);
        else if (nq == 2)
            exec_step<R, REV, 2, APT>(ops, o0, nop, q0, q1, q2, mb, phi, lam, sh, parity);
        else
            exec_step<R, REV, 3, APT>(ops, o0, nop, q0, q1, q2, mb, phi, lam, sh, parity);
        __syncthreads();
        if (REV) {
            const int kk = threadIdx.x;
            if (kk < nop && ops[o0 + kk].gen) {
                double s = 0.0;
                for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
                    s += sh.red[parity][kk][w];
                sh.pacc[ops[o0 + kk].slot] += s;
            }
            parity ^= 1;
        }
    }
}

// Tile loading: local amplitude l of tile `base` is global base | deposit(l, B).
__device__ __forceinline__ uint64_t deposit_mask(uint64_t l, uint64_t mask)
{
    uint64_t out = 0;
    int b = 0;
    for (uint64_t m = mask; m; m &= m - 1, ++b)
        if ((l >> b) & 1ull)
            out |= m & (~m + 1);
    return out;
}

__device__ __forceinline__ uint64_t insert_mask(uint64_t t, uint64_t mask)
{
    for (uint64_t m = mask; m; m &= m - 1) {
        const uint64_t lo = (m & (~m + 1)) - 1;
        t = ((t & ~lo) << 1) | (t & lo);
    }
    return t;
}

}  // namespace tx
}  // namespace qsv
