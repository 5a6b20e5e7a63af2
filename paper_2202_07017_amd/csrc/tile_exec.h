// Device executor of tile programs (qsv_tileprog.h) on LDS-resident tiles.
//
// stage() copies a pass's steps into LDS and turns its gates into 2x2
// matrices (U for forward passes, U^dagger for reverse passes; rotations
// exp(-i theta P/2) read theta from the parameter vector).  exec_tile() runs
// the steps over a tile of 2^mb amplitudes: per step each thread takes groups
// of the tile (fixed values of the non-step qubits), holds the step's 2^nq
// amplitudes in registers, applies the step's gates in order (reverse passes:
// reverse order, and before each rotation's uncompute it adds
// Im <lambda|P psi> over the group to a per-thread partial), writes them
// back, and the block meets one barrier per step.  Per-gate partials are
// reduced in a fixed order (wave shuffle tree, then one thread over the
// waves) into per-slot FP64 accumulators in LDS.
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

// Run the staged pass over one LDS tile of 2^mb amplitudes (phi; REV: and lam).
template <typename R, bool REV>
__device__ void exec_tile(const LOp<R>* ops, const DStep* steps, int nsteps, int mb, R* phi, R* lam,
                          ExecShared& sh, int& parity)
{
    for (int si = 0; si < nsteps; ++si) {
        // Step and gate descriptors are the same for every lane; readfirstlane
        // keeps them in scalar registers so the guards below are scalar
        // branches rather than masked execution of every case.
        const DStep st = steps[REV ? nsteps - 1 - si : si];
        const int nq = __builtin_amdgcn_readfirstlane(st.nq);
        const int na = 1 << nq;
        const int o0 = __builtin_amdgcn_readfirstlane(st.o0);
        const int nop = __builtin_amdgcn_readfirstlane(st.o1) - o0;
        const int qp[3] = {__builtin_amdgcn_readfirstlane(st.q[0]),
                           __builtin_amdgcn_readfirstlane(st.q[1]),
                           __builtin_amdgcn_readfirstlane(st.q[2])};
        uint32_t off[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            uint32_t o = 0;
#pragma unroll
            for (int x = 0; x < 3; ++x)
                if (x < nq)
                    o |= ((uint32_t)(j >> x) & 1u) << qp[x];
            off[j] = o;
        }
        double acc[kMaxStepOps];
#pragma unroll
        for (int k = 0; k < kMaxStepOps; ++k)
            acc[k] = 0.0;
        const uint32_t ngroups = 1u << (mb - nq);
        for (uint32_t g = threadIdx.x; g < ngroups; g += blockDim.x) {
            uint32_t base = g;
#pragma unroll
            for (int x = 0; x < 3; ++x)
                if (x < nq) {
                    const uint32_t lo = (1u << qp[x]) - 1;
                    base = ((base & ~lo) << 1) | (base & lo);
                }
            R pr[8], pi[8], lr[8], li[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (j < na) {
                    pr[j] = phi[2 * (base + off[j])];
                    pi[j] = phi[2 * (base + off[j]) + 1];
                    if (REV) {
                        lr[j] = lam[2 * (base + off[j])];
                        li[j] = lam[2 * (base + off[j]) + 1];
                    }
                }
#pragma unroll
            for (int kk = 0; kk < kMaxStepOps; ++kk) {
                if (kk >= nop)
                    break;
                const int k = REV ? nop - 1 - kk : kk;
                const LOp<R>& o = ops[o0 + k];
                const int tb = 1 << __builtin_amdgcn_readfirstlane(o.tq);
                const int cm = __builtin_amdgcn_readfirstlane(o.cm);
                const int gen = __builtin_amdgcn_readfirstlane(o.gen);
#pragma unroll
                for (int u0 = 0; u0 < 8; ++u0) {
                    if (u0 >= na || (u0 & tb) || (u0 & cm) != cm)
                        continue;
                    const int u1 = u0 | tb;
                    if (REV) {
                        if (gen)
                            acc[kk] += gen_term(gen, (double)lr[u0], (double)li[u0], (double)lr[u1],
                                               (double)li[u1], (double)pr[u0], (double)pi[u0],
                                               (double)pr[u1], (double)pi[u1]);
                        apply2(o.m, lr[u0], li[u0], lr[u1], li[u1]);
                    }
                    apply2(o.m, pr[u0], pi[u0], pr[u1], pi[u1]);
                }
            }
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (j < na) {
                    phi[2 * (base + off[j])] = pr[j];
                    phi[2 * (base + off[j]) + 1] = pi[j];
                    if (REV) {
                        lam[2 * (base + off[j])] = lr[j];
                        lam[2 * (base + off[j]) + 1] = li[j];
                    }
                }
        }
        // acc[kk] belongs to the gate at position nop - 1 - kk (reverse passes)
        if (REV) {
#pragma unroll
            for (int kk = 0; kk < kMaxStepOps; ++kk) {
                if (kk >= nop)
                    break;
                if (__builtin_amdgcn_readfirstlane(ops[o0 + nop - 1 - kk].gen)) {
                    const double v = wave_sum(acc[kk]);
                    if ((threadIdx.x & 63) == 0)
                        sh.red[parity][kk][threadIdx.x >> 6] = v;
                }
            }
        }
        __syncthreads();
        if (REV) {
            const int kk = threadIdx.x;
            if (kk < nop && ops[o0 + nop - 1 - kk].gen) {
                double s = 0.0;
                for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
                    s += sh.red[parity][kk][w];
                sh.pacc[ops[o0 + nop - 1 - kk].slot] += s;
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
