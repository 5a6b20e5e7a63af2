// Device executor of tile programs (qsv_tileprog.h) on LDS-resident tiles.
//
// make_lop() turns a gate into its 2x2 matrix (U for forward passes, U^dagger
// for reverse passes; rotations exp(-i theta P/2) read theta from the
// parameter vector) and classifies the matrix into a form (swap, diagonal,
// real, ...) that the executor applies with the fewest operations.  stage()
// does this for a pass into LDS (batched mode); the single-state passes read
// descriptors staged once per run in global memory, through scalar loads.
// exec_tile() runs the steps over a tile of 2^mb amplitudes: per step (three
// qubits) each thread takes a fixed number of groups of the tile (fixed
// values of the non-step qubits), holds their amplitudes in registers,
// applies the step's gates in order (reverse passes: reverse order, and
// before each rotation's uncompute it adds Im <lambda|P psi> over its groups
// to a partial), writes them back, and the block meets one barrier per step.
// Per-gate partials are reduced in a fixed order (wave reduction, then one
// thread over the waves) into per-slot FP64 accumulators in LDS.
#pragma once

#include "qsv_internal.h"
#include "qsv_tileprog.h"

namespace qsv {
namespace tx {

// Matrix forms, each applied with its own arithmetic (per amplitude pair:
// general 16 multiply-adds, diagonal 8, real 8, real diagonal 4, swap none).
enum : int {
    kFormGeneral = 0,   // any complex 2x2
    kFormSwap = 1,      // [[0, 1], [1, 0]]: X, and with controls CNOT, Toffoli
    kFormDiag = 2,      // diag(d0, d1): RZ, S, T, phase gates
    kFormRealDiag = 3,  // real diag(d0, d1): Z, CZ (on its target)
    kFormReal = 4,      // real entries: RY, H
    kFormOffImag = 5,   // real diagonal, imaginary off-diagonal: RX, Y
};

// A gate as the executor reads it.  The small fields share one 32-bit word,
// so a uniform descriptor is two scalar loads (matrix, word).
template <typename R>
struct LOp {
    R m[8];         // 2x2 matrix, row-major (re, im)
    uint32_t info;  // target position in the step (bits 0-7), control mask over
                    // the step's qubits (8-15), rotation generator 5 / 6 / 7
                    // = X / Y / Z or 0 for a fixed gate (16-23), kForm* (24-31)
    int32_t slot;   // rotation slot inside the pass
};

__device__ __forceinline__ int lop_tq(uint32_t info)
{
    return info & 0xff;
}
__device__ __forceinline__ int lop_cm(uint32_t info)
{
    return (info >> 8) & 0xff;
}
__device__ __forceinline__ int lop_gen(uint32_t info)
{
    return (info >> 16) & 0xff;
}
__device__ __forceinline__ int lop_form(uint32_t info)
{
    return info >> 24;
}

struct ExecShared {
    double red[2][kMaxStepOps][16];  // per-wave partials, double-buffered by step parity
};

// One DPP move of a double across lanes (CTRL: a DPP control word).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int lane)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Sum over the 64 lanes of a wave, the same value in every lane: rows of 16
// lanes reduce through DPP (quad swaps, then rotations by 4 and 8 inside the
// row), then the four row sums are added in a fixed order.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_move<0xb1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4e>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x124>(v);  // row_ror 4
    v += dpp_move<0x128>(v);  // row_ror 8
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
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

__device__ __forceinline__ int gate_form(const double* m)
{
    const bool offdiag0 = m[2] == 0.0 && m[3] == 0.0 && m[4] == 0.0 && m[5] == 0.0;
    const bool realdiag = m[1] == 0.0 && m[7] == 0.0;
    if (m[0] == 0.0 && realdiag && m[6] == 0.0 && m[2] == 1.0 && m[3] == 0.0 && m[4] == 1.0 &&
        m[5] == 0.0)
        return kFormSwap;
    if (offdiag0)
        return realdiag ? kFormRealDiag : kFormDiag;
    if (realdiag && m[3] == 0.0 && m[5] == 0.0)
        return kFormReal;
    if (realdiag && m[2] == 0.0 && m[4] == 0.0)
        return kFormOffImag;
    return kFormGeneral;
}

template <typename R>
__device__ __forceinline__ LOp<R> make_lop(const DOp& d, const double* mats, const double* params,
                                           bool dag)
{
    double m[8];
    gate_matrix(d, mats, params, dag, m);
    LOp<R> o;
    for (int q = 0; q < 8; ++q)
        o.m[q] = (R)m[q];
    const uint32_t gen = d.kind == 0 ? 0u : (uint32_t)d.kind;
    o.info = (uint32_t)d.tq | ((uint32_t)d.cm << 8) | (gen << 16) | ((uint32_t)gate_form(m) << 24);
    o.slot = d.slot;
    return o;
}

// Stage a pass into LDS: its gates (as LOp), its steps, zeroed slot sums.
template <typename R>
__device__ void stage(const DPass& P, const DStep* steps, const DOp* ops, const double* mats,
                      const double* params, bool dag, LOp<R>* lops, DStep* lsteps, double* pacc)
{
    for (int j = threadIdx.x; j < P.nops; j += blockDim.x)
        lops[j] = make_lop<R>(ops[P.op_off + j], mats, params, dag);
    for (int j = threadIdx.x; j < P.nsteps; j += blockDim.x)
        lsteps[j] = steps[P.step_off + j];
    for (int j = threadIdx.x; j < P.nrot; j += blockDim.x)
        pacc[j] = 0.0;
}

// Im <l|P v> over one pair (l0, l1), (v0, v1) for P = X (5), Y (6), Z (7),
// in the state's precision (the caller sums it in FP64).
template <int GEN, typename R>
__device__ __forceinline__ R gen_term(R l0r, R l0i, R l1r, R l1i, R v0r, R v0i, R v1r, R v1i)
{
    if constexpr (GEN == 5)
        return (l0r * v1i - l0i * v1r) + (l1r * v0i - l1i * v0r);
    else if constexpr (GEN == 6)
        return (l1r * v0r + l1i * v0i) - (l0r * v1r + l0i * v1i);
    else
        return (l0r * v0i - l0i * v0r) - (l1r * v1i - l1i * v1r);
}

// (a, b) <- G (a, b) for a matrix of form F (row-major re, im entries m).
template <int F, typename R>
__device__ __forceinline__ void apply_form(const R* m, R& ar, R& ai, R& br, R& bi)
{
    const R xr = ar, xi = ai, yr = br, yi = bi;
    if constexpr (F == kFormSwap) {
        ar = yr;
        ai = yi;
        br = xr;
        bi = xi;
    } else if constexpr (F == kFormDiag) {
        ar = m[0] * xr - m[1] * xi;
        ai = m[0] * xi + m[1] * xr;
        br = m[6] * yr - m[7] * yi;
        bi = m[6] * yi + m[7] * yr;
    } else if constexpr (F == kFormRealDiag) {
        ar = m[0] * xr;
        ai = m[0] * xi;
        br = m[6] * yr;
        bi = m[6] * yi;
    } else if constexpr (F == kFormReal) {
        ar = m[0] * xr + m[2] * yr;
        ai = m[0] * xi + m[2] * yi;
        br = m[4] * xr + m[6] * yr;
        bi = m[4] * xi + m[6] * yi;
    } else if constexpr (F == kFormOffImag) {
        ar = m[0] * xr - m[3] * yi;
        ai = m[0] * xi + m[3] * yr;
        br = m[6] * yr - m[5] * xi;
        bi = m[6] * yi + m[5] * xr;
    } else {
        ar = m[0] * xr - m[1] * xi + m[2] * yr - m[3] * yi;
        ai = m[0] * xi + m[1] * xr + m[2] * yi + m[3] * yr;
        br = m[4] * xr - m[5] * xi + m[6] * yr - m[7] * yi;
        bi = m[4] * xi + m[5] * xr + m[6] * yi + m[7] * yr;
    }
}

// Steps always span three qubits (the host pads them), so a thread holds
// GP = APT / 8 groups of 8 amplitudes, group gi at registers [gi * 8 + u].
constexpr int kNA = 8;

// Apply one gate of form F (target at step position TQ, controls CM over the
// step's qubits) to every group a thread holds; reverse passes also apply it
// to lambda and, for a rotation (GEN != 0), first sum its generator term.
// All register indices are compile-time constants.
template <typename R, bool REV, int TQ, int CM, int GP, int F, int GEN>
__device__ __forceinline__ void gate_pairs(const R* m, R* pr, R* pi, R* lr, R* li, double& acc)
{
    constexpr int TB = 1 << TQ;
    R t = 0;
#pragma unroll
    for (int gi = 0; gi < GP; ++gi)
#pragma unroll
        for (int p = 0; p < kNA / 2; ++p) {
            const int u0 = ((p >> TQ) << (TQ + 1)) | (p & (TB - 1));
            const int u1 = u0 | TB;
            if ((u0 & CM) != CM)
                continue;
            const int a = gi * kNA + u0, b = gi * kNA + u1;
            if constexpr (REV) {
                if constexpr (GEN != 0)
                    t += gen_term<GEN, R>(lr[a], li[a], lr[b], li[b], pr[a], pi[a], pr[b], pi[b]);
                apply_form<F>(m, lr[a], li[a], lr[b], li[b]);
            }
            apply_form<F>(m, pr[a], pi[a], pr[b], pi[b]);
        }
    if constexpr (GEN != 0)
        acc = (double)t;
}

// Dispatch on the gate: reverse-pass rotations by generator (the form of
// U^dagger follows from it), everything else by form.
template <typename R, bool REV, int TQ, int CM, int GP>
__device__ __forceinline__ void apply_op(int form, int gen, const R* m, R* pr, R* pi, R* lr, R* li,
                                         double& acc)
{
    if (REV && gen == 5)
        gate_pairs<R, REV, TQ, CM, GP, kFormOffImag, 5>(m, pr, pi, lr, li, acc);
    else if (REV && gen == 6)
        gate_pairs<R, REV, TQ, CM, GP, kFormReal, 6>(m, pr, pi, lr, li, acc);
    else if (REV && gen == 7)
        gate_pairs<R, REV, TQ, CM, GP, kFormDiag, 7>(m, pr, pi, lr, li, acc);
    else if (form == kFormSwap)
        gate_pairs<R, REV, TQ, CM, GP, kFormSwap, 0>(m, pr, pi, lr, li, acc);
    else if (form == kFormDiag)
        gate_pairs<R, REV, TQ, CM, GP, kFormDiag, 0>(m, pr, pi, lr, li, acc);
    else if (form == kFormRealDiag)
        gate_pairs<R, REV, TQ, CM, GP, kFormRealDiag, 0>(m, pr, pi, lr, li, acc);
    else if (form == kFormReal)
        gate_pairs<R, REV, TQ, CM, GP, kFormReal, 0>(m, pr, pi, lr, li, acc);
    else if (form == kFormOffImag)
        gate_pairs<R, REV, TQ, CM, GP, kFormOffImag, 0>(m, pr, pi, lr, li, acc);
    else
        gate_pairs<R, REV, TQ, CM, GP, kFormGeneral, 0>(m, pr, pi, lr, li, acc);
}

// ... and on the control mask, a subset of the two non-target step qubits.
template <typename R, bool REV, int TQ, int GP>
__device__ __forceinline__ void apply_tq(int cm, int form, int gen, const R* m, R* pr, R* pi,
                                         R* lr, R* li, double& acc)
{
    constexpr int A = TQ == 0 ? 2 : 1;
    constexpr int B = TQ == 2 ? 2 : 4;
    if (cm == 0)
        apply_op<R, REV, TQ, 0, GP>(form, gen, m, pr, pi, lr, li, acc);
    else if (cm == A)
        apply_op<R, REV, TQ, A, GP>(form, gen, m, pr, pi, lr, li, acc);
    else if (cm == B)
        apply_op<R, REV, TQ, B, GP>(form, gen, m, pr, pi, lr, li, acc);
    else
        apply_op<R, REV, TQ, A | B, GP>(form, gen, m, pr, pi, lr, li, acc);
}

template <typename R, bool REV, int GP>
__device__ __forceinline__ void apply_gate(int tq, int cm, int form, int gen, const R* m, R* pr,
                                           R* pi, R* lr, R* li, double& acc)
{
    if (tq == 0)
        apply_tq<R, REV, 0, GP>(cm, form, gen, m, pr, pi, lr, li, acc);
    else if (tq == 1)
        apply_tq<R, REV, 1, GP>(cm, form, gen, m, pr, pi, lr, li, acc);
    else
        apply_tq<R, REV, 2, GP>(cm, form, gen, m, pr, pi, lr, li, acc);
}

// One step on three qubits q0 < q1 < q2: each active thread holds APT
// amplitudes (APT / 8 groups), applies the step's gates in order (reverse:
// in reverse order), and the per-gate gradient partials go to LDS after a
// wave reduction.  `ops` may point to LDS or to global memory; the gate
// descriptors are the same for every lane.
template <typename R, bool REV, int APT, bool PAIR2>
__device__ __forceinline__ void exec_step(const LOp<R>* ops, int o0, int nop, int q0, int q1,
                                          int q2, int mb, R* phi, R* lam, ExecShared& sh,
                                          int parity)
{
    constexpr int GP = APT / kNA;
    const uint32_t nthr = (1u << mb) / APT;  // threads holding amplitudes
    const bool active = threadIdx.x < nthr;
    const int qp[3] = {q0, q1, q2};
    uint32_t off[kNA];
#pragma unroll
    for (int j = 0; j < kNA; ++j)
        off[j] = ((uint32_t)(j & 1) << q0) | ((uint32_t)((j >> 1) & 1) << q1) |
                 ((uint32_t)((j >> 2) & 1) << q2);
    // (threads without amplitudes run the gates on zeros: no predicate per
    // gate, and their generator terms are zero)
    R pr[APT], pi[APT], lr[REV ? APT : 1], li[REV ? APT : 1];
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        pr[j] = pi[j] = R(0);
        if (REV)
            lr[j] = li[j] = R(0);
    }
    uint32_t base[GP];
    if (active) {
#pragma unroll
        for (int gi = 0; gi < GP; ++gi) {
            uint32_t b = gi * nthr + threadIdx.x;
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                const uint32_t lo = (1u << qp[x]) - 1;
                b = ((b & ~lo) << 1) | (b & lo);
            }
            base[gi] = b;
#pragma unroll
            for (int j = 0; j < kNA; ++j) {
                pr[gi * kNA + j] = phi[2 * (b + off[j])];
                pi[gi * kNA + j] = phi[2 * (b + off[j]) + 1];
                if (REV) {
                    lr[gi * kNA + j] = lam[2 * (b + off[j])];
                    li[gi * kNA + j] = lam[2 * (b + off[j]) + 1];
                }
            }
        }
    }
    auto one = [&](int k) __attribute__((always_inline)) {
        const int kk = REV ? nop - 1 - k : k;
        const LOp<R>& o = ops[o0 + kk];
        const uint32_t info = __builtin_amdgcn_readfirstlane(o.info);
        const int gen = REV ? lop_gen(info) : 0;
        R m[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            m[q] = o.m[q];
        double acc = 0.0;
        apply_gate<R, REV, GP>(lop_tq(info), lop_cm(info), lop_form(info), gen, m, pr, pi, lr, li,
                               acc);
        if (REV && gen) {
            acc = wave_sum(acc);
            if ((threadIdx.x & 63) == 0)
                sh.red[parity][kk][threadIdx.x >> 6] = acc;
        }
    };
    // Two gates per iteration: the register allocator then alternates
    // between two sets of amplitude registers instead of copying the results
    // back after every gate (forward passes 12-14% faster, reverse passes of
    // the single-state kernel 3-4%).  PAIR2 = false keeps one gate per
    // iteration for reverse passes where registers are short (the batched
    // kernel would spill).
    if (REV && !PAIR2) {
        for (int k = 0; k < nop; ++k)
            one(k);
    } else {
        for (int k = 0; k < nop; k += 2) {
            one(k);
            if (k + 1 < nop)
                one(k + 1);
        }
    }
    if (active) {
#pragma unroll
        for (int gi = 0; gi < GP; ++gi)
#pragma unroll
            for (int j = 0; j < kNA; ++j) {
                const uint32_t b = base[gi];
                phi[2 * (b + off[j])] = pr[gi * kNA + j];
                phi[2 * (b + off[j]) + 1] = pi[gi * kNA + j];
                if (REV) {
                    lam[2 * (b + off[j])] = lr[gi * kNA + j];
                    lam[2 * (b + off[j]) + 1] = li[gi * kNA + j];
                }
            }
    }
}

// Run a pass over one LDS tile of 2^mb amplitudes (phi; REV: and lam).  APT
// amplitudes per thread: the block needs 2^mb / APT threads (mb >= 3 and
// 2^mb >= APT); extra threads only take part in the barriers.  `ops` and
// `steps` point to the pass's first gate and step (LDS or global memory);
// reverse passes add each rotation's sum to pacc[slot] (LDS).
template <typename R, bool REV, int APT, bool PAIR2 = false>
__device__ __forceinline__ void exec_tile(const LOp<R>* ops, const DStep* steps, int nsteps, int mb,
                                          R* phi, R* lam, ExecShared& sh, double* pacc, int& parity)
{
    for (int si = 0; si < nsteps; ++si) {
        // Step and gate descriptors are the same for every lane; readfirstlane
        // keeps them in scalar registers.
        // (read as two words: byte fields would need vector loads)
        const uint2 sw = reinterpret_cast<const uint2*>(steps)[REV ? nsteps - 1 - si : si];
        const uint32_t w0 = __builtin_amdgcn_readfirstlane(sw.x);
        const uint32_t w1 = __builtin_amdgcn_readfirstlane(sw.y);
        const int q0 = (w0 >> 8) & 0xff, q1 = (w0 >> 16) & 0xff, q2 = w0 >> 24;
        const int o0 = (int16_t)(w1 & 0xffff);
        const int nop = (int16_t)(w1 >> 16) - o0;
        exec_step<R, REV, APT, PAIR2>(ops, o0, nop, q0, q1, q2, mb, phi, lam, sh, parity);
        __syncthreads();
        if (REV) {
            const int kk = threadIdx.x;
            if (kk < nop && lop_gen(ops[o0 + kk].info)) {
                double s = 0.0;
                for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
                    s += sh.red[parity][kk][w];
                pacc[ops[o0 + kk].slot] += s;
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
