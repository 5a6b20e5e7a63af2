// Circuits: the fusion planner, plans (launch lists replayed through HIP
// graphs) and the adjoint-gradient driver.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <set>
#include <vector>

#include "qsv.h"
#include "qsv_fuse_plan.h"
#include "qsv_host.h"
#include "qsv_qperm_plan.h"
#include "qsv_internal.h"
#include "qsv_tileprog.h"
#include "qsv_tpass.h"

using namespace qsv;

namespace qsv {

// ------------------------------------------------------------ op matrices

// Matrix of a non-rotation kind, or of a rotation at angle theta (2x2 or 4x4,
// row-major complex128, user target order).
std::vector<double> op_matrix(const qsv_op& op, double theta)
{
    const double r2 = 1.0 / std::sqrt(2.0);
    const double c = std::cos(0.5 * theta), s = std::sin(0.5 * theta);
    switch (op.kind) {
    case QSV_OP_H: return {r2, 0, r2, 0, r2, 0, -r2, 0};
    case QSV_OP_X: return {0, 0, 1, 0, 1, 0, 0, 0};
    case QSV_OP_Y: return {0, 0, 0, -1, 0, 1, 0, 0};
    case QSV_OP_Z: return {1, 0, 0, 0, 0, 0, -1, 0};
    case QSV_OP_RX: return {c, 0, 0, -s, 0, -s, c, 0};
    case QSV_OP_RY: return {c, 0, -s, 0, s, 0, c, 0};
    case QSV_OP_RZ: return {c, -s, 0, 0, 0, 0, c, s};
    case QSV_OP_SWAP: {
        std::vector<double> m(32, 0.0);
        m[0] = 1;                 // |00> -> |00>
        m[(1 * 4 + 2) * 2] = 1;   // row 1 <- col 2
        m[(2 * 4 + 1) * 2] = 1;   // row 2 <- col 1
        m[(3 * 4 + 3) * 2] = 1;
        return m;
    }
    default: {
        const int D = 1 << op.k;
        return std::vector<double>(op.M, op.M + (size_t)2 * D * D);
    }
    }
}

qsv_status check_circuit(const qsv_circuit* C, int max_n)
{
    if (!C || (C->nops > 0 && !C->ops) || C->nops < 0)
        return fail(QSV_ERR_ARG, "circuit is NULL or has a NULL op list");
    if (C->n < 1 || C->n > max_n)
        return fail(QSV_ERR_ARG, "circuit n = %d outside [1, %d]", C->n, max_n);
    if (C->nparams < 0)
        return fail(QSV_ERR_ARG, "negative nparams");
    for (int o = 0; o < C->nops; ++o) {
        const qsv_op& op = C->ops[o];
        if (op.kind < QSV_OP_MATRIX || op.kind > QSV_OP_SWAP)
            return fail(QSV_ERR_ARG, "op %d: unknown kind %d", o, op.kind);
        if (op.c < 0 || op.c > QSV_MAX_CONTROLS)
            return fail(QSV_ERR_ARG, "op %d: control count %d outside [0, %d]", o, op.c,
                        QSV_MAX_CONTROLS);
        const int kneed = op.kind == QSV_OP_SWAP ? 2 : (op.kind == QSV_OP_MATRIX ? -1 : 1);
        if (kneed > 0 && op.k != kneed)
            return fail(QSV_ERR_ARG, "op %d: kind %d needs k = %d, got %d", o, op.kind, kneed, op.k);
        qsv_status st = check_qubits(C->n, op.targets, op.k, QSV_MAX_TARGETS, op.controls, op.c);
        if (st)
            return fail(st, "op %d: %s", o, qsv_last_error());
        if (op.kind == QSV_OP_MATRIX && !op.M)
            return fail(QSV_ERR_ARG, "op %d: MATRIX op with NULL M", o);
        if (is_rotation(op.kind) && (op.param < 0 || op.param >= C->nparams))
            return fail(QSV_ERR_ARG, "op %d: parameter index %d outside [0, %d)", o, op.param,
                        C->nparams);
    }
    return QSV_OK;
}

// ------------------------------------------------------------ the planner

// Matrix of `op` embedded in the block on ascending qubits qs (bit j <-> qs[j]).
static std::vector<double> embed(const qsv_op& op, const std::vector<double>& G,
                                 const std::vector<int>& qs)
{
    const int m = (int)qs.size(), Dm = 1 << m, k = op.k, D = 1 << k;
    auto pos = [&](int q) { return (int)(std::find(qs.begin(), qs.end(), q) - qs.begin()); };
    std::vector<double> E((size_t)2 * Dm * Dm, 0.0);
    int tp[QSV_MAX_TARGETS], cp[QSV_MAX_CONTROLS];
    for (int i = 0; i < k; ++i)
        tp[i] = pos(op.targets[i]);
    for (int i = 0; i < op.c; ++i)
        cp[i] = pos(op.controls[i]);
    for (int b = 0; b < Dm; ++b) {
        bool on = true;
        for (int i = 0; i < op.c; ++i)
            on = on && ((b >> cp[i]) & 1);
        if (!on) {
            E[((size_t)b * Dm + b) * 2] = 1.0;
            continue;
        }
        int tin = 0, cleared = b;
        for (int i = 0; i < k; ++i) {
            tin |= ((b >> tp[i]) & 1) << (k - 1 - i);
            cleared &= ~(1 << tp[i]);
        }
        for (int tau = 0; tau < D; ++tau) {
            int r = cleared;
            for (int i = 0; i < k; ++i)
                r |= ((tau >> (k - 1 - i)) & 1) << tp[i];
            E[((size_t)r * Dm + b) * 2] = G[((size_t)tau * D + tin) * 2];
            E[((size_t)r * Dm + b) * 2 + 1] = G[((size_t)tau * D + tin) * 2 + 1];
        }
    }
    return E;
}

static std::vector<double> matmul(const std::vector<double>& A, const std::vector<double>& B, int D)
{
    std::vector<double> C((size_t)2 * D * D, 0.0);
    for (int i = 0; i < D; ++i)
        for (int k = 0; k < D; ++k) {
            const double ar = A[((size_t)i * D + k) * 2], ai = A[((size_t)i * D + k) * 2 + 1];
            if (ar == 0.0 && ai == 0.0)
                continue;
            for (int j = 0; j < D; ++j) {
                const double br = B[((size_t)k * D + j) * 2], bi = B[((size_t)k * D + j) * 2 + 1];
                C[((size_t)i * D + j) * 2] += ar * br - ai * bi;
                C[((size_t)i * D + j) * 2 + 1] += ar * bi + ai * br;
            }
        }
    return C;
}

static std::vector<double> dagger(const std::vector<double>& A, int D)
{
    std::vector<double> B(A.size());
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) {
            B[((size_t)i * D + j) * 2] = A[((size_t)j * D + i) * 2];
            B[((size_t)i * D + j) * 2 + 1] = -A[((size_t)j * D + i) * 2 + 1];
        }
    return B;
}

static bool is_unitary(const std::vector<double>& A, int D)
{
    std::vector<double> P = matmul(A, dagger(A, D), D);
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) {
            const double re = P[((size_t)i * D + j) * 2] - (i == j ? 1.0 : 0.0);
            const double im = P[((size_t)i * D + j) * 2 + 1];
            if (std::fabs(re) > 1e-9 || std::fabs(im) > 1e-9)
                return false;
        }
    return true;
}

// Launch for an item (block or native op) with host-known matrices.
// dag: build the launch for the conjugate transpose.
static Built item_launch(const qsv_circuit* C, const Item& it, int dt, const double* params_host,
                         bool dag)
{
    auto theta = [&](const qsv_op& op) {
        return is_rotation(op.kind) && params_host ? params_host[op.param] : 0.0;
    };
    if (it.ops.size() == 1) {
        const qsv_op& op = C->ops[it.ops[0]];
        std::vector<double> G = op_matrix(op, theta(op));
        if (dag)
            G = dagger(G, 1 << op.k);
        int ct[QSV_MAX_TARGETS];
        std::vector<double> Gc;
        canonicalize(op.targets, op.k, G.data(), ct, Gc);
        return build_launch(C->n, dt, ct, op.k, op.controls, op.c, Gc.data(), true);
    }
    const int m = (int)it.qs.size(), Dm = 1 << m;
    std::vector<double> M((size_t)2 * Dm * Dm, 0.0);
    for (int i = 0; i < Dm; ++i)
        M[((size_t)i * Dm + i) * 2] = 1.0;
    for (int o : it.ops) {
        const qsv_op& op = C->ops[o];
        M = matmul(embed(op, op_matrix(op, theta(op)), it.qs), M, Dm);
    }
    if (dag)
        M = dagger(M, Dm);
    return build_launch(C->n, dt, it.qs.data(), m, nullptr, 0, M.data(), true);
}

}  // namespace qsv

namespace qsv {

// Estimated traffic of a diagonal launch as a fraction of a full read+write
// sweep: the touched fraction 2^-(fixed bits), scaled up when the touched runs
// (2^(lowest fixed bit) amplitudes) are shorter than a 128-byte line.
static double diag_cost(uint64_t fix, int S)
{
    if (!fix)
        return 1.0;
    const int pmin = __builtin_ctzll(fix);
    double frac = std::ldexp(1.0, -__builtin_popcountll(fix));
    const double run = std::ldexp((double)S, pmin);
    if (run < 128.0)
        frac *= 128.0 / run;
    return frac < 1.0 ? frac : 1.0;
}

static bool as_factor(const GateLaunch& L, uint64_t& fix, uint64_t& val)
{
    if (L.type != L_DIAG || L.rot != ROT_NONE || L.K > 5 || L.ngroups == 0)
        return false;
    const int shift = L.mode == W2 ? 1 : 0;
    fix = 0;
    for (int j = 0; j < L.ins.nins; ++j)
        fix |= 1ull << (__builtin_popcountll(L.ins.low[j]) + shift);
    val = L.ins.setmask << shift;
    return true;
}

// Diagonal gates commute with each other and with any gate on other qubits,
// so a run collects diagonal launches and lets every other launch that acts
// on none of the run's qubits go ahead of it; a launch that touches one of
// them closes the run.  A closed run of >= 2 launches whose separate traffic
// is estimated at >= 1.25 full sweeps becomes one L_DIAGRUN sweep (at most
// kMaxRunFactors factors); otherwise its launches are kept as they are.
void merge_diagonal_runs(std::vector<GateLaunch>& Ls, std::vector<long long>& upload_off, int n, int dt)
{
    const int S = dt == C64 ? 8 : 16;
    std::vector<GateLaunch> out;
    std::vector<long long> offs;
    std::vector<size_t> run;
    uint64_t runq = 0;
    double cost = 0.0;
    auto close = [&]() {
        if (run.size() >= 2 && cost >= 1.25) {
            GateLaunch R{};
            R.type = L_DIAGRUN;
            R.dt = dt;
            R.n = n;
            R.mode = W1;
            R.ngroups = dt == C64 ? (1ull << n) / 2 : (1ull << n);
            R.qmask = runq;
            for (size_t k : run) {
                const GateLaunch& D = Ls[k];
                const int f = R.run_nf++;
                as_factor(D, R.run_fix[f], R.run_val[f]);
                R.run_nt[f] = D.K;
                for (int b = 0; b < D.K; ++b)
                    R.run_tpos[f][b] = D.tpos[b];
                R.run_off[f] = (int)(R.run_tab.size() / 2);
                R.run_tab.insert(R.run_tab.end(), D.g.begin(), D.g.begin() + (2 << D.K));
                R.flops += 6.0 * std::ldexp(1.0, n);
            }
            R.bytes = 2.0 * S * std::ldexp(1.0, n);
            out.push_back(R);
            offs.push_back(-1);
        } else {
            for (size_t k : run) {
                out.push_back(Ls[k]);
                offs.push_back(upload_off[k]);
            }
        }
        run.clear();
        runq = 0;
        cost = 0.0;
    };
    for (size_t j = 0; j < Ls.size(); ++j) {
        uint64_t fix, val;
        if (as_factor(Ls[j], fix, val)) {
            if (run.size() == (size_t)kMaxRunFactors)
                close();
            run.push_back(j);
            runq |= Ls[j].qmask;
            cost += diag_cost(fix, S);
            continue;
        }
        if (!run.empty() && (Ls[j].qmask & runq))
            close();
        out.push_back(Ls[j]);
        offs.push_back(upload_off[j]);
    }
    close();
    Ls.swap(out);
    upload_off.swap(offs);
}

// A plain single-qubit gate (uncontrolled, bound matrix) directly before or
// after a diagonal run joins the run's sweep when the run kernel holds both
// amplitudes of its pairs: complex64 qubit 0 (inside a 16-byte unit), a
// target on unit bits 0..5 (across lanes: complex64 qubits 1..6, complex128
// 0..5), or one on a unit bit >= 6 with the window of four varying unit bits
// placed over it (complex64 qubits >= 7, complex128 >= 6; a window below
// unit bit 8 moves the block's wave bits above it); states of >= 2^12 units.
// The window with the cheapest factor classes is taken, also for runs
// without a gate.
static bool plain_1q(const GateLaunch& L, int& t)
{
    // no controls: the only inserted bit is the target's (none in complex64
    // INTRA mode, where the target is qubit 0 inside a 16-byte unit)
    if (L.type != L_DENSE || L.K != 1 || L.rot != ROT_NONE || L.ins.setmask != 0 ||
        L.ins.nins != (L.mode == INTRA ? 0 : 1) || L.g.size() < 8)
        return false;
    t = L.lowq;
    return true;
}

static double run_cost(const GateLaunch& R, int w, int dt)
{
    uint64_t vm = 0;
    for (int j = 0; j < 4; ++j)
        vm |= 1ull << (w + j + (dt == C64 ? 1 : 0));
    if (dt == C64)
        vm |= 1;
    double c = 0.0;
    for (int f = 0; f < R.run_nf; ++f) {
        uint64_t dep = R.run_fix[f];
        for (int b = 0; b < R.run_nt[f]; ++b)
            dep |= 1ull << R.run_tpos[f][b];
        const int nr = __builtin_popcountll(dep & vm);
        c += nr == 0 ? 1.0 : (nr == 1 ? 2.0 : 16.0);
    }
    return c;
}

void fold_gates_into_runs(std::vector<GateLaunch>& Ls, std::vector<long long>& upload_off, int n, int dt)
{
    const int nu = dt == C64 ? n - 1 : n;  // bits of the 16-byte unit index
    if (nu < 12)
        return;
    for (size_t j = 0; j < Ls.size(); ++j) {
        if (Ls[j].type != L_DIAGRUN || Ls[j].run_gate)
            continue;
        for (int side = 0; side < 2; ++side) {  // the launch before, then the one after
            if (side == 0 && j == 0)
                continue;
            const size_t k = side == 0 ? j - 1 : j + 1;
            int t;
            if (k >= Ls.size() || !plain_1q(Ls[k], t) || upload_off[k] >= 0)
                continue;
            int wlo, whi;
            const int tb = dt == C64 ? t - 1 : t;  // the target's unit bit (-1: inside a unit)
            if (tb < 6) {
                // inside a 16-byte unit or across lanes: any window
                wlo = 8;
                whi = nu - 4;
            } else {
                wlo = std::max(6, tb - 3);
                whi = std::min(tb, nu - 4);
            }
            int best = -1;
            for (int w = wlo; w <= whi; ++w) {
                if (w < 8 && w + 6 > nu)
                    continue;  // below 8 the waves sit above the window
                if (best < 0 || run_cost(Ls[j], w, dt) < run_cost(Ls[j], best, dt))
                    best = w;
            }
            if (best < 0)
                continue;
            GateLaunch& R = Ls[j];
            R.run_w = best;
            R.run_gate = side == 0 ? 1 : 2;
            R.run_gt = t;
            for (int q = 0; q < 8; ++q)
                R.run_g[q] = Ls[k].g[q];
            R.qmask |= Ls[k].qmask;
            R.flops += Ls[k].flops;
            Ls.erase(Ls.begin() + (long)k);
            upload_off.erase(upload_off.begin() + (long)k);
            if (side == 0)
                --j;  // the run moved down by one
            break;
        }
    }
    // runs without a gate take the window with the cheapest factor classes
    for (GateLaunch& R : Ls)
        if (R.type == L_DIAGRUN && !R.run_gate)
            for (int w = 9; w + 4 <= nu; ++w)
                if (run_cost(R, w, dt) < run_cost(R, R.run_w, dt))
                    R.run_w = w;
}

// A SWAP moves the half of the state whose two bits differ; when the lower
// qubit is below 4 its moved amplitudes share 128-byte lines with unmoved
// ones, so it costs a full sweep.  A run of consecutive SWAPs composes into
// one bit permutation, applied by qubit permutation passes of one full sweep
// each; the run is replaced when that is cheaper.
void merge_swaps(std::vector<GateLaunch>& Ls, std::vector<long long>& upload_off, int n, int dt)
{
    const int rl = dt == C64 ? kQpRowBitsC64 : kQpRowBitsC128;
    if (n < 2 * rl)
        return;
    std::vector<GateLaunch> out;
    std::vector<long long> offs;
    size_t j = 0;
    while (j < Ls.size()) {
        if (Ls[j].type != L_PERM || Ls[j].swapq[0] < 0) {
            out.push_back(Ls[j]);
            offs.push_back(upload_off[j]);
            ++j;
            continue;
        }
        size_t e = j;
        std::vector<std::pair<int, int>> sw;
        double sep = 0.0;
        uint64_t qm = 0;
        for (; e < Ls.size() && Ls[e].type == L_PERM && Ls[e].swapq[0] >= 0; ++e) {
            const int a = Ls[e].swapq[0], b = Ls[e].swapq[1];
            sw.push_back({a, b});
            sep += std::min(a, b) < 4 ? 1.0 : 0.5;
            qm |= (1ull << a) | (1ull << b);
        }
        std::vector<QPermPass> passes;
        plan_qubit_permutation(compose_swaps(sw, n), n, rl, passes);
        if ((double)passes.size() < sep) {
            for (const QPermPass& P : passes) {
                GateLaunch R{};
                R.type = L_QPERM;
                R.dt = dt;
                R.n = n;
                R.ngroups = P.ntiles;
                R.qp_rl = P.rl;
                R.qp_hb = P.hb;
                std::vector<int> tpos;
                for (int k = 0; k < P.rl; ++k)
                    tpos.push_back(k);
                for (int k = 0; k < P.hb; ++k) {
                    R.qp_hpos[k] = P.hpos[k];
                    tpos.push_back(P.hpos[k]);
                }
                for (int k = 0; k < P.rl + P.hb; ++k)
                    R.qp_cmap[k] = P.cmap[k];
                for (int b = 0; b < n; ++b) {
                    R.qp_q[b] = P.q[b];
                    R.qp_wsrc[b] = P.wsrc[b];
                }
                R.ins = make_ins(tpos, 0);
                R.qmask = qm;
                R.bytes = 2.0 * amp_bytes(dt) * std::ldexp(1.0, n);
                out.push_back(R);
                offs.push_back(-1);
            }
        } else {
            for (size_t k = j; k < e; ++k) {
                out.push_back(Ls[k]);
                offs.push_back(upload_off[k]);
            }
        }
        j = e;
    }
    Ls.swap(out);
    upload_off.swap(offs);
}

}  // namespace qsv

// ================================================================= plans

struct qsv_plan {
    int n = 0, dt = 0, nparams = 0;
    std::vector<GateLaunch> launches;
    std::vector<long long> upload_off;
    DevPack dev;
    GraphCache graph;
    double bytes = 0, flops = 0;
};

struct AdjItem {
    bool rotation;
    int slot;
    GateLaunch L;
    long long uoff;
};

struct qsv_adjoint_plan {
    int n = 0, dt = 0, nparams = 0, nslots = 0, nb = 0;
    std::vector<GateLaunch> fwd;
    std::vector<long long> fwd_off;
    std::vector<AdjItem> rev;
    std::vector<uint64_t> hx, hz;
    std::vector<double> hc;
    qsv_pauli_sum H{};
    DevPack dev;
    size_t off_csr = 0;
    size_t off_lam = 0, off_part = 0, off_red = 0, work_bytes = 0;
    GraphCache graph;
    GraphCache egraph;
    // cache-blocked mode (every gate single-target with <= 2 controls)
    bool tiled = false;
    TileProgram tp;
    int tm = 0;       // tile qubits
    int tblocks = 0;  // blocks per pass launch (= partial columns)
    size_t o_steps = 0, o_ops = 0, o_mats = 0;
    size_t off_lops = 0;  // workspace: staged gate descriptors (forward, reverse)
};

namespace {

static uint64_t op_qubits(const qsv_op& op)
{
    uint64_t m = 0;
    for (int j = 0; j < op.k; ++j)
        m |= 1ull << op.targets[j];
    for (int j = 0; j < op.c; ++j)
        m |= 1ull << op.controls[j];
    return m;
}

qsv_status build_plan(const qsv_circuit* circ, int dt, int fuse_k, const double* params_host,
                      qsv_plan* P)
{
    P->n = circ->n;
    P->dt = dt;
    P->nparams = circ->nparams;
    // deferring diagonal gates pays when blocks have room to pack them: with
    // fuse_k = 2 a deferred CZ becomes a launch of its own instead of
    // starting a block with the gates after it (measured slower)
    const char* nodd = getenv("QSV_NO_DIAG_DEFER");
    const bool defer = fuse_k >= 3 && (!nodd || nodd[0] != '1');
    std::vector<Item> items = fuse_ops(circ, fuse_k, params_host == nullptr, defer);
    for (const Item& it : items) {
        if (it.rotation) {
            const qsv_op& op = circ->ops[it.ops[0]];
            GateLaunch L = rotation_launch(circ->n, dt, op.kind, op.targets[0], op.controls, op.c,
                                           op.param);
            P->bytes += L.bytes;
            P->flops += L.flops;
            L.qmask = op_qubits(op);
            P->launches.push_back(L);
            P->upload_off.push_back(-1);
            continue;
        }
        Built b = item_launch(circ, it, dt, params_host, false);
        if (b.noop)
            continue;
        b.L.qmask = 0;
        for (int o : it.ops)
            b.L.qmask |= op_qubits(circ->ops[o]);
        P->bytes += b.L.bytes;
        P->flops += b.L.flops;
        P->upload_off.push_back(b.upload.empty() ? -1 : (long long)P->dev.add(std::move(b.upload)));
        P->launches.push_back(b.L);
    }
    const char* nosw = getenv("QSV_NO_SWAP_MERGE");
    if (!nosw || nosw[0] != '1')
        merge_swaps(P->launches, P->upload_off, P->n, dt);
    const char* nodr = getenv("QSV_NO_DIAG_RUN");
    if (!nodr || nodr[0] != '1') {
        merge_diagonal_runs(P->launches, P->upload_off, P->n, dt);
        const char* nogf = getenv("QSV_NO_GATE_FOLD");
        if (!nogf || nogf[0] != '1')
            fold_gates_into_runs(P->launches, P->upload_off, P->n, dt);
        for (size_t j = 0; j < P->launches.size(); ++j) {
            const GateLaunch& L = P->launches[j];
            if (L.type != L_DIAGRUN)
                continue;
            std::vector<unsigned char> bytes;
            if (dt == QSV_C64) {
                const std::vector<float> f(L.run_tab.begin(), L.run_tab.end());
                const unsigned char* b = reinterpret_cast<const unsigned char*>(f.data());
                bytes.assign(b, b + f.size() * sizeof(float));
            } else {
                const unsigned char* b = reinterpret_cast<const unsigned char*>(L.run_tab.data());
                bytes.assign(b, b + L.run_tab.size() * sizeof(double));
            }
            P->upload_off[j] = (long long)P->dev.add(std::move(bytes));
        }
        P->bytes = P->flops = 0.0;
        for (const GateLaunch& L : P->launches) {
            P->bytes += L.bytes;
            P->flops += L.flops;
        }
    }
    qsv_status st = P->dev.commit();
    if (st)
        return st;
    for (size_t j = 0; j < P->launches.size(); ++j)
        if (P->upload_off[j] >= 0)
            P->launches[j].gdev = P->dev.at((size_t)P->upload_off[j]);
    return QSV_OK;
}

qsv_status enqueue_launches(const std::vector<GateLaunch>& Ls, void* psi, const double* params,
                            hipStream_t s)
{
    for (const GateLaunch& L0 : Ls) {
        if (L0.rot != ROT_NONE) {
            GateLaunch L = L0;
            L.params = params;
            qsv_status st = launch_checked(L, psi, nullptr, s);
            if (st)
                return st;
        } else {
            qsv_status st = launch_checked(L0, psi, nullptr, s);
            if (st)
                return st;
        }
    }
    return QSV_OK;
}

bool has_rotation(const std::vector<GateLaunch>& Ls)
{
    for (const GateLaunch& L : Ls)
        if (L.rot != ROT_NONE)
            return true;
    return false;
}

}  // namespace

extern "C" {

qsv_status qsv_plan_create(const qsv_circuit* circ, qsv_dtype dt, int fuse_k,
                           const double* params_host, qsv_plan** plan)
{
    qsv_status st = check_circuit(circ, QSV_MAX_QUBITS);
    if (st)
        return st;
    if ((st = check_n_dt(circ->n, dt)))
        return st;
    if (fuse_k < 1 || fuse_k > QSV_MAX_TARGETS)
        return fail(QSV_ERR_ARG, "fuse_k = %d outside [1, %d]", fuse_k, QSV_MAX_TARGETS);
    if (!plan)
        return fail(QSV_ERR_ARG, "plan is NULL");
    std::unique_ptr<qsv_plan> P(new qsv_plan);
    if ((st = build_plan(circ, dt, fuse_k, params_host, P.get())))
        return st;
    *plan = P.release();
    return ok();
}

qsv_status qsv_plan_run(qsv_plan* plan, void* psi, const double* params_dev, void* stream)
{
    if (!plan)
        return fail(QSV_ERR_ARG, "plan is NULL");
    qsv_status st = check_state(psi, plan->n, plan->dt, "psi");
    if (st)
        return st;
    if (has_rotation(plan->launches) && !params_dev)
        return fail(QSV_ERR_ARG, "plan has unbound rotations but params_dev is NULL");
    if (plan->launches.empty())
        return ok();  // nothing to enqueue (empty or all-identity circuit)
    if ((st = enqueue_gate()))
        return st;
    hipStream_t s = (hipStream_t)stream;
    std::vector<const void*> key = {psi, params_dev};
    if ((st = run_graph(plan->graph, key, s, [&](hipStream_t cs) {
             return enqueue_launches(plan->launches, psi, params_dev, cs);
         })))
        return st;
    return ok();
}

qsv_status qsv_plan_info(const qsv_plan* plan, int* nlaunches, double* bytes, double* flops)
{
    if (!plan)
        return fail(QSV_ERR_ARG, "plan is NULL");
    if (nlaunches)
        *nlaunches = (int)plan->launches.size();
    if (bytes)
        *bytes = plan->bytes;
    if (flops)
        *flops = plan->flops;
    return ok();
}

qsv_status qsv_plan_destroy(qsv_plan* plan)
{
    delete plan;
    return ok();
}

// --------------------------------------------------------------- adjoint

qsv_status qsv_adjoint_plan_create(const qsv_circuit* circ, const qsv_pauli_sum* H, qsv_dtype dt,
                                   int fuse_k, qsv_adjoint_plan** plan, size_t* work_bytes)
{
    qsv_status st = check_circuit(circ, QSV_MAX_QUBITS);
    if (st)
        return st;
    if ((st = check_n_dt(circ->n, dt)))
        return st;
    if ((st = check_hamiltonian(H, circ->n)))
        return st;
    if (fuse_k < 1 || fuse_k > QSV_MAX_TARGETS)
        return fail(QSV_ERR_ARG, "fuse_k = %d outside [1, %d]", fuse_k, QSV_MAX_TARGETS);
    if (!plan || !work_bytes)
        return fail(QSV_ERR_ARG, "plan or work_bytes is NULL");
    const int n = circ->n;
    std::unique_ptr<qsv_adjoint_plan> P(new qsv_adjoint_plan);
    P->n = n;
    P->dt = dt;
    P->nparams = circ->nparams;
    P->nb = reduce_blocks(n, dt);
    P->hx.assign(H->x_mask, H->x_mask + H->nterms);
    P->hz.assign(H->z_mask, H->z_mask + H->nterms);
    P->hc.assign(H->coeff, H->coeff + H->nterms);
    P->H = qsv_pauli_sum{H->nterms, P->hx.data(), P->hz.data(), P->hc.data()};

    // tile steps hold 8 amplitudes per thread: the cache-blocked mode needs n >= 3
    bool tileable = n >= 3 && (getenv("QSV_NO_TILES") == nullptr || getenv("QSV_NO_TILES")[0] != '1');
    for (int o = 0; o < circ->nops && tileable; ++o) {
        const qsv_op& op = circ->ops[o];
        tileable = op.k == 1 && op.c <= 2 && op.kind != QSV_OP_SWAP;
        if (tileable && op.kind == QSV_OP_MATRIX && !is_unitary(op_matrix(op, 0.0), 2))
            return fail(QSV_ERR_ARG, "op %d: MATRIX is not unitary (the adjoint uncomputes with "
                                     "G^dagger)", o);
    }
    if (tileable) {
        std::vector<HGate> gates;
        std::vector<double> mats;
        for (int o = 0; o < circ->nops; ++o) {
            const qsv_op& op = circ->ops[o];
            HGate g{};
            g.t = op.targets[0];
            g.nc = op.c;
            g.c0 = op.c > 0 ? op.controls[0] : 0;
            g.c1 = op.c > 1 ? op.controls[1] : 0;
            g.param = -1;
            g.mat = -1;
            if (is_rotation(op.kind)) {
                g.kind = op.kind;
                g.param = op.param;
            } else {
                g.kind = 0;
                g.mat = (int)(mats.size() / 8);
                std::vector<double> m = op_matrix(op, 0.0);
                mats.insert(mats.end(), m.begin(), m.end());
            }
            gates.push_back(g);
        }
        // Full-size tiles (2^12 complex64, 2^11 complex128 amplitudes), down
        // to 2^10 while the state would give fewer tiles than there are CUs
        // (small states: more, smaller blocks spread the steps over the
        // whole GPU).
        P->tm = std::min(n, dt == QSV_C64 ? 12 : 11);
        {
            int dev = 0, cus = 256;
            if (hipGetDevice(&dev) == hipSuccess)
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            while (P->tm > 10 && (1ll << (n - P->tm)) < (long long)cus)
                --P->tm;
        }
        compile_tile_program(gates, n, P->tm, kMaxTpassOps, P->tp);
        const int res = tpass_resident_blocks(dt, P->tm, true);
        if (res <= 0)
            return fail(QSV_ERR_UNSUPPORTED, "tile pass kernel does not fit this device");
        const uint64_t ntiles = 1ull << (n - P->tm);
        P->tblocks = (int)std::min<uint64_t>(ntiles, (uint64_t)res);
        P->tiled = true;
        P->nslots = (int)P->tp.slot_param.size();
        P->o_steps = P->dev.add(table_bytes(P->tp.steps));
        P->o_ops = P->dev.add(table_bytes(P->tp.ops));
        P->o_mats = P->dev.add(table_bytes(mats, 8));
        std::vector<std::vector<int>> sl(circ->nparams);
        for (int sidx = 0; sidx < P->nslots; ++sidx)
            sl[P->tp.slot_param[sidx]].push_back(sidx);
        std::vector<int> csr(circ->nparams + 1 + P->nslots + 1, 0);
        int fill = 0;
        for (int p = 0; p < circ->nparams; ++p) {
            csr[p] = fill;
            for (int v : sl[p])
                csr[circ->nparams + 1 + fill++] = v;
        }
        csr[circ->nparams] = fill;
        P->off_csr = P->dev.add(table_bytes(csr));
        if ((st = P->dev.commit()))
            return st;
        const size_t sb = amp_bytes(dt) << n;
        auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
        P->off_lam = up(sb);
        P->off_part = P->off_lam + up(sb);
        P->off_red = P->off_part +
                     up(sizeof(double) * (size_t)std::max(P->nslots, 1) * (size_t)P->tblocks);
        P->off_lops = P->off_red + up(kReduceWorkBytes);
        P->work_bytes = P->off_lops + tpass_lop_bytes(dt, (int)P->tp.ops.size());
        *work_bytes = P->work_bytes;
        *plan = P.release();
        return ok();
    }

    std::vector<Item> items = fuse_ops(circ, fuse_k, true);
    std::vector<std::vector<int>> slots_of(circ->nparams);
    std::vector<long long> rev_off;
    for (const Item& it : items) {
        if (it.rotation) {
            const qsv_op& op = circ->ops[it.ops[0]];
            GateLaunch L = rotation_launch(n, dt, op.kind, op.targets[0], op.controls, op.c, op.param);
            P->fwd.push_back(L);
            P->fwd_off.push_back(-1);
            const int slot = P->nslots++;
            slots_of[op.param].push_back(slot);
            P->rev.push_back(AdjItem{true, slot, L, -1});
            continue;
        }
        for (int o : it.ops) {
            const qsv_op& op = circ->ops[o];
            const int D = 1 << op.k;
            if (op.kind == QSV_OP_MATRIX && !is_unitary(op_matrix(op, 0.0), D))
                return fail(QSV_ERR_ARG, "op %d: MATRIX is not unitary (the adjoint uncomputes with "
                                         "G^dagger)", o);
        }
        Built f = item_launch(circ, it, dt, nullptr, false);
        if (f.noop)
            continue;
        P->fwd_off.push_back(f.upload.empty() ? -1 : (long long)P->dev.add(std::move(f.upload)));
        P->fwd.push_back(f.L);
        Built r = item_launch(circ, it, dt, nullptr, true);
        const long long ro = r.upload.empty() ? -1 : (long long)P->dev.add(std::move(r.upload));
        P->rev.push_back(AdjItem{false, -1, r.L, ro});
    }
    std::reverse(P->rev.begin(), P->rev.end());
    // CSR of slots per parameter
    std::vector<int> csr(circ->nparams + 1 + P->nslots + 1, 0);
    int fill = 0;
    for (int p = 0; p < circ->nparams; ++p) {
        csr[p] = fill;
        for (int sl : slots_of[p])
            csr[circ->nparams + 1 + fill++] = sl;
    }
    csr[circ->nparams] = fill;
    std::vector<unsigned char> cbytes(csr.size() * sizeof(int));
    std::memcpy(cbytes.data(), csr.data(), cbytes.size());
    P->off_csr = P->dev.add(std::move(cbytes));
    if ((st = P->dev.commit()))
        return st;
    for (size_t j = 0; j < P->fwd.size(); ++j)
        if (P->fwd_off[j] >= 0)
            P->fwd[j].gdev = P->dev.at((size_t)P->fwd_off[j]);
    for (AdjItem& a : P->rev)
        if (a.uoff >= 0)
            a.L.gdev = P->dev.at((size_t)a.uoff);
    const size_t sb = amp_bytes(dt) << n;
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    P->off_lam = up(sb);
    P->off_part = P->off_lam + up(sb);
    P->off_red = P->off_part + up(sizeof(double) * (size_t)(P->nslots > 0 ? P->nslots : 1) * P->nb);
    P->work_bytes = P->off_red + kReduceWorkBytes;
    *work_bytes = P->work_bytes;
    *plan = P.release();
    return ok();
}

static qsv_status adjoint_enqueue_tiled(qsv_adjoint_plan* P, const double* params, void* psi,
                                        void* lam, double* part, double* red, double* energy,
                                        double* grad, bool with_grad, hipStream_t s)
{
    TPassArgs a{};
    a.steps = static_cast<const DStep*>(P->dev.at(P->o_steps));
    a.ops = static_cast<const DOp*>(P->dev.at(P->o_ops));
    a.mats = static_cast<const double*>(P->dev.at(P->o_mats));
    a.params = params;
    a.lops = static_cast<char*>(psi) + P->off_lops;
    a.partials = part;
    a.nops_total = (int)P->tp.ops.size();
    a.n = P->n;
    a.m = P->tm;
    hipError_t es = launch_tstage(a, P->dt, s);
    if (es != hipSuccess)
        return fail(QSV_ERR_HIP, "tile program staging launch: %s", hipGetErrorString(es));
    for (const DPass& pass : P->tp.passes) {
        a.pass = pass;
        hipError_t e = launch_tpass(a, P->dt, false, psi, nullptr, P->tblocks, s);
        if (e != hipSuccess)
            return fail(QSV_ERR_HIP, "tile pass launch: %s", hipGetErrorString(e));
    }
    if (!with_grad)
        return enqueue_expectation(psi, P->n, P->dt, &P->H, energy, red, 1, s);
    qsv_status st = enqueue_hpsi(psi, lam, P->n, P->dt, &P->H, s);
    if (st)
        return st;
    hipError_t e = launch_inner(psi, lam, P->n, P->dt, red, 0, s);
    if (e == hipSuccess)
        e = launch_finalize(red, reduce_blocks(P->n, P->dt), 1, energy, s);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "energy launch: %s", hipGetErrorString(e));
    for (int p = (int)P->tp.passes.size() - 1; p >= 0; --p) {
        a.pass = P->tp.passes[p];
        e = launch_tpass(a, P->dt, true, psi, lam, P->tblocks, s);
        if (e != hipSuccess)
            return fail(QSV_ERR_HIP, "tile pass launch: %s", hipGetErrorString(e));
    }
    const int* csr = static_cast<const int*>(P->dev.at(P->off_csr));
    e = launch_grad_finalize(part, P->tblocks, csr, csr + P->nparams + 1, P->nparams, grad, s);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "gradient finalize launch: %s", hipGetErrorString(e));
    return QSV_OK;
}

static qsv_status adjoint_enqueue(qsv_adjoint_plan* P, const double* params, void* work,
                                  double* energy, double* grad, bool with_grad, hipStream_t s)
{
    char* w = static_cast<char*>(work);
    void* psi = w;
    void* lam = w + P->off_lam;
    double* part = reinterpret_cast<double*>(w + P->off_part);
    double* red = reinterpret_cast<double*>(w + P->off_red);
    hipError_t e = launch_init_basis(psi, P->n, P->dt, 0, s);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "init launch: %s", hipGetErrorString(e));
    if (P->tiled)
        return adjoint_enqueue_tiled(P, params, psi, lam, part, red, energy, grad, with_grad, s);
    qsv_status st = enqueue_launches(P->fwd, psi, params, s);
    if (st)
        return st;
    if (!with_grad)
        return enqueue_expectation(psi, P->n, P->dt, &P->H, energy, red, 1, s);
    if ((st = enqueue_hpsi(psi, lam, P->n, P->dt, &P->H, s)))
        return st;
    e = launch_inner(psi, lam, P->n, P->dt, red, 0, s);
    if (e == hipSuccess)
        e = launch_finalize(red, P->nb, 1, energy, s);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "energy launch: %s", hipGetErrorString(e));
    for (const AdjItem& a : P->rev) {
        if (a.rotation) {
            GateLaunch L = a.L;
            L.params = params;
            e = launch_adj_step(L, psi, lam, part + (size_t)a.slot * P->nb, P->nb, s);
            if (e != hipSuccess)
                return fail(QSV_ERR_HIP, "adjoint step launch: %s", hipGetErrorString(e));
        } else if ((st = launch_checked(a.L, psi, lam, s))) {
            return st;
        }
    }
    const int* csr = static_cast<const int*>(P->dev.at(P->off_csr));
    e = launch_grad_finalize(part, P->nb, csr, csr + P->nparams + 1, P->nparams, grad, s);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "gradient finalize launch: %s", hipGetErrorString(e));
    return QSV_OK;
}

}  // extern "C"

namespace qsv {
qsv_status adjoint_enqueue_direct(qsv_adjoint_plan* P, const double* params, void* work,
                                  double* energy, double* grad, hipStream_t s)
{
    return adjoint_enqueue(P, params, work, energy, grad, true, s);
}
size_t adjoint_work_bytes(const qsv_adjoint_plan* P)
{
    return P->work_bytes;
}
}  // namespace qsv

extern "C" {

qsv_status qsv_adjoint_run(qsv_adjoint_plan* plan, const double* params_dev, void* work,
                           double* energy_dev, double* grad_dev, void* stream)
{
    if (!plan)
        return fail(QSV_ERR_ARG, "plan is NULL");
    if (!work || !energy_dev || (plan->nparams > 0 && (!grad_dev || !params_dev)))
        return fail(QSV_ERR_ARG, "NULL work, energy, gradient or parameter pointer");
    if (reinterpret_cast<uintptr_t>(work) % 256)
        return fail(QSV_ERR_ARG, "work is not 256-byte aligned");
    if (qsv_status gst = enqueue_gate())
        return gst;
    hipStream_t s = (hipStream_t)stream;
    std::vector<const void*> key = {params_dev, work, energy_dev, grad_dev};
    qsv_status st = run_graph(plan->graph, key, s, [&](hipStream_t cs) {
        return adjoint_enqueue(plan, params_dev, work, energy_dev, grad_dev, true, cs);
    });
    if (st)
        return st;
    return ok();
}

qsv_status qsv_adjoint_energy(qsv_adjoint_plan* plan, const double* params_dev, void* work,
                              double* energy_dev, void* stream)
{
    if (!plan)
        return fail(QSV_ERR_ARG, "plan is NULL");
    if (!work || !energy_dev || (plan->nparams > 0 && !params_dev))
        return fail(QSV_ERR_ARG, "NULL work, energy or parameter pointer");
    if (reinterpret_cast<uintptr_t>(work) % 256)
        return fail(QSV_ERR_ARG, "work is not 256-byte aligned");
    if (qsv_status gst = enqueue_gate())
        return gst;
    hipStream_t s = (hipStream_t)stream;
    std::vector<const void*> key = {params_dev, work, energy_dev};
    qsv_status st = run_graph(plan->egraph, key, s, [&](hipStream_t cs) {
        return adjoint_enqueue(plan, params_dev, work, energy_dev, nullptr, false, cs);
    });
    if (st)
        return st;
    return ok();
}

qsv_status qsv_adjoint_state(const qsv_adjoint_plan* plan, void* work, int slot, void** psi)
{
    if (!plan || !work || !psi || slot < 0 || slot > 1)
        return fail(QSV_ERR_ARG, "bad argument");
    *psi = static_cast<char*>(work) + (slot ? plan->off_lam : 0);
    return ok();
}

qsv_status qsv_adjoint_plan_destroy(qsv_adjoint_plan* plan)
{
    delete plan;
    return ok();
}

qsv_status qsv_adjoint_gradient(const qsv_circuit* circ, const double* params_dev,
                                const qsv_pauli_sum* H, qsv_dtype dt, int fuse_k, void* work,
                                size_t work_bytes, double* energy_dev, double* grad_dev,
                                void* stream)
{
    qsv_adjoint_plan* P = nullptr;
    size_t wb = 0;
    qsv_status st = qsv_adjoint_plan_create(circ, H, dt, fuse_k, &P, &wb);
    if (st)
        return st;
    if (!work || !energy_dev || (P->nparams > 0 && (!grad_dev || !params_dev))) {
        delete P;
        return fail(QSV_ERR_ARG, "NULL work, energy, gradient or parameter pointer");
    }
    if (reinterpret_cast<uintptr_t>(work) % 256) {
        delete P;
        return fail(QSV_ERR_ARG, "work is not 256-byte aligned");
    }
    if (work_bytes < wb) {
        delete P;
        return fail(QSV_ERR_ARG, "work holds %zu bytes, this circuit needs %zu", work_bytes, wb);
    }
    if ((st = enqueue_gate())) {
        delete P;
        return st;
    }
    hipStream_t s = (hipStream_t)stream;
    st = adjoint_enqueue(P, params_dev, work, energy_dev, grad_dev, true, s);
    // the plan's device memory is read by the enqueued kernels: wait for
    // them before releasing it, whatever the enqueue returned
    const hipError_t e = hipStreamSynchronize(s);
    delete P;
    if (st)
        return st;
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "stream synchronisation: %s", hipGetErrorString(e));
    return ok();
}

}  // extern "C"
