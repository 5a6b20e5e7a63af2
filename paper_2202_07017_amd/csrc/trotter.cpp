// Trotterised time evolution of Pauli-sum Hamiltonians (Sec. 3: Hamiltonian
// objects interfaced with a time-evolution solver using the Trotter
// decomposition).  exp(-i tau H), H = sum_j c_j P_j, is approximated per step
// by the product of the exact factors exp(-i theta P_j) = cos(theta) I
// - i sin(theta) P_j, each a dense gate on the support of P_j; the gate list
// is compiled by the ordinary plan compiler, so runs of factors fuse into
// dense blocks exactly like circuit gates.
#include <cmath>
#include <vector>

#include "qsv_host.h"

using namespace qsv;

namespace {

struct Factor {
    int k;
    int t[QSV_MAX_TARGETS];
    std::vector<double> G;   // 2^k x 2^k complex128, row-major, interleaved
};

// exp(-i theta P) for the Pauli string (x, z) on its support; targets in
// descending qubit order (t[0] = highest qubit = most significant bit of the
// matrix index).  An identity string gives the global phase exp(-i theta)
// as a one-qubit diagonal on qubit 0.
Factor pauli_exp(uint64_t x, uint64_t z, double theta)
{
    Factor f{};
    const uint64_t supp = x | z;
    if (!supp) {
        f.k = 1;
        f.t[0] = 0;
        f.G.assign(8, 0.0);
        f.G[0] = f.G[6] = std::cos(theta);
        f.G[1] = f.G[7] = -std::sin(theta);
        return f;
    }
    for (int q = 63; q >= 0; --q)
        if ((supp >> q) & 1ull)
            f.t[f.k++] = q;
    const int dim = 1 << f.k;
    uint64_t xl = 0, zl = 0;
    for (int j = 0; j < f.k; ++j) {
        xl |= ((x >> f.t[j]) & 1ull) << (f.k - 1 - j);
        zl |= ((z >> f.t[j]) & 1ull) << (f.k - 1 - j);
    }
    const int ny = __builtin_popcountll(x & z) & 3;
    // i^ny as (re, im)
    const double yr[4] = {1.0, 0.0, -1.0, 0.0}, yi[4] = {0.0, 1.0, 0.0, -1.0};
    const double c = std::cos(theta), s = std::sin(theta);
    f.G.assign((size_t)2 * dim * dim, 0.0);
    for (int col = 0; col < dim; ++col) {
        f.G[2 * ((size_t)col * dim + col)] += c;
        // P|col> = i^ny (-1)^popcount(col & zl) |col ^ xl>; the factor adds
        // -i s times that column.
        const double sign = (__builtin_popcountll((uint64_t)col & zl) & 1) ? -1.0 : 1.0;
        const int row = col ^ (int)xl;
        // (-i s) * i^ny * sign = s * sign * (yi - i yr)
        f.G[2 * ((size_t)row * dim + col)] += s * sign * yi[ny];
        f.G[2 * ((size_t)row * dim + col) + 1] += -s * sign * yr[ny];
    }
    return f;
}

}  // namespace

extern "C" qsv_status qsv_trotter_plan_create(const qsv_pauli_sum* H, int n, double tau, int steps,
                                              int order, qsv_dtype dt, int fuse_k, qsv_plan** plan)
{
    qsv_status st = check_n_dt(n, dt);
    if (st)
        return st;
    if ((st = check_hamiltonian(H, n)))
        return st;
    if (!plan)
        return fail(QSV_ERR_ARG, "plan is NULL");
    if (steps < 0)
        return fail(QSV_ERR_ARG, "steps = %d is negative", steps);
    if (order != 1 && order != 2)
        return fail(QSV_ERR_ARG, "order = %d is neither 1 nor 2", order);
    if (!std::isfinite(tau))
        return fail(QSV_ERR_ARG, "tau is not finite");
    for (int j = 0; j < H->nterms; ++j)
        if (__builtin_popcountll(H->x_mask[j] | H->z_mask[j]) > QSV_MAX_TARGETS)
            return fail(QSV_ERR_UNSUPPORTED, "Pauli term %d acts on more than %d qubits", j,
                        QSV_MAX_TARGETS);
    // One step's factors: order 1 applies terms 0..T-1 with theta = tau c_j;
    // order 2 (symmetric) applies 0..T-1 then T-1..0, each with tau c_j / 2.
    const int T = H->nterms;
    std::vector<Factor> one;
    one.reserve((size_t)2 * T);
    const double w = order == 1 ? tau : 0.5 * tau;
    for (int j = 0; j < T; ++j)
        one.push_back(pauli_exp(H->x_mask[j], H->z_mask[j], w * H->coeff[j]));
    if (order == 2)
        for (int j = T - 1; j >= 0; --j)
            one.push_back(one[j]);
    std::vector<qsv_op> ops;
    ops.reserve(one.size() * (size_t)steps);
    for (int s = 0; s < steps; ++s)
        for (const Factor& f : one) {
            qsv_op op{};
            op.kind = QSV_OP_MATRIX;
            op.k = f.k;
            for (int j = 0; j < f.k; ++j)
                op.targets[j] = f.t[j];
            op.c = 0;
            op.param = -1;
            op.M = f.G.data();
            ops.push_back(op);
        }
    qsv_circuit circ{};
    circ.n = n;
    circ.nops = (int)ops.size();
    circ.ops = ops.empty() ? nullptr : ops.data();
    circ.nparams = 0;
    return qsv_plan_create(&circ, dt, fuse_k, nullptr, plan);
}
