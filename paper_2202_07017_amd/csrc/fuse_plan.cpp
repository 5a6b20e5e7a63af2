// Gate fusion planner (declared in qsv_fuse_plan.h).
#include "qsv_fuse_plan.h"

#include <set>

namespace qsv {

// Whether op's matrix is diagonal (controls keep it diagonal).
static bool is_diagonal_op(const qsv_op& op)
{
    if (op.kind == QSV_OP_Z)
        return true;
    if (op.kind != QSV_OP_MATRIX || !op.M)
        return false;
    const int D = 1 << op.k;
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c)
            if (r != c && (op.M[((size_t)r * D + c) * 2] != 0.0 || op.M[((size_t)r * D + c) * 2 + 1] != 0.0))
                return false;
    return true;
}

std::vector<Item> fuse_ops(const qsv_circuit* C, int fuse_k, bool rotations_standalone,
                           bool defer_diagonal)
{
    struct Blk {
        std::set<int> qs;
        std::vector<int> ops;
        bool open = true;
    };
    std::vector<Blk> blks;
    std::vector<int> owner(C->n, -1);
    std::vector<Item> out;
    auto emit = [&](int b) {
        Blk& B = blks[b];
        if (!B.open)
            return;
        B.open = false;
        for (int q : B.qs)
            if (owner[q] == b)
                owner[q] = -1;
        Item it;
        it.ops = B.ops;
        it.qs.assign(B.qs.begin(), B.qs.end());
        out.push_back(it);
    };
    std::vector<int> pool;  // deferred diagonal gates
    std::vector<char> pooled(C->n, 0);
    auto flush = [&]() {
        if (pool.empty())
            return;
        for (int q = 0; q < C->n; ++q)
            if (pooled[q] && owner[q] >= 0)
                emit(owner[q]);
        std::vector<Item> groups;
        for (int o : pool) {
            const qsv_op& op = C->ops[o];
            std::set<int> Q(op.targets, op.targets + op.k);
            Q.insert(op.controls, op.controls + op.c);
            Item* g = nullptr;
            for (Item& G : groups) {
                std::set<int> U(G.qs.begin(), G.qs.end());
                U.insert(Q.begin(), Q.end());
                if ((int)U.size() <= fuse_k) {
                    G.qs.assign(U.begin(), U.end());
                    g = &G;
                    break;
                }
            }
            if (!g) {
                groups.emplace_back();
                g = &groups.back();
                g->qs.assign(Q.begin(), Q.end());
            }
            g->ops.push_back(o);
        }
        out.insert(out.end(), groups.begin(), groups.end());
        pool.clear();
        std::fill(pooled.begin(), pooled.end(), 0);
    };
    for (int o = 0; o < C->nops; ++o) {
        const qsv_op& op = C->ops[o];
        std::vector<int> Q(op.targets, op.targets + op.k);
        Q.insert(Q.end(), op.controls, op.controls + op.c);
        const bool diag = defer_diagonal && !is_rotation(op.kind) && is_diagonal_op(op);
        if (!pool.empty() && !diag)
            for (int q : Q)
                if (pooled[q]) {
                    flush();
                    break;
                }
        std::set<int> owners;
        for (int q : Q)
            if (owner[q] >= 0)
                owners.insert(owner[q]);
        if (rotations_standalone && is_rotation(op.kind)) {
            for (int b : owners)
                emit(b);
            Item it;
            it.rotation = true;
            it.ops = {o};
            out.push_back(it);
            continue;
        }
        std::set<int> U(Q.begin(), Q.end());
        for (int b : owners)
            U.insert(blks[b].qs.begin(), blks[b].qs.end());
        if (diag && (int)U.size() > fuse_k && (int)Q.size() <= fuse_k) {
            pool.push_back(o);
            for (int q : Q)
                pooled[q] = 1;
            continue;
        }
        if ((int)U.size() <= fuse_k) {
            int tgt;
            if (owners.empty()) {
                blks.push_back(Blk{});
                tgt = (int)blks.size() - 1;
            } else {
                tgt = *owners.begin();
                for (int b : owners)
                    if (b != tgt) {
                        blks[tgt].ops.insert(blks[tgt].ops.end(), blks[b].ops.begin(),
                                             blks[b].ops.end());
                        blks[b].open = false;
                    }
            }
            blks[tgt].ops.push_back(o);
            blks[tgt].qs = U;
            for (int q : U)
                owner[q] = tgt;
        } else {
            for (int b : owners)
                emit(b);
            if ((int)Q.size() <= fuse_k) {
                blks.push_back(Blk{});
                const int tgt = (int)blks.size() - 1;
                blks[tgt].ops = {o};
                blks[tgt].qs = std::set<int>(Q.begin(), Q.end());
                for (int q : Q)
                    owner[q] = tgt;
            } else {
                Item it;
                it.ops = {o};
                out.push_back(it);
            }
        }
    }
    flush();
    for (int b = 0; b < (int)blks.size(); ++b)
        emit(b);
    return out;
}


}  // namespace qsv
