// Host compiler of tile programs (see qsv_tileprog.h).
#include <algorithm>

#include "qsv_tileprog.h"

namespace qsv {
namespace {

uint64_t gate_qubits(const HGate& g)
{
    uint64_t q = 1ull << g.t;
    if (g.nc > 0)
        q |= 1ull << g.c0;
    if (g.nc > 1)
        q |= 1ull << g.c1;
    return q;
}

int popc(uint64_t v)
{
    return __builtin_popcountll(v);
}

int local_bit(uint64_t B, int q)
{
    return popc(B & ((1ull << q) - 1));
}

// Passes: each takes, in circuit order, every remaining gate whose qubits are
// tile qubits and that no earlier unscheduled gate blocks (an unscheduled
// gate blocks its qubits for every later gate).  Tile qubits: 0, 1, 2 (so a
// tile is made of >= 64-byte contiguous chunks), then the qubits of the
// remaining gates in order of first appearance, then the lowest unused ones.
std::vector<std::pair<uint64_t, std::vector<int>>> schedule(const std::vector<HGate>& g, int n, int m)
{
    std::vector<std::pair<uint64_t, std::vector<int>>> out;
    const int N = (int)g.size();
    if (n <= m) {
        for (int s = 0; s < N || (s == 0 && N == 0); s += kMaxPassOps) {
            std::vector<int> ops;
            for (int o = s; o < N && o < s + kMaxPassOps; ++o)
                ops.push_back(o);
            out.push_back({(n >= 64 ? ~0ull : ((1ull << n) - 1)), ops});
            if (N == 0)
                break;
        }
        return out;
    }
    std::vector<bool> done(N, false);
    int left = N;
    while (left > 0) {
        uint64_t B = 0x7;
        for (int o = 0; o < N && popc(B) < m; ++o) {
            if (done[o])
                continue;
            uint64_t q = gate_qubits(g[o]) & ~B;
            while (q && popc(B) < m) {
                B |= q & (~q + 1);
                q &= q - 1;
            }
        }
        for (int b = 0; b < n && popc(B) < m; ++b)
            B |= 1ull << b;
        std::vector<int> ops;
        uint64_t blocked = 0;
        for (int o = 0; o < N; ++o) {
            if (done[o])
                continue;
            const uint64_t q = gate_qubits(g[o]);
            if ((q & ~B) == 0 && (q & blocked) == 0 && (int)ops.size() < kMaxPassOps) {
                ops.push_back(o);
                done[o] = true;
                --left;
            } else {
                blocked |= q;
            }
        }
        out.push_back({B, ops});
    }
    return out;
}

}  // namespace

void compile_tile_program(const std::vector<HGate>& gates, int n, int m, TileProgram& out)
{
    out = TileProgram{};
    for (const auto& pr : schedule(gates, n, m)) {
        const uint64_t B = pr.first;
        DPass P{};
        P.bmask = B;
        P.step_off = (int)out.steps.size();
        P.op_off = (int)out.ops.size();
        P.nops = (int)pr.second.size();
        P.slot_base = (int)out.slot_param.size();
        // steps: consecutive gates whose (tile-local) qubits fit 3 qubits
        size_t i = 0;
        const std::vector<int>& ops = pr.second;
        while (i < ops.size()) {
            uint32_t S = 0;
            size_t j = i;
            while (j < ops.size() && (int)(j - i) < kMaxStepOps) {
                const HGate& h = gates[ops[j]];
                uint32_t q = 1u << local_bit(B, h.t);
                if (h.nc > 0)
                    q |= 1u << local_bit(B, h.c0);
                if (h.nc > 1)
                    q |= 1u << local_bit(B, h.c1);
                if (popc(S | q) > kStepQubits)
                    break;
                S |= q;
                ++j;
            }
            DStep st{};
            st.nq = (uint8_t)popc(S);
            int k = 0;
            for (int b = 0; b < 32; ++b)
                if ((S >> b) & 1)
                    st.q[k++] = (uint8_t)b;
            st.o0 = (int16_t)(out.ops.size() - P.op_off);
            auto stepbit = [&](int q_global) {
                const int lb = local_bit(B, q_global);
                for (int x = 0; x < st.nq; ++x)
                    if (st.q[x] == lb)
                        return x;
                return -1;
            };
            for (size_t o = i; o < j; ++o) {
                const HGate& h = gates[ops[o]];
                DOp d{};
                d.kind = (uint8_t)h.kind;
                d.tq = (uint8_t)stepbit(h.t);
                d.cm = (uint8_t)((h.nc > 0 ? 1 << stepbit(h.c0) : 0) | (h.nc > 1 ? 1 << stepbit(h.c1) : 0));
                d.param = h.param;
                d.mat = h.mat;
                d.slot = -1;
                if (h.kind != 0) {
                    d.slot = P.nrot++;
                    out.slot_param.push_back(h.param);
                }
                out.ops.push_back(d);
            }
            st.o1 = (int16_t)(out.ops.size() - P.op_off);
            out.steps.push_back(st);
            i = j;
        }
        P.nsteps = (int)out.steps.size() - P.step_off;
        std::vector<int> ps(out.slot_param.begin() + P.slot_base, out.slot_param.end());
        std::sort(ps.begin(), ps.end());
        P.shared = std::adjacent_find(ps.begin(), ps.end()) != ps.end() ? 1 : 0;
        out.passes.push_back(P);
    }
}

}  // namespace qsv
