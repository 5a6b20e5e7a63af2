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

// Gates (indices into `rest`, circuit order) that a pass with tile qubits B
// takes: every gate whose qubits are tile qubits and that no earlier gate
// left behind blocks (a gate left behind blocks its qubits for every later
// gate, so the taken gates commute with all of them), at most cap gates.
int take(const std::vector<uint64_t>& rest, uint64_t B, int cap, std::vector<int>* out)
{
    uint64_t blocked = 0;
    int c = 0;
    for (int o = 0; o < (int)rest.size(); ++o) {
        const uint64_t q = rest[o];
        if ((q & ~B) == 0 && (q & blocked) == 0 && c < cap) {
            ++c;
            if (out)
                out->push_back(o);
        } else {
            blocked |= q;
        }
    }
    return c;
}

// Passes.  Tile qubits: 0, 1, 2 (so a tile is made of >= 64-byte contiguous
// chunks), then one qubit at a time the one that lets the pass take the most
// gates; where no single qubit adds a gate, the first qubit outside the tile
// of the first remaining gate.
std::vector<std::pair<uint64_t, std::vector<int>>> schedule(const std::vector<HGate>& g, int n, int m,
                                                            int cap)
{
    std::vector<std::pair<uint64_t, std::vector<int>>> out;
    const int N = (int)g.size();
    if (n <= m) {
        for (int s = 0; s < N || (s == 0 && N == 0); s += cap) {
            std::vector<int> ops;
            for (int o = s; o < N && o < s + cap; ++o)
                ops.push_back(o);
            out.push_back({(n >= 64 ? ~0ull : ((1ull << n) - 1)), ops});
            if (N == 0)
                break;
        }
        return out;
    }
    std::vector<int> idx(N);
    std::vector<uint64_t> rest(N);
    for (int o = 0; o < N; ++o) {
        idx[o] = o;
        rest[o] = gate_qubits(g[o]);
    }
    while (!rest.empty()) {
        uint64_t B = 0x7;
        while (popc(B) < m) {
            const int base = take(rest, B, cap, nullptr);
            int best = -1, gain = base;
            for (int q = 0; q < n; ++q) {
                if ((B >> q) & 1)
                    continue;
                const int c = take(rest, B | (1ull << q), cap, nullptr);
                if (c > gain) {
                    gain = c;
                    best = q;
                }
            }
            for (size_t o = 0; o < rest.size() && best < 0; ++o)
                if (rest[o] & ~B)
                    best = __builtin_ctzll(rest[o] & ~B);
            for (int q = 0; q < n && best < 0; ++q)
                if (!((B >> q) & 1))
                    best = q;
            B |= 1ull << best;
        }
        std::vector<int> sel;
        if (take(rest, B, cap, &sel) == 0) {
            // (only when the first remaining gate's qubits do not fit beside
            // 0, 1, 2, i.e. m < 6) its qubits first, then the lowest others
            B = rest[0];
            for (int b = 0; b < n && popc(B) < m; ++b)
                B |= 1ull << b;
            take(rest, B, cap, &sel);
        }
        std::vector<int> ops;
        std::vector<bool> taken(rest.size(), false);
        for (int o : sel) {
            ops.push_back(idx[o]);
            taken[o] = true;
        }
        size_t w = 0;
        for (size_t o = 0; o < rest.size(); ++o)
            if (!taken[o]) {
                rest[w] = rest[o];
                idx[w] = idx[o];
                ++w;
            }
        rest.resize(w);
        idx.resize(w);
        out.push_back({B, ops});
    }
    return out;
}

}  // namespace

void compile_tile_program(const std::vector<HGate>& gates, int n, int m, int cap, TileProgram& out)
{
    out = TileProgram{};
    for (const auto& pr : schedule(gates, n, m, cap)) {
        const uint64_t B = pr.first;
        DPass P{};
        P.bmask = B;
        P.step_off = (int)out.steps.size();
        P.op_off = (int)out.ops.size();
        P.nops = (int)pr.second.size();
        P.slot_base = (int)out.slot_param.size();
        auto local = [&](const HGate& h) {
            uint32_t q = 1u << local_bit(B, h.t);
            if (h.nc > 0)
                q |= 1u << local_bit(B, h.c0);
            if (h.nc > 1)
                q |= 1u << local_bit(B, h.c1);
            return q;
        };
        // Steps: the first remaining gate, then every later one whose qubits
        // fit the step's three and that commutes with the gates passed over
        // (no shared qubit), at most kMaxStepOps; gates keep circuit order.
        std::vector<int> rest = pr.second;
        while (!rest.empty()) {
            uint32_t S = 0, blocked = 0;
            std::vector<int> step;
            std::vector<int> left;
            for (int o : rest) {
                const uint32_t q = local(gates[o]);
                if ((int)step.size() < kMaxStepOps && (q & blocked) == 0 && popc(S | q) <= kStepQubits) {
                    S |= q;
                    step.push_back(o);
                } else {
                    blocked |= q;
                    left.push_back(o);
                }
            }
            rest.swap(left);
            // pad to three qubits with the highest free tile positions: the
            // executor always works on groups of 8 amplitudes
            for (int b = popc(B) - 1; b >= 0 && popc(S) < kStepQubits; --b)
                S |= 1u << b;
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
            for (int o : step) {
                const HGate& h = gates[o];
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
        }
        P.nsteps = (int)out.steps.size() - P.step_off;
        std::vector<int> ps(out.slot_param.begin() + P.slot_base, out.slot_param.end());
        std::sort(ps.begin(), ps.end());
        P.shared = std::adjacent_find(ps.begin(), ps.end()) != ps.end() ? 1 : 0;
        out.passes.push_back(P);
    }
}

}  // namespace qsv
