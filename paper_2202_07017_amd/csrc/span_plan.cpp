// Host planner of the span passes (kernels_span.hip).
//
// Strings are grouped by x mask (first appearance order); a pass takes up to
// kSpanDirs masks whose parts on qubits >= 6 are linearly independent, with
// all their strings (a mask with more strings than a pass holds continues in
// the next pass).  A pass with fewer masks is padded with single-qubit
// directions, which keeps every tile at 2^11 amplitudes.
#include <algorithm>
#include <cstdint>
#include <unordered_map>
#include <vector>

#include "qsv_span_plan.h"

namespace qsv {

namespace {

constexpr uint64_t kLaneMask = (1ull << kSpanLaneQubits) - 1;

int par(uint64_t v) { return __builtin_popcountll(v) & 1; }

// Reduced row echelon form over GF(2) of the parts of the directions above
// the lane qubits: each row has a pivot bit that no other row has.
struct Echelon {
    std::vector<uint64_t> row;
    std::vector<int> piv;
    // v reduced by the rows (zero iff v lies in their span)
    uint64_t reduce(uint64_t v) const
    {
        for (size_t j = 0; j < row.size(); ++j)
            if ((v >> piv[j]) & 1)
                v ^= row[j];
        return v;
    }
    void add(uint64_t v)  // v already reduced and nonzero
    {
        const int p = __builtin_ctzll(v);
        for (uint64_t& r : row)
            if ((r >> p) & 1)
                r ^= v;
        row.push_back(v);
        piv.push_back(p);
    }
};

}  // namespace

void plan_span_passes(const qsv_pauli_sum* H, int n, std::vector<SpanPassK>& out, std::vector<int>& rest)
{
    std::vector<uint64_t> masks;
    std::vector<std::vector<int>> strings;
    std::unordered_map<uint64_t, size_t> index;
    for (int j = 0; j < H->nterms; ++j) {
        const uint64_t x = H->x_mask[j];
        if ((x & ~kLaneMask) == 0) {
            rest.push_back(j);
            continue;
        }
        auto it = index.find(x);
        if (it == index.end()) {
            it = index.emplace(x, masks.size()).first;
            masks.push_back(x);
            strings.emplace_back();
        }
        strings[it->second].push_back(j);
    }
    std::vector<size_t> pos(masks.size(), 0);  // strings of each mask already placed
    size_t left = masks.size();
    while (left > 0) {
        Echelon E;
        std::vector<uint64_t> dirs;
        std::vector<std::pair<int, int>> take;  // (string, direction)
        for (size_t m = 0; m < masks.size() && dirs.size() < (size_t)kSpanDirs; ++m) {
            if (pos[m] == strings[m].size() || (int)take.size() == kMaxSpanTerms)
                continue;
            const uint64_t v = E.reduce(masks[m] & ~kLaneMask);
            if (v == 0)
                continue;  // dependent on this pass's directions: a later pass
            E.add(v);
            const int d = (int)dirs.size();
            dirs.push_back(masks[m]);
            while (pos[m] < strings[m].size() && (int)take.size() < kMaxSpanTerms)
                take.push_back({strings[m][pos[m]++], d});
            if (pos[m] == strings[m].size())
                --left;
        }
        // pad with single qubits >= 6 outside the span so far (a qubit that
        // is no pivot always is: the rows have no bit at it after reduction
        // that a combination of them could cancel)
        for (int q = kSpanLaneQubits; q < n && dirs.size() < (size_t)kSpanDirs; ++q) {
            const uint64_t v = E.reduce(1ull << q);
            if (v == 0)
                continue;
            E.add(v);
            dirs.push_back(1ull << q);
        }
        std::vector<int> tileq(E.piv);
        for (int b = 0; b < kSpanLaneQubits; ++b)
            tileq.push_back(b);
        std::sort(tileq.begin(), tileq.end());
        SpanPassK k{};
        k.ntiles = 1ull << (n - kSpanTileQubits);
        for (int j = 0; j < kSpanTileQubits; ++j)
            k.low[j] = (1ull << tileq[j]) - 1;
        for (int j = 0; j < kSpanDirs; ++j)
            k.d[j] = dirs[j];
        std::vector<STerm> ts;
        for (const auto& pr : take) {
            const int j = pr.first, d = pr.second;
            const uint64_t x = H->x_mask[j], z = H->z_mask[j];
            const int ylo = __builtin_popcountll(x & z) & 3;
            STerm t{};
            t.z = z;
            t.dir = d;
            t.im = ylo & 1;
            // 2 Re w (ylo 0: +, 2: -) or 2 Im w (ylo 1: -, 3: +), w = conj(psi_b) psi_a
            t.c = (ylo == 1 || ylo == 2) ? -2.0 * H->coeff[j] : 2.0 * H->coeff[j];
            uint32_t zr = 0;
            for (int q = 0; q < kSpanDirs; ++q)
                zr |= (uint32_t)par(z & dirs[q]) << q;
            for (int i = 0; i < 16; ++i) {
                const uint32_t r = ((uint32_t)(i >> d) << (d + 1)) | ((uint32_t)i & ((1u << d) - 1));
                t.sgn |= (uint32_t)par(zr & r) << i;
            }
            ts.push_back(t);
        }
        std::stable_sort(ts.begin(), ts.end(), [](const STerm& a, const STerm& b) {
            return a.dir != b.dir ? a.dir < b.dir : a.im < b.im;
        });
        k.nt = (int)ts.size();
        for (int i = 0; i < k.nt; ++i)
            k.t[i] = ts[i];
        for (int g = 0, i = 0; g <= 2 * kSpanDirs; ++g) {
            while (i < k.nt && 2 * k.t[i].dir + k.t[i].im < g)
                ++i;
            k.koff[g] = i;
        }
        out.push_back(k);
    }
}

}  // namespace qsv
