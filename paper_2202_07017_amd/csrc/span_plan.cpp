// Host planner of the span passes (kernels_span.hip).
//
// Strings whose x mask has a qubit at 6 or above are grouped by x mask
// (first appearance order); a pass takes up to kSpanDirs masks whose parts
// above qubit 5 are linearly independent, with their strings (a mask with
// more strings than a pass holds continues in the next pass).  Lane strings
// (x mask on qubits 0..5) and diagonal strings then go to the pass with the
// least estimated arithmetic that has room.  A pass with fewer masks is
// padded with single-qubit directions, which keeps every tile at 2^11
// amplitudes.
#include <algorithm>
#include <cstdint>
#include <unordered_map>
#include <vector>

#include "qsv_span_plan.h"

namespace qsv {

namespace {

constexpr uint64_t kLaneMask = (1ull << kSpanLaneQubits) - 1;

// estimated arithmetic per lane and tile, in units of one direction string
// (16 pair products): a lane string has 32 products and an exchange, a
// diagonal string a table read once the pass has its 32-point transform
constexpr double kLoadDir = 1.0, kLoadLane = 2.5, kLoadDiag = 0.1, kLoadTransform = 2.0;

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

struct Draft {
    Echelon E;
    std::vector<uint64_t> dirs;
    std::vector<std::pair<int, int>> take;  // (string, direction; -1: lane or diagonal string)
    double load = 0.0;
    bool diag = false;
};

}  // namespace

void plan_span_passes(const qsv_pauli_sum* H, int n, std::vector<SpanPassK>& out)
{
    std::vector<uint64_t> masks;
    std::vector<std::vector<int>> strings;
    std::unordered_map<uint64_t, size_t> index;
    std::vector<int> lanes, diags;
    for (int j = 0; j < H->nterms; ++j) {
        const uint64_t x = H->x_mask[j];
        if (x == 0) {
            diags.push_back(j);
            continue;
        }
        if ((x & ~kLaneMask) == 0) {
            lanes.push_back(j);
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
    std::vector<Draft> drafts;
    std::vector<size_t> pos(masks.size(), 0);  // strings of each mask already placed
    size_t left = masks.size();
    while (left > 0) {
        Draft D;
        for (size_t m = 0; m < masks.size() && D.dirs.size() < (size_t)kSpanDirs; ++m) {
            if (pos[m] == strings[m].size() || (int)D.take.size() == kMaxSpanTerms)
                continue;
            const uint64_t v = D.E.reduce(masks[m] & ~kLaneMask);
            if (v == 0)
                continue;  // dependent on this pass's directions: a later pass
            D.E.add(v);
            const int d = (int)D.dirs.size();
            D.dirs.push_back(masks[m]);
            while (pos[m] < strings[m].size() && (int)D.take.size() < kMaxSpanTerms) {
                D.take.push_back({strings[m][pos[m]++], d});
                D.load += kLoadDir;
            }
            if (pos[m] == strings[m].size())
                --left;
        }
        drafts.push_back(D);
    }
    auto place = [&](int j, bool diag) {
        Draft* best = nullptr;
        for (Draft& D : drafts)
            if ((int)D.take.size() < kMaxSpanTerms && (!best || D.load < best->load))
                best = &D;
        if (!best) {
            drafts.emplace_back();
            best = &drafts.back();
        }
        best->take.push_back({j, -1});
        best->load += diag ? kLoadDiag : kLoadLane;
        if (diag && !best->diag) {
            best->diag = true;
            best->load += kLoadTransform;
        }
    };
    for (int j : lanes)
        place(j, false);
    for (int j : diags)
        place(j, true);
    for (Draft& D : drafts) {
        // pad with single qubits >= 6 outside the span so far
        for (int q = kSpanLaneQubits; q < n && D.dirs.size() < (size_t)kSpanDirs; ++q) {
            const uint64_t v = D.E.reduce(1ull << q);
            if (v == 0)
                continue;
            D.E.add(v);
            D.dirs.push_back(1ull << q);
        }
        std::vector<int> tileq(D.E.piv);
        for (int b = 0; b < kSpanLaneQubits; ++b)
            tileq.push_back(b);
        std::sort(tileq.begin(), tileq.end());
        SpanPassK k{};
        k.ntiles = 1ull << (n - kSpanTileQubits);
        for (int j = 0; j < kSpanTileQubits; ++j)
            k.low[j] = (1ull << tileq[j]) - 1;
        for (int j = 0; j < kSpanDirs; ++j)
            k.d[j] = D.dirs[j];
        std::vector<std::pair<int, STerm>> ts;  // (sort key, term); lane strings by xl within their group
        for (const auto& pr : D.take) {
            const int j = pr.first, d = pr.second;
            const uint64_t x = H->x_mask[j], z = H->z_mask[j];
            const int ylo = __builtin_popcountll(x & z) & 3;
            STerm t{};
            t.z = z;
            t.im = ylo & 1;
            for (int q = 0; q < kSpanDirs; ++q)
                t.zr |= (uint32_t)par(z & D.dirs[q]) << q;
            // Re w (ylo 0: +, 2: -) or Im w (ylo 1: -, 3: +), w = conj(psi_b) psi_a
            const double sc = (ylo == 1 || ylo == 2) ? -H->coeff[j] : H->coeff[j];
            int key;
            if (x == 0) {
                t.dir = -1;
                t.c = H->coeff[j];
                key = kSpanGroups + (int)t.zr;
            } else if (d < 0) {
                t.dir = -1;
                t.xl = (uint32_t)x;
                t.c = sc;
                for (int r = 0; r < (1 << kSpanDirs); ++r)
                    t.sgn |= (uint32_t)par(t.zr & (uint32_t)r) << r;
                key = 2 * kSpanDirs + t.im;
            } else {
                t.dir = d;
                t.c = 2.0 * sc;  // each unordered pair once
                for (int i = 0; i < (1 << (kSpanDirs - 1)); ++i) {
                    const uint32_t r = ((uint32_t)(i >> d) << (d + 1)) | ((uint32_t)i & ((1u << d) - 1));
                    t.sgn |= (uint32_t)par(t.zr & r) << i;
                }
                key = 2 * d + t.im;
            }
            ts.push_back({key, t});
        }
        std::stable_sort(ts.begin(), ts.end(), [](const std::pair<int, STerm>& a, const std::pair<int, STerm>& b) {
            return a.first != b.first ? a.first < b.first : a.second.xl < b.second.xl;
        });
        k.nt = (int)ts.size();
        for (int i = 0; i < k.nt; ++i)
            k.t[i] = ts[i].second;
        for (int g = 0, i = 0; g <= kSpanGroups + (1 << kSpanDirs); ++g) {
            while (i < k.nt && ts[i].first < g)
                ++i;
            if (g <= kSpanGroups)
                k.koff[g] = i;
            if (g >= kSpanGroups)
                k.mofs[g - kSpanGroups] = i;
        }
        out.push_back(k);
    }
}

}  // namespace qsv
