// Host planner of the register-tile Pauli passes (kernels_rpass.hip).
//
// Strings are sorted into diagonal ones, ones whose x mask is one or two of
// qubits 0..4, ones whose x mask is one or two qubits above 4, ones whose x
// mask is qubit 4 and one qubit above, and the rest (for the LDS-tile
// passes).  The qubits above 4 are grouped, in term order, into register
// sets of kRegQubits qubits, each set one pass; the first pass also takes
// the strings on qubits 0..4 and those with qubit 4 and one of its lane
// qubits (after an in-wave transpose), and the second (or only) one the
// diagonal strings.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "qsv_rpass_plan.h"

namespace qsv {

void plan_reg_passes(const qsv_pauli_sum* H, int n, std::vector<RegPassK>& out, std::vector<int>& rest)
{
    const uint64_t lowq = (1ull << (kRegLanes - 1)) - 1;  // qubits 0..4
    std::vector<int> diag, low, high, cross;
    // diagonal strings; strings whose x mask is one or two of qubits 0..4;
    // strings whose x mask is one or two qubits above 4 (both with a z check
    // once the register qubits are known, below); strings whose x mask is
    // qubit 4 and one qubit above (cross-lane candidates of the first pass);
    // the rest go to the LDS-tile passes
    for (int j = 0; j < H->nterms; ++j) {
        const uint64_t x = H->x_mask[j];
        const int px = __builtin_popcountll(x);
        if (x == 0)
            diag.push_back(j);
        else if (px <= 2 && (x & ~lowq) == 0)
            low.push_back(j);
        else if (px <= 2 && (x & lowq) == 0)
            high.push_back(j);
        else if (px == 2 && (x & lowq) == 16)
            cross.push_back(j);
        else
            rest.push_back(j);
    }
    // register sets
    std::vector<std::pair<uint64_t, std::vector<int>>> sets;
    std::vector<bool> used(high.size(), false);
    for (size_t i = 0; i < high.size(); ++i) {
        if (used[i])
            continue;
        uint64_t Q = 0;
        std::vector<int> take;
        for (size_t k = i; k < high.size(); ++k) {
            if (used[k])
                continue;
            const uint64_t x = H->x_mask[high[k]];
            if (__builtin_popcountll(Q | x) <= kRegQubits) {
                Q |= x;
                take.push_back(high[k]);
                used[k] = true;
            }
        }
        sets.push_back({Q, take});
    }
    if (sets.empty() && (!diag.empty() || !low.empty() || !cross.empty()))
        sets.push_back({0, {}});
    if (sets.empty())
        rest.insert(rest.end(), cross.begin(), cross.end());
    for (size_t si = 0; si < sets.size(); ++si) {
        uint64_t Q = sets[si].first;
        // fill the register set up to kRegQubits qubits with the lowest free ones >= 5
        for (int q = kRegLanes - 1; q < n && __builtin_popcountll(Q) < kRegQubits; ++q)
            Q |= 1ull << q;
        std::vector<int> qreg;
        for (int q = 0; q < n; ++q)
            if ((Q >> q) & 1)
                qreg.push_back(q);
        int h = kRegLanes - 1;
        while ((Q >> h) & 1)
            ++h;
        std::vector<int> tileq = qreg;
        for (int b = 0; b < kRegLanes - 1; ++b)
            tileq.push_back(b);
        tileq.push_back(h);
        std::sort(tileq.begin(), tileq.end());
        RegPassK k{};
        k.ntiles = 1ull << (n - kRegTileQubits);
        for (int j = 0; j < kRegTileQubits; ++j)
            k.low[j] = (1ull << tileq[j]) - 1;
        for (int j = 0; j < kRegQubits; ++j)
            k.qstride[j] = 1ull << qreg[j];
        for (int b = 0; b < kRegLanes - 1; ++b)
            k.lanepos[b] = b;
        k.lanepos[kRegLanes - 1] = h;
        auto comp_reg = [&](uint64_t v) {
            uint32_t o = 0;
            for (int j = 0; j < kRegQubits; ++j)
                if ((v >> qreg[j]) & 1)
                    o |= 1u << j;
            return o;
        };
        auto comp_lane = [&](uint64_t v) {
            uint32_t o = 0;
            for (int b = 0; b < kRegLanes; ++b)
                if ((v >> k.lanepos[b]) & 1)
                    o |= 1u << b;
            return o;
        };
        auto comp_lane2 = [&](uint64_t v) {  // transposed lane roles
            uint32_t o = (uint32_t)((v >> h) & 1);
            for (int j = 0; j < kRegQubits; ++j)
                if ((v >> qreg[j]) & 1)
                    o |= 1u << (1 + j);
            return o;
        };
        uint64_t tilemask = 0;
        for (int q : tileq)
            tilemask |= 1ull << q;
        auto term = [&](int j, int phase) {
            RTerm t{};
            const uint64_t x = H->x_mask[j], z = H->z_mask[j];
            t.z = z;
            t.c = H->coeff[j];
            t.ylo = __builtin_popcountll(x & z) & 3;
            if (phase >= 2) {
                t.xr = (uint32_t)(x & lowq);
                t.zr = (uint32_t)(z & lowq);
                t.zl = comp_lane2(z);
                if (phase == 3)
                    t.xl = comp_lane2(x & ~lowq);
            } else {
                t.xr = comp_reg(x);
                t.zr = comp_reg(z);
                t.zl = comp_lane(z);
            }
            if (phase != 0) {
                // 2 Re w times i^ylo's sign (ylo 0: +, 2: -), or 2 Im w (ylo 1:
                // -, 3: +); the half sum s1 (lower x bit of the pair's first
                // member set) also takes the register part of the z sign
                const double cf = (t.ylo == 1 || t.ylo == 2) ? -2.0 * t.c : 2.0 * t.c;
                const bool two = (t.xr & (t.xr - 1)) != 0;
                const bool slb = two && (t.zr & t.xr & (0u - t.xr)) != 0;
                t.c = cf;
                t.c2 = slb ? -cf : cf;
            }
            return t;
        };
        // strings of one phase with the same x mask, Re/Im kind, lane z bits
        // and z bits outside the tile share every sign but the register one
        // (already in c2): one term with the summed coefficients
        auto merge = [&](std::vector<RTerm>& v) {
            std::vector<RTerm> out;
            for (const RTerm& t : v) {
                bool done = false;
                for (RTerm& u : out)
                    if (u.xr == t.xr && u.xl == t.xl && ((u.ylo ^ t.ylo) & 1) == 0 && u.zl == t.zl &&
                        (u.z & ~tilemask) == (t.z & ~tilemask)) {
                        u.c += t.c;
                        u.c2 += t.c2;
                        done = true;
                        break;
                    }
                if (!done)
                    out.push_back(t);
            }
            v.swap(out);
        };
        // launches of <= kMaxRegTerms terms with this geometry: the first
        // register set also takes the diagonal and low-qubit strings
        std::vector<std::pair<int, int>> items;  // (term, phase 0 diag / 1 register / 2 low / 3 cross-lane)
        // the diagonal terms ride with the second register set when there is
        // one and the first also takes the transposed low-qubit strings
        // (measured: TFIM at n = 30, complex64 7.55 -> 7.15 ms, complex128
        // 14.5 -> 13.1 ms)
        const size_t dset = (sets.size() > 1 && !low.empty()) ? 1 : 0;
        if (si == dset) {
            for (int j : diag)
                items.push_back({j, 0});
        }
        // a string's x mask must be one register bit of its phase or two
        // neighbouring ones, and its z bits on those register qubits must lie
        // in the x mask (the pass signs pairs by the lower x bit only); other
        // strings go to the LDS-tile passes
        auto reg_ok = [](uint32_t xr) {
            return xr != 0 && ((xr & (xr - 1)) == 0 || (xr >> __builtin_ctz(xr)) == 3u);
        };
        for (int j : sets[si].second) {
            if (reg_ok(comp_reg(H->x_mask[j])) && (H->z_mask[j] & Q & ~H->x_mask[j]) == 0)
                items.push_back({j, 1});
            else
                rest.push_back(j);
        }
        if (si == 0) {
            for (int j : low) {
                if (reg_ok((uint32_t)(H->x_mask[j] & lowq)) && (H->z_mask[j] & lowq & ~H->x_mask[j]) == 0)
                    items.push_back({j, 2});
                else
                    rest.push_back(j);
            }
            // qubit 4 with a qubit that is a lane qubit after the transpose
            // (h or a register qubit of this set): the partner is register
            // r ^ 16 of another lane; z on qubits 0..3 would need a register
            // sign the pass does not apply
            const uint64_t lanes2 = Q | (1ull << h);
            for (int j : cross) {
                const uint64_t x = H->x_mask[j];
                if ((x & ~lowq & lanes2) != 0 && (H->z_mask[j] & lowq & ~x) == 0)
                    items.push_back({j, 3});
                else
                    rest.push_back(j);
            }
        }
        size_t pos = 0;
        do {
            RegPassK L = k;
            int nt = 0, cnt[4] = {0, 0, 0, 0};
            std::vector<RTerm> byphase[4];
            while (pos < items.size() && nt < kMaxRegTerms) {
                byphase[items[pos].second].push_back(term(items[pos].first, items[pos].second));
                ++cnt[items[pos].second];
                ++nt;
                ++pos;
            }
            // diagonal terms sorted by register mask, with group offsets;
            // in the other phases single-qubit X strings without Z or Y
            // factors (the short pair sums) come first
            std::stable_sort(byphase[0].begin(), byphase[0].end(),
                             [](const RTerm& x, const RTerm& y) { return x.zr < y.zr; });
            auto plain = [](const RTerm& t) { return t.z == 0 && __builtin_popcount(t.xr) == 1; };
            int nplain[3] = {0, 0, 0};
            for (int ph = 1; ph < 4; ++ph) {
                merge(byphase[ph]);
                cnt[ph] = (int)byphase[ph].size();
                if (ph < 3) {
                    std::stable_partition(byphase[ph].begin(), byphase[ph].end(), plain);
                    nplain[ph] = (int)std::count_if(byphase[ph].begin(), byphase[ph].end(), plain);
                }
            }
            for (int m = 0, q = 0; m <= (1 << kRegQubits); ++m) {
                while (q < (int)byphase[0].size() && (int)byphase[0][q].zr < m)
                    ++q;
                L.mofs[m] = q;
            }
            int w = 0;
            for (int ph = 0; ph < 4; ++ph)
                for (const RTerm& t : byphase[ph])
                    L.t[w++] = t;
            L.nd = cnt[0];
            L.ns1 = cnt[0] + nplain[1];
            L.n1 = cnt[0] + cnt[1];
            L.ns2 = L.n1 + nplain[2];
            L.nc = L.n1 + cnt[2];
            L.nt = L.nc + cnt[3];
            out.push_back(L);
        } while (pos < items.size());
    }
}

}  // namespace qsv
