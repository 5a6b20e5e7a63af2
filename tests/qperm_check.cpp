// CPU checker of the qubit permutation planner
// (paper_2202_07017_amd/csrc/qperm_plan.cpp).
//
// Reads "n rl nswaps" and then nswaps pairs "a b" from stdin.  It applies the
// swaps one after another to the index vector 0..2^n-1 (a swap exchanges two
// bits of every index), plans the composed permutation, checks each pass's
// structure (q an involution, tile bits closed under q and holding q of the
// row bits, cmap consistent with q), then replays each pass the way the GPU
// kernel walks it (one tile, or a tile and its image, per workgroup; output
// tile-local index l takes source tile-local index s with bit k of s = bit
// cmap[k] of l) and requires every index to be written exactly once per pass
// and the final vector to equal the sequential result.  Prints
// "passes <count>".  Exit 0 on success, 1 with a message otherwise.
#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <utility>
#include <vector>

#include "qsv_qperm_plan.h"

static void require(bool ok, const char* what)
{
    if (!ok) {
        std::fprintf(stderr, "%s\n", what);
        std::exit(1);
    }
}

int main()
{
    int n = 0, rl = 0, m = 0;
    if (std::scanf("%d %d %d", &n, &rl, &m) != 3)
        return 1;
    std::vector<std::pair<int, int>> sw(m);
    for (auto& s : sw)
        if (std::scanf("%d %d", &s.first, &s.second) != 2)
            return 1;
    const uint64_t N = 1ull << n;
    std::vector<uint32_t> ref(N), cur(N), tmp(N);
    for (uint64_t i = 0; i < N; ++i)
        ref[i] = cur[i] = (uint32_t)i;
    for (const auto& s : sw) {
        for (uint64_t j = 0; j < N; ++j) {
            const uint64_t a = (j >> s.first) & 1, b = (j >> s.second) & 1;
            const uint64_t i = (j & ~((1ull << s.first) | (1ull << s.second))) | (a << s.second) | (b << s.first);
            tmp[j] = ref[i];
        }
        ref.swap(tmp);
    }
    const std::vector<int> Q = qsv::compose_swaps(sw, n);
    std::vector<qsv::QPermPass> passes;
    qsv::plan_qubit_permutation(Q, n, rl, passes);
    for (const qsv::QPermPass& P : passes) {
        require(P.n == n && P.rl == rl && P.hb >= 0 && P.hb <= rl, "pass geometry");
        std::vector<int> T;
        std::vector<char> in_t(n, 0);
        for (int k = 0; k < rl; ++k)
            T.push_back(k);
        for (int k = 0; k < P.hb; ++k) {
            require(P.hpos[k] >= rl && P.hpos[k] < n && (k == 0 || P.hpos[k] > P.hpos[k - 1]), "tile bits ascending");
            T.push_back(P.hpos[k]);
        }
        for (int t : T)
            in_t[t] = 1;
        for (int b = 0; b < n; ++b) {
            require(P.q[b] >= 0 && P.q[b] < n && P.q[P.q[b]] == b, "q is an involution");
            require(in_t[b] == in_t[P.q[b]], "tile bits closed under q");
        }
        const int tb = rl + P.hb;
        for (int k = 0; k < tb; ++k)
            require(P.cmap[k] >= 0 && P.cmap[k] < tb && T[P.cmap[k]] == P.q[T[k]], "cmap");
        require(P.ntiles == (1ull << (n - tb)), "tile count");
        std::vector<int> wseen(n - tb, 0);
        for (int p = 0; p < n - tb; ++p) {
            require(P.wsrc[p] >= 0 && P.wsrc[p] < n - tb, "tile order bit");
            ++wseen[P.wsrc[p]];
        }
        for (int p = 0; p < n - tb; ++p)
            require(wseen[p] == 1, "tile order is not a bijection");
        auto dep = [&](uint64_t l) {
            uint64_t o = 0;
            for (int k = 0; k < tb; ++k)
                o |= ((l >> k) & 1ull) << T[k];
            return o;
        };
        auto image = [&](uint64_t x) {  // bit b of the image = bit q[b] of x
            uint64_t o = 0;
            for (int b = 0; b < n; ++b)
                o |= ((x >> P.q[b]) & 1ull) << b;
            return o;
        };
        std::vector<unsigned char> hit(N, 0);
        for (uint64_t w = 0; w < P.ntiles; ++w) {
            uint64_t t = 0;  // the tile of workgroup w
            for (int p = 0; p < n - tb; ++p)
                t |= ((w >> P.wsrc[p]) & 1ull) << p;
            uint64_t ba = t;  // insert zeros at the tile bits, ascending
            std::vector<int> Ts(T);
            std::sort(Ts.begin(), Ts.end());
            for (int p : Ts)
                ba = ((ba >> p) << (p + 1)) | (ba & ((1ull << p) - 1));
            const uint64_t bb = image(ba);
            require((bb & dep((1ull << tb) - 1)) == 0, "partner base outside the tile bits");
            if (bb < ba)
                continue;
            for (uint64_t l = 0; l < (1ull << tb); ++l) {
                uint64_t s = 0;
                for (int k = 0; k < tb; ++k)
                    s |= ((l >> P.cmap[k]) & 1ull) << k;
                const uint64_t d1 = ba | dep(l), s1 = bb | dep(s);
                require(hit[d1] == 0, "index written twice");
                hit[d1] = 1;
                tmp[d1] = cur[s1];
                if (bb != ba) {
                    const uint64_t d2 = bb | dep(l), s2 = ba | dep(s);
                    require(hit[d2] == 0, "index written twice");
                    hit[d2] = 1;
                    tmp[d2] = cur[s2];
                }
            }
        }
        for (uint64_t i = 0; i < N; ++i)
            require(hit[i] == 1, "index not written");
        cur.swap(tmp);
    }
    for (uint64_t i = 0; i < N; ++i)
        require(cur[i] == ref[i], "result differs from the swaps applied in order");
    std::printf("passes %d\n", (int)passes.size());
    return 0;
}
