// Host planner of qubit permutation passes (declared in qsv_qperm_plan.h).
#include "qsv_qperm_plan.h"

#include <algorithm>

namespace qsv {

std::vector<int> compose_swaps(const std::vector<std::pair<int, int>>& swaps, int n)
{
    // After swaps s_1..s_m the state is psi_m[j] = psi[s_1(s_2(...s_m(j)))];
    // appending s means composing it on the inside, which relabels the
    // source bits: Q[b] -> s(Q[b]).
    std::vector<int> Q(n);
    for (int b = 0; b < n; ++b)
        Q[b] = b;
    for (const auto& s : swaps)
        for (int b = 0; b < n; ++b) {
            if (Q[b] == s.first)
                Q[b] = s.second;
            else if (Q[b] == s.second)
                Q[b] = s.first;
        }
    return Q;
}

namespace {

QPermPass make_pass(const std::vector<int>& q, int n, int rl)
{
    QPermPass P;
    P.n = n;
    P.rl = rl;
    std::vector<char> in_t(n, 0);
    for (int b = 0; b < rl; ++b)
        in_t[b] = 1;
    std::vector<int> hi;
    for (int b = 0; b < rl; ++b)
        if (!in_t[q[b]]) {
            in_t[q[b]] = 1;
            hi.push_back(q[b]);
        }
    // fill the tile up to 2^(2 rl) amplitudes with bits the map keeps in
    // place, then with exchanged pairs (both bits of a pair, so T stays closed)
    for (int b = rl; b < n && (int)hi.size() < rl; ++b)
        if (!in_t[b] && q[b] == b) {
            in_t[b] = 1;
            hi.push_back(b);
        }
    for (int b = rl; b < n && (int)hi.size() + 2 <= rl; ++b)
        if (!in_t[b] && q[b] != b && !in_t[q[b]]) {
            in_t[b] = in_t[q[b]] = 1;
            hi.push_back(b);
            hi.push_back(q[b]);
        }
    std::sort(hi.begin(), hi.end());
    P.hb = (int)hi.size();
    std::vector<int> T(rl + P.hb), cpos(n, -1);
    for (int k = 0; k < rl; ++k)
        T[k] = k;
    for (int k = 0; k < P.hb; ++k) {
        P.hpos[k] = hi[k];
        T[rl + k] = hi[k];
    }
    for (int k = 0; k < rl + P.hb; ++k)
        cpos[T[k]] = k;
    for (int k = 0; k < rl + P.hb; ++k)
        P.cmap[k] = cpos[q[T[k]]];
    for (int b = 0; b < n; ++b)
        P.q[b] = q[b];
    P.ntiles = 1ull << (n - rl - P.hb);
    // Outer bits (not tile bits) in compact order; the workgroup index takes
    // them alternately from the lowest outer bit not yet taken and from the
    // one whose image is the lowest not yet taken, so the low workgroup bits
    // vary the low bits of both the tile and its image.
    std::vector<int> outer;
    for (int b = 0; b < n; ++b)
        if (!in_t[b])
            outer.push_back(b);
    std::vector<int> opos(n, -1);
    for (size_t p = 0; p < outer.size(); ++p)
        opos[outer[p]] = (int)p;
    std::vector<char> taken(outer.size(), 0);
    int w = 0;
    size_t lo = 0, lo_img = 0;
    std::vector<int> by_image(outer);
    std::sort(by_image.begin(), by_image.end(), [&](int a, int b) { return q[a] < q[b]; });
    for (int turn = 0; w < (int)outer.size(); turn ^= 1) {
        int b = -1;
        if (turn == 0) {
            while (lo < outer.size() && taken[opos[outer[lo]]])
                ++lo;
            if (lo < outer.size())
                b = outer[lo];
        } else {
            while (lo_img < by_image.size() && taken[opos[by_image[lo_img]]])
                ++lo_img;
            if (lo_img < by_image.size())
                b = by_image[lo_img];
        }
        if (b < 0)
            continue;
        taken[opos[b]] = 1;
        P.wsrc[opos[b]] = w++;
    }
    return P;
}

}  // namespace

void plan_qubit_permutation(const std::vector<int>& Q, int n, int rl, std::vector<QPermPass>& out)
{
    bool ident = true, invol = true;
    for (int b = 0; b < n; ++b) {
        ident &= Q[b] == b;
        invol &= Q[Q[b]] == b;
    }
    if (ident)
        return;
    if (invol) {
        out.push_back(make_pass(Q, n, rl));
        return;
    }
    // Two reflections of every cycle c_0 -> c_1 -> ... -> c_{m-1} (Q[c_j] =
    // c_{j+1}): q1[c_j] = c_{-j}, q2[c_j] = c_{1-j}, so q2[q1[c_j]] = c_{j+1}.
    // Pass 1 (map q1) then pass 2 (map q2) take amplitude j from the input
    // amplitude whose bit b is bit q2[q1[b]] = Q[b] of j.
    std::vector<int> q1(n), q2(n);
    std::vector<char> done(n, 0);
    for (int s = 0; s < n; ++s) {
        if (done[s])
            continue;
        std::vector<int> c;
        for (int b = s; !done[b]; b = Q[b]) {
            done[b] = 1;
            c.push_back(b);
        }
        const int m = (int)c.size();
        for (int j = 0; j < m; ++j) {
            q1[c[j]] = c[(m - j) % m];
            q2[c[j]] = c[(m + 1 - j) % m];
        }
    }
    out.push_back(make_pass(q1, n, rl));
    out.push_back(make_pass(q2, n, rl));
}

}  // namespace qsv
