// CPU checker of the span pass planner (paper_2202_07017_amd/csrc/span_plan.cpp).
//
// Reads a Pauli sum from stdin ("n nterms", then one "x z c" line per term)
// and a state (2^n complex128, interleaved) from the file named by argv[1].
// It plans the span passes, checks their structure (tile insertion masks on
// qubits 0..5 and the pivots, the group offsets, every index of the state reached exactly
// once per pass as base ^ lane ^ D(r)), evaluates every pass on the CPU as
// its descriptor says (the lane, tile and register parts of each string's
// sign, Re or Im of the pair products, the folded coefficient) and prints
// the span passes' part of <psi|H|psi> and the strings left to other passes:
//   passes <count>
//   rest <i> <i> ...
//   energy <value>
// Exit 0 on success, 1 with a message on a structural error.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "qsv_span_plan.h"

using qsv::SpanPassK;
using qsv::STerm;
using cd = std::complex<double>;

static void require(bool ok, const char* what, int pass)
{
    if (!ok) {
        std::fprintf(stderr, "pass %d: %s\n", pass, what);
        std::exit(1);
    }
}

static int par(uint64_t v) { return __builtin_popcountll(v) & 1; }

int main(int argc, char** argv)
{
    if (argc < 2)
        return 1;
    int n = 0, nt = 0;
    if (std::scanf("%d %d", &n, &nt) != 2)
        return 1;
    std::vector<uint64_t> X(nt), Z(nt);
    std::vector<double> C(nt);
    for (int j = 0; j < nt; ++j) {
        unsigned long long x, z;
        if (std::scanf("%llu %llu %lf", &x, &z, &C[j]) != 3)
            return 1;
        X[j] = x;
        Z[j] = z;
    }
    const uint64_t N = 1ull << n;
    std::vector<cd> psi(N);
    FILE* f = std::fopen(argv[1], "rb");
    if (!f || std::fread(psi.data(), sizeof(cd), N, f) != N)
        return 1;
    std::fclose(f);

    const qsv_pauli_sum H{nt, X.data(), Z.data(), C.data()};
    std::vector<SpanPassK> passes;
    qsv::plan_span_passes(&H, n, passes);

    double energy = 0.0;
    std::vector<unsigned char> seen(N);
    for (int pi = 0; pi < (int)passes.size(); ++pi) {
        const SpanPassK& P = passes[pi];
        require(P.ntiles == (1ull << (n - qsv::kSpanTileQubits)), "tile count", pi);
        require(P.nt >= 1 && P.nt <= qsv::kMaxSpanTerms, "string count", pi);
        uint64_t tmask = 0;
        int prevq = -1;
        for (int j = 0; j < qsv::kSpanTileQubits; ++j) {
            const uint64_t lo = P.low[j];
            require((lo & (lo + 1)) == 0, "insertion mask", pi);
            const int q = __builtin_popcountll(lo);
            require(q > prevq && q < n, "tile qubits ascending", pi);
            prevq = q;
            tmask |= 1ull << q;
        }
        require((tmask & 63) == 63, "lanes on qubits 0..5", pi);
        const int G = qsv::kSpanGroups, NM = 1 << qsv::kSpanDirs;
        require(P.koff[0] == 0 && P.mofs[0] == P.koff[G] && P.mofs[NM] == P.nt, "group offsets", pi);
        for (int g = 0; g < G; ++g) {
            require(P.koff[g] <= P.koff[g + 1], "group offsets ascending", pi);
            for (int k = P.koff[g]; k < P.koff[g + 1]; ++k) {
                const STerm& t = P.t[k];
                if (g < 2 * qsv::kSpanDirs)
                    require(2 * t.dir + t.im == g && t.xl == 0, "direction string group", pi);
                else
                    require(t.dir == -1 && t.im == g - 2 * qsv::kSpanDirs && t.xl != 0 && t.xl < 64,
                            "lane string group", pi);
            }
        }
        for (int m = 0; m < NM; ++m) {
            require(P.mofs[m] <= P.mofs[m + 1], "diagonal offsets ascending", pi);
            for (int k = P.mofs[m]; k < P.mofs[m + 1]; ++k)
                require(P.t[k].dir == -1 && P.t[k].xl == 0 && (int)P.t[k].zr == m, "diagonal group", pi);
        }
        auto D = [&](int r) {
            uint64_t o = 0;
            for (int j = 0; j < qsv::kSpanDirs; ++j)
                if ((r >> j) & 1)
                    o ^= P.d[j];
            return o;
        };
        std::fill(seen.begin(), seen.end(), 0);
        for (uint64_t tl = 0; tl < P.ntiles; ++tl) {
            uint64_t base = tl;
            for (int j = 0; j < qsv::kSpanTileQubits; ++j)
                base = ((base & ~P.low[j]) << 1) | (base & P.low[j]);
            require(base < N && (base & tmask) == 0, "tile base", pi);
            static cd a[64][32];
            for (int lane = 0; lane < 64; ++lane)
                for (int r = 0; r < 32; ++r) {
                    const uint64_t i = base ^ (uint64_t)lane ^ D(r);
                    require(i < N, "index in range", pi);
                    require(seen[i] == 0, "index reached twice", pi);
                    seen[i] = 1;
                    a[lane][r] = psi[i];
                }
            for (int lane = 0; lane < 64; ++lane)
                for (int k = 0; k < P.nt; ++k) {
                    const STerm& t = P.t[k];
                    double s = 0.0;
                    if (k < P.koff[2 * qsv::kSpanDirs]) {  // direction string
                        for (int i = 0; i < 16; ++i) {
                            const int r = ((i >> t.dir) << (t.dir + 1)) | (i & ((1 << t.dir) - 1));
                            const cd w = std::conj(a[lane][r ^ (1 << t.dir)]) * a[lane][r];
                            const double fv = t.im ? w.imag() : w.real();
                            s += ((t.sgn >> i) & 1) ? -fv : fv;
                        }
                    } else if (k < P.koff[G]) {  // lane string
                        for (int r = 0; r < 32; ++r) {
                            const cd w = std::conj(a[lane ^ t.xl][r]) * a[lane][r];
                            const double fv = t.im ? w.imag() : w.real();
                            s += ((t.sgn >> r) & 1) ? -fv : fv;
                        }
                    } else {  // diagonal string
                        for (int r = 0; r < 32; ++r)
                            s += (par((uint64_t)(r & t.zr)) ? -1.0 : 1.0) * std::norm(a[lane][r]);
                    }
                    const int sg = par(t.z & base) ^ par(t.z & (uint64_t)lane);
                    energy += (sg ? -1.0 : 1.0) * t.c * s;
                }
        }
        for (uint64_t i = 0; i < N; ++i)
            require(seen[i] == 1, "index not reached", pi);
    }
    std::printf("passes %d\nenergy %.17g\n", (int)passes.size(), energy);
    return 0;
}
