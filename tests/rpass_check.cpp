// CPU checker of the register-tile Pauli pass planner
// (paper_2202_07017_amd/csrc/rpass_plan.cpp).
//
// Reads a Pauli sum from stdin ("n nterms", then one "x z c" line per term)
// and a state (2^n complex128, interleaved) from the file named by argv[1].
// It plans the passes, checks their structure, and evaluates every pass on
// the CPU as its descriptor says -- tile insertion masks, lane and register
// positions, the transpose of the first pass, the sign parts (lane mask,
// tile parity, register mask or half-sum coefficients), the chunked tables
// of the diagonal strings -- and prints the register passes' part of
// <psi|H|psi> and the indices left to the LDS-tile passes:
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

#include "qsv_rpass_plan.h"

using qsv::RegPassK;
using qsv::RTerm;
using cd = std::complex<double>;

static void require(bool ok, const char* what, int pass)
{
    if (!ok) {
        std::fprintf(stderr, "pass %d: %s\n", pass, what);
        std::exit(1);
    }
}

static int par(uint64_t v) { return __builtin_popcountll(v) & 1; }

static bool plain(const RTerm& t) { return t.z == 0 && __builtin_popcount(t.xr) == 1; }

// x masks the kernel takes: one register bit or two neighbouring ones
static bool reg_ok(uint32_t xr)
{
    return xr != 0 && xr < 32 && ((xr & (xr - 1)) == 0 || (xr >> __builtin_ctz(xr)) == 3u);
}

// sum over the pairs (a, a ^ xr), a with the highest bit of xr clear, of Re
// (im = false) or Im (im = true) of conj(amp[a ^ xr]) amp[a], split into two
// halves as the kernel does (by the lower x bit, alternating for one bit)
static void halves(const cd* amp, uint32_t xr, bool im, double& s0, double& s1)
{
    int hb = 31 - __builtin_clz(xr), lb = __builtin_ctz(xr);
    s0 = s1 = 0.0;
    int m = 0;
    for (int a = 0; a < 32; ++a) {
        if ((a >> hb) & 1)
            continue;
        const cd w = std::conj(amp[a ^ xr]) * amp[a];
        const double d = im ? w.imag() : w.real();
        if (lb != hb ? ((a >> lb) & 1) : (m++ & 1))
            s1 += d;
        else
            s0 += d;
    }
}

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
    std::vector<RegPassK> passes;
    std::vector<int> rest;
    qsv::plan_reg_passes(&H, n, passes, rest);

    double energy = 0.0;
    for (int pi = 0; pi < (int)passes.size(); ++pi) {
        const RegPassK& P = passes[pi];
        // structure
        require(P.ntiles == (1ull << (n - qsv::kRegTileQubits)), "tile count", pi);
        require(P.nd >= 0 && P.nd <= P.ns1 && P.ns1 <= P.n1 && P.n1 <= P.ns2 && P.ns2 <= P.nc &&
                    P.nc <= P.nt && P.nt <= qsv::kMaxRegTerms, "term ranges", pi);
        require(P.mofs[0] == 0 && P.mofs[32] == P.nd, "diagonal offsets", pi);
        uint64_t tmask = 0;
        int prevq = -1;
        for (int j = 0; j < qsv::kRegTileQubits; ++j) {
            const uint64_t lo = P.low[j];
            require((lo & (lo + 1)) == 0, "insertion mask", pi);
            const int q = __builtin_popcountll(lo);
            require(q > prevq && q < n, "tile qubits ascending", pi);
            prevq = q;
            tmask |= 1ull << q;
        }
        uint64_t lmask = 0, rmask = 0;
        for (int b = 0; b < qsv::kRegLanes; ++b)
            lmask |= 1ull << P.lanepos[b];
        for (int b = 0; b < qsv::kRegLanes - 1; ++b)
            require(P.lanepos[b] == b, "lane qubits 0..4", pi);
        for (int k = 0; k < qsv::kRegQubits; ++k) {
            require(P.qstride[k] != 0 && (P.qstride[k] & (P.qstride[k] - 1)) == 0, "register stride", pi);
            rmask |= P.qstride[k];
            if (k)
                require(P.qstride[k] > P.qstride[k - 1], "register qubits ascending", pi);
        }
        require((lmask & rmask) == 0 && (lmask | rmask) == tmask, "tile = lanes + registers", pi);
        for (int m = 0; m < 32; ++m) {
            require(P.mofs[m] <= P.mofs[m + 1], "diagonal offsets ascending", pi);
            for (int k = P.mofs[m]; k < P.mofs[m + 1]; ++k)
                require(P.t[k].xr == 0 && (int)P.t[k].zr == m, "diagonal group", pi);
        }
        for (int k = P.nd; k < P.nc; ++k) {
            const RTerm& t = P.t[k];
            require(reg_ok(t.xr) && t.xl == 0, "register x mask", pi);
            const bool pl = (k < P.ns1) || (k >= P.n1 && k < P.ns2);
            require(pl == plain(t), "plain / general split", pi);
            require((t.zr & ~t.xr) == 0, "register z bits inside the x mask", pi);
        }
        for (int k = P.nc; k < P.nt; ++k) {
            const RTerm& t = P.t[k];
            require(t.xr == 16 && t.xl != 0 && t.xl < 64 && (t.xl & (t.xl - 1)) == 0, "cross-lane masks", pi);
            require((t.zr & ~16u) == 0, "cross-lane z on qubits 0..3", pi);
        }
        // evaluation, tile by tile
        for (uint64_t tl = 0; tl < P.ntiles; ++tl) {
            uint64_t base = tl;
            for (int j = 0; j < qsv::kRegTileQubits; ++j)
                base = ((base & ~P.low[j]) << 1) | (base & P.low[j]);
            require(base < N && (base & tmask) == 0, "tile base", pi);
            static cd amp[64][32], amp2[64][32];
            for (int lane = 0; lane < 64; ++lane)
                for (int r = 0; r < 32; ++r) {
                    uint64_t i = base;
                    for (int b = 0; b < 6; ++b)
                        if ((lane >> b) & 1)
                            i |= 1ull << P.lanepos[b];
                    for (int k = 0; k < 5; ++k)
                        if ((r >> k) & 1)
                            i |= P.qstride[k];
                    amp[lane][r] = psi[i];
                }
            // transposed roles: element (L, r') = (lane r' + 32 (L & 1), register L >> 1)
            for (int L = 0; L < 64; ++L)
                for (int rp = 0; rp < 32; ++rp)
                    amp2[L][rp] = amp[rp + 32 * (L & 1)][L >> 1];
            for (int lane = 0; lane < 64; ++lane) {
                uint64_t sg = 0;
                for (int k = 0; k < P.nt; ++k)
                    sg |= (uint64_t)(par((uint64_t)lane & P.t[k].zl) ^ par(base & P.t[k].z)) << k;
                double s = 0.0;
                // diagonal: N(m) and the chunk tables of signed coefficients
                if (P.nd > 0) {
                    double Nm[32];
                    for (int m = 0; m < 32; ++m) {
                        Nm[m] = 0.0;
                        for (int r = 0; r < 32; ++r)
                            Nm[m] += (par((uint64_t)(r & m)) ? -1.0 : 1.0) * std::norm(amp[lane][r]);
                    }
                    for (int m = 0; m < 32; ++m)
                        for (int k0 = P.mofs[m]; k0 < P.mofs[m + 1]; k0 += 5) {
                            const int g = std::min(5, P.mofs[m + 1] - k0);
                            const int q = (int)(sg >> k0) & ((1 << g) - 1);
                            double w = 0.0;
                            for (int i = 0; i < g; ++i)
                                w += ((q >> i) & 1) ? -P.t[k0 + i].c : P.t[k0 + i].c;
                            s += w * Nm[m];
                        }
                }
                for (int ph = 0; ph < 2; ++ph) {
                    const cd* a = ph ? amp2[lane] : amp[lane];
                    const int k0 = ph ? P.n1 : P.nd, k1 = ph ? P.nc : P.n1;
                    for (int k = k0; k < k1; ++k) {
                        const RTerm& t = P.t[k];
                        double s0, s1;
                        halves(a, t.xr, (t.ylo & 1) != 0, s0, s1);
                        const double v = plain(t) ? t.c * (s0 + s1) : t.c * s0 + t.c2 * s1;
                        s += ((sg >> k) & 1) ? -v : v;
                    }
                }
                // cross-lane strings: the pair of (lane, r), r < 16, is (lane ^ xl, r + 16)
                for (int k = P.nc; k < P.nt; ++k) {
                    const RTerm& t = P.t[k];
                    double d = 0.0;
                    for (int r = 0; r < 16; ++r) {
                        const cd w = std::conj(amp2[lane ^ t.xl][r + 16]) * amp2[lane][r];
                        d += (t.ylo & 1) ? w.imag() : w.real();
                    }
                    const double v = t.c * d;
                    s += ((sg >> k) & 1) ? -v : v;
                }
                energy += s;
            }
        }
    }
    std::printf("passes %d\nrest", (int)passes.size());
    for (int j : rest)
        std::printf(" %d", j);
    std::printf("\nenergy %.17g\n", energy);
    return 0;
}
