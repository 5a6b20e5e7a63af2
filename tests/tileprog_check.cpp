// Host-side check of the tile-program compiler (tileprog.cpp): compiles a
// gate list, checks the structure of the result, then executes the passes
// and steps on the CPU exactly as their descriptors say (tiles gathered
// through the pass's qubit mask, three-qubit steps over groups of eight
// amplitudes, gates in step order with their step-local target and
// controls) and prints the final state.  The caller compares that state with
// the oracle applying the gates in circuit order.
//
// stdin:  n m cap ngates
//         per gate: kind t nc c0 c1 param  re00 im00 re01 im01 re10 im10 re11 im11
//         2^n lines: re im of the input state
// stdout: 2^n lines: re im of the output state (%.17g)
// exit 1 with a message on stderr if a structural check fails.
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "qsv_tileprog.h"

using namespace qsv;
typedef std::complex<double> cd;

static void fail(const char* what, int a = 0, int b = 0)
{
    std::fprintf(stderr, "tile program check failed: %s (%d, %d)\n", what, a, b);
    std::exit(1);
}

static uint64_t deposit(uint64_t v, uint64_t mask)
{
    uint64_t out = 0;
    int b = 0;
    for (uint64_t m = mask; m; m &= m - 1, ++b)
        if ((v >> b) & 1)
            out |= m & (~m + 1);
    return out;
}

int main()
{
    int n, m, cap, ng;
    if (std::scanf("%d %d %d %d", &n, &m, &cap, &ng) != 4)
        fail("input header");
    std::vector<HGate> gates(ng);
    std::vector<cd> mat(4 * (size_t)ng);
    for (int g = 0; g < ng; ++g) {
        HGate& h = gates[g];
        double v[8];
        if (std::scanf("%d %d %d %d %d %d", &h.kind, &h.t, &h.nc, &h.c0, &h.c1, &h.param) != 6)
            fail("gate", g);
        for (double& x : v)
            if (std::scanf("%lf", &x) != 1)
                fail("matrix", g);
        for (int e = 0; e < 4; ++e)
            mat[4 * (size_t)g + e] = cd(v[2 * e], v[2 * e + 1]);
        h.mat = g;  // the executor below finds each gate's matrix through it
    }
    const size_t N = (size_t)1 << n;
    std::vector<cd> psi(N);
    for (size_t i = 0; i < N; ++i) {
        double re, im;
        if (std::scanf("%lf %lf", &re, &im) != 2)
            fail("state");
        psi[i] = cd(re, im);
    }

    TileProgram tp;
    compile_tile_program(gates, n, m, cap, tp);

    // structure
    std::vector<int> seen(ng, 0);
    const int mb_want = m < n ? m : n;
    for (size_t p = 0; p < tp.passes.size(); ++p) {
        const DPass& P = tp.passes[p];
        const int mb = __builtin_popcountll(P.bmask);
        if (mb != mb_want || (n < 64 && (P.bmask >> n) != 0))
            fail("tile mask", (int)p, mb);
        if (P.nops > cap)
            fail("gates per pass", (int)p, P.nops);
        std::vector<int> slot_used(P.nrot, 0);
        int ops_in_steps = 0;
        for (int s = 0; s < P.nsteps; ++s) {
            const DStep& st = tp.steps[P.step_off + s];
            if (st.nq != 3 || !(st.q[0] < st.q[1] && st.q[1] < st.q[2]) || st.q[2] >= mb)
                fail("step qubits", (int)p, s);
            if (st.o1 - st.o0 < 1 || st.o1 - st.o0 > kMaxStepOps || st.o0 != ops_in_steps)
                fail("step gate range", (int)p, s);
            ops_in_steps = st.o1;
            for (int o = st.o0; o < st.o1; ++o) {
                const DOp& d = tp.ops[P.op_off + o];
                if (d.tq > 2 || (d.cm & ~7) || ((d.cm >> d.tq) & 1))
                    fail("step-local target or controls", (int)p, o);
                const HGate& h = gates[d.mat];
                if (__builtin_popcount(d.cm) != h.nc)
                    fail("control count", (int)p, o);
                if (seen[d.mat]++)
                    fail("gate scheduled twice", d.mat);
                if (h.kind != 0) {
                    if (d.slot < 0 || d.slot >= P.nrot || slot_used[d.slot]++)
                        fail("rotation slot", (int)p, o);
                    if (tp.slot_param[P.slot_base + d.slot] != h.param || d.param != h.param)
                        fail("slot parameter", (int)p, o);
                } else if (d.slot != -1) {
                    fail("slot on a fixed gate", (int)p, o);
                }
            }
        }
        if (ops_in_steps != P.nops)
            fail("steps do not cover the pass", (int)p);
    }
    for (int g = 0; g < ng; ++g)
        if (seen[g] != 1)
            fail("gate not scheduled", g);

    // execution
    std::vector<cd> tile;
    for (const DPass& P : tp.passes) {
        const int mb = __builtin_popcountll(P.bmask);
        const uint64_t rest = (n >= 64 ? ~0ull : ((1ull << n) - 1)) & ~P.bmask;
        const uint64_t ntiles = 1ull << (n - mb);
        tile.assign((size_t)1 << mb, cd());
        for (uint64_t t = 0; t < ntiles; ++t) {
            const uint64_t base = deposit(t, rest);
            for (uint64_t l = 0; l < tile.size(); ++l)
                tile[l] = psi[base | deposit(l, P.bmask)];
            for (int s = 0; s < P.nsteps; ++s) {
                const DStep& st = tp.steps[P.step_off + s];
                const uint64_t smask = (1ull << st.q[0]) | (1ull << st.q[1]) | (1ull << st.q[2]);
                const uint64_t others = (((uint64_t)1 << mb) - 1) & ~smask;
                for (uint64_t g = 0; g < ((uint64_t)1 << (mb - 3)); ++g) {
                    const uint64_t b = deposit(g, others);
                    cd a[8];
                    for (int j = 0; j < 8; ++j)
                        a[j] = tile[b | deposit(j, smask)];
                    for (int o = st.o0; o < st.o1; ++o) {
                        const DOp& d = tp.ops[P.op_off + o];
                        const cd* G = &mat[4 * (size_t)d.mat];
                        for (int u0 = 0; u0 < 8; ++u0) {
                            if ((u0 >> d.tq) & 1 || (u0 & d.cm) != d.cm)
                                continue;
                            const int u1 = u0 | (1 << d.tq);
                            const cd x = a[u0], y = a[u1];
                            a[u0] = G[0] * x + G[1] * y;
                            a[u1] = G[2] * x + G[3] * y;
                        }
                    }
                    for (int j = 0; j < 8; ++j)
                        tile[b | deposit(j, smask)] = a[j];
                }
            }
            for (uint64_t l = 0; l < tile.size(); ++l)
                psi[base | deposit(l, P.bmask)] = tile[l];
        }
    }
    std::fprintf(stderr, "passes %zu steps %zu\n", tp.passes.size(), tp.steps.size());
    for (size_t i = 0; i < N; ++i)
        std::printf("%.17g %.17g\n", psi[i].real(), psi[i].imag());
    return 0;
}
