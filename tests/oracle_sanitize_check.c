/*
 * Drives every entry point of the CPU oracle (oracle/oracle.c) on small
 * inputs, so that a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitizers.py) sees each code path once: gate application with
 * 1..5 targets and controls, permutations, inner products and norms, Pauli
 * expectations and H psi, the seeded state and its sampled form, circuits,
 * energies, parameter-shift and finite-difference gradients, the adjoint,
 * marginals, sampling, frequencies, collapse, seeded uniforms, and the
 * argument errors.  A few numeric checks make sure the calls did real work;
 * the value checks proper live in the Python pins.  Exit 0 on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_apply(int n, const double* in, double* out, const int* t, int k, const int* ctl, int c,
              const double* G);
int orc_inner(int n, const double* a, const double* b, double* out2);
int orc_expect(int n, const double* psi, int nterms, const uint64_t* x, const uint64_t* z,
               const double* coeff, double* out2, double* per_term);
int orc_apply_hamiltonian(int n, const double* psi, double* lam, int nterms, const uint64_t* x,
                          const uint64_t* z, const double* coeff);
int orc_norm2(int n, const double* psi, double* out);
int orc_random_norm2(int n, uint64_t seed, double* out);
int orc_random_state(int n, uint64_t seed, double* psi);
int orc_random_amps(uint64_t seed, double scale, const uint64_t* idx, int m, double* out);
int orc_apply_sampled_random(int n, uint64_t seed, double scale, const int* t, int k, const int* ctl,
                             int c, const double* G, const uint64_t* idx, int m, double* out);
int orc_run(int n, int nops, const int* kind, const int* k, const int* tgt, const int* c,
            const int* ctl, const int* param, const long long* moff, const double* mats,
            const double* params, const double* psi0, double* psi);
int orc_energy(int n, int nops, const int* kind, const int* k, const int* tgt, const int* c,
               const int* ctl, const int* param, const long long* moff, const double* mats,
               const double* params, int nterms, const uint64_t* x, const uint64_t* z,
               const double* coeff, double* E);
int orc_grad(int n, int nops, const int* kind, const int* k, const int* tgt, const int* c,
             const int* ctl, const int* param, const long long* moff, const double* mats,
             const double* params, int nparams, int nterms, const uint64_t* x, const uint64_t* z,
             const double* coeff, const int* which, int m, int mode, double h, double* grad);
int orc_adjoint(int n, int nops, const int* kind, const int* k, const int* tgt, const int* c,
                const int* ctl, const int* param, const long long* moff, const double* mats,
                const double* params, int nparams, int nterms, const uint64_t* x,
                const uint64_t* z, const double* coeff, double* E, double* grad);
int orc_probabilities(int n, const double* psi, const int* q, int m, double* out);
int orc_sample(int n, const double* psi, const double* u, int64_t nshots, int64_t* out);
int orc_frequencies(int n, const int64_t* samples, int64_t nshots, const int* q, int m,
                    int64_t* counts);
int orc_collapse(int n, const double* psi, double* out, const int* q, int m, uint64_t b, double p);
int orc_uniforms(uint64_t seed, int64_t count, double* u);

static void require(int cond, const char* what)
{
    if (!cond) {
        fprintf(stderr, "oracle sanitizer check failed: %s\n", what);
        exit(1);
    }
}

/* A dense non-unitary 2^k x 2^k matrix with entries in [-1, 1]. */
static void fill_matrix(double* G, int k, unsigned seed)
{
    const int dim = 1 << k;
    for (int j = 0; j < 2 * dim * dim; ++j) {
        seed = seed * 1103515245u + 12345u;
        G[j] = ((double)(seed >> 8) / 16777216.0) * 2.0 - 1.0;
    }
}

int main(void)
{
    const int n = 7;
    const size_t N = (size_t)1 << n;
    double* psi = malloc(sizeof(double) * 2 * N);
    double* out = malloc(sizeof(double) * 2 * N);
    double* tmp = malloc(sizeof(double) * 2 * N);
    require(psi && out && tmp, "allocation");
    require(orc_random_state(n, 17, psi) == 0, "random state");
    double nrm;
    orc_norm2(n, psi, &nrm);
    require(fabs(nrm - 1.0) < 1e-12, "random state norm");

    /* gates of every width, with and without controls */
    static double G[2 * 32 * 32];
    const int tg[5] = {3, 0, 6, 1, 4};
    const int ct[2] = {2, 5};
    for (int k = 1; k <= 5; ++k)
        for (int c = 0; c <= 2 && k + c <= n; ++c) {
            fill_matrix(G, k, 31u * (unsigned)k + (unsigned)c);
            require(orc_apply(n, psi, out, tg, k, ct, c, G) == 0, "apply");
        }
    const double X[8] = {0, 0, 1, 0, 1, 0, 0, 0};
    require(orc_apply(n, psi, out, tg, 1, ct, 1, X) == 0, "permutation");
    const int bad_t[2] = {1, 1};
    require(orc_apply(n, psi, out, bad_t, 2, NULL, 0, G) != 0, "repeated qubit refused");
    const int big_t[1] = {n};
    require(orc_apply(n, psi, out, big_t, 1, NULL, 0, X) != 0, "qubit out of range refused");
    require(orc_apply(n, psi, psi, tg, 1, NULL, 0, X) != 0, "in place refused");

    double ip[2];
    orc_inner(n, psi, out, ip);

    /* Pauli sums */
    const uint64_t x[4] = {0, 3, 0x40, 0x11};
    const uint64_t z[4] = {0x5, 0, 0x40, 0x10};
    const double cf[4] = {0.5, -1.0, 0.25, 2.0};
    double e2[2], per[8];
    require(orc_expect(n, psi, 4, x, z, cf, e2, per) == 0, "expect");
    require(orc_apply_hamiltonian(n, psi, out, 4, x, z, cf) == 0, "H psi");

    /* seeded amplitudes and sampled application */
    const uint64_t idx[4] = {0, 5, 77, N - 1};
    double amps[8];
    orc_random_amps(17, 1.0, idx, 4, amps);
    fill_matrix(G, 2, 5u);
    require(orc_apply_sampled_random(n, 17, 1.0 / sqrt(2.0), tg, 2, ct, 1, G, idx, 4, amps) == 0,
            "sampled apply");
    double s2;
    orc_random_norm2(n, 17, &s2);

    /* a circuit of every kind: matrix, H, X, Y, Z, RX, RY, RZ, SWAP, controls */
    enum { NOPS = 10 };
    int kind[NOPS] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 7};
    int kk[NOPS] = {2, 1, 1, 1, 1, 1, 1, 1, 2, 1};
    int tgt[NOPS * 5] = {0};
    int cc[NOPS] = {0, 0, 1, 0, 0, 0, 0, 0, 0, 1};
    int ctl[NOPS * 4] = {0};
    int param[NOPS] = {-1, -1, -1, -1, -1, 0, 1, 2, -1, 3};
    long long moff[NOPS];
    for (int o = 0; o < NOPS; ++o) {
        moff[o] = -1;
        tgt[5 * o] = o % n;
        if (kk[o] == 2)
            tgt[5 * o + 1] = (o + 3) % n;
        if (cc[o])
            ctl[4 * o] = (o + 5) % n;
    }
    moff[0] = 0;
    fill_matrix(G, 2, 9u);
    const double params[4] = {0.3, 1.1, -0.7, 2.0};
    require(orc_run(n, NOPS, kind, kk, tgt, cc, ctl, param, moff, G, params, NULL, out) == 0, "run");
    require(orc_run(n, NOPS, kind, kk, tgt, cc, ctl, param, moff, G, params, psi, out) == 0,
            "run from a state");
    double E;
    require(orc_energy(n, NOPS, kind, kk, tgt, cc, ctl, param, moff, G, params, 4, x, z, cf, &E) == 0,
            "energy");
    /* gradients on a unitary circuit (the matrix op replaced by H) */
    kind[0] = 1;
    kk[0] = 1;
    double ga[4], gf[4], gp[3];
    const int which[4] = {0, 1, 2, 3};
    require(orc_adjoint(n, NOPS, kind, kk, tgt, cc, ctl, param, moff, G, params, 4, 4, x, z, cf,
                        &E, ga) == 0, "adjoint");
    require(orc_grad(n, NOPS, kind, kk, tgt, cc, ctl, param, moff, G, params, 4, 4, x, z, cf,
                     which, 4, 1, 1e-6, gf) == 0, "finite differences");
    for (int j = 0; j < 4; ++j)
        require(fabs(ga[j] - gf[j]) < 1e-6, "adjoint vs finite differences");
    require(orc_grad(n, NOPS, kind, kk, tgt, cc, ctl, param, moff, G, params, 4, 4, x, z, cf,
                     which, 3, 0, 0.0, gp) == 0, "parameter shift");
    require(orc_grad(n, NOPS, kind, kk, tgt, cc, ctl, param, moff, G, params, 4, 4, x, z, cf,
                     which + 3, 1, 0, 0.0, gp) != 0, "parameter shift refuses a controlled rotation");

    /* measurement */
    const int q[3] = {6, 0, 3};
    double marg[8];
    require(orc_probabilities(n, psi, q, 3, marg) == 0, "marginals");
    require(orc_probabilities(n, psi, bad_t, 2, marg) != 0, "marginals refuse a repeated qubit");
    double u[64];
    require(orc_uniforms(99, 64, u) == 0, "uniforms");
    u[0] = 1.0;
    u[1] = -0.5;
    u[2] = NAN;
    int64_t shots[64], counts[8];
    require(orc_sample(n, psi, u, 64, shots) == 0, "sample");
    for (int s = 0; s < 64; ++s)
        require(shots[s] >= 0 && (size_t)shots[s] < N, "shot in range");
    require(orc_frequencies(n, shots, 64, q, 3, counts) == 0, "frequencies");
    int64_t tot = 0;
    for (int b = 0; b < 8; ++b)
        tot += counts[b];
    require(tot == 64, "frequencies add up");
    require(orc_collapse(n, psi, out, q, 3, 5, marg[5]) == 0, "collapse");
    require(orc_collapse(n, psi, out, q, 3, 8, 0.5) != 0, "collapse refuses an outcome >= 2^m");
    require(orc_collapse(n, psi, out, q, 3, 2, 0.0) == 0, "collapse onto an impossible outcome");

    /* the chunked reduction path (n >= 11) */
    const int nb = 12;
    double* a = malloc(sizeof(double) * (2u << nb));
    double* b = malloc(sizeof(double) * (2u << nb));
    require(a && b, "allocation");
    orc_random_state(nb, 1, a);
    orc_random_state(nb, 2, b);
    orc_inner(nb, a, b, ip);
    orc_norm2(nb, a, &nrm);
    require(fabs(nrm - 1.0) < 1e-12, "chunked norm");
    free(a);
    free(b);
    free(psi);
    free(out);
    free(tmp);
    printf("oracle sanitizer check ok\n");
    return 0;
}
