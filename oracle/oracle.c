/*
 * CPU oracle for the state-vector path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * use this file.  It shares no code, header, table or helper with the GPU
 * library and must never be linked into it.
 *
 * Everything is complex128, out of place, in the plainest form:
 *   - gate application is the matrix product of the paper's eq. (1) (Sec. 2):
 *     for every output index i, psi'(tau, q) = sum_tau' G(tau, tau') psi(tau', q),
 *     tau = the target bits of i, q = the other bits;
 *   - controlled gates (Sec. 2, "controlled gates ... modified index
 *     generation") apply G only where every control bit of i is 1 and copy
 *     psi[i] elsewhere;
 *   - a gate whose matrix is exactly a 0/1 permutation copies amplitudes
 *     (same result as eq. (1), raw bits preserved);
 *   - Pauli-sum expectation values (Sec. 3, Hamiltonian primitives) multiply
 *     the Pauli factors into a copy of psi one 2x2 matrix at a time and take
 *     the inner product with pairwise summation;
 *   - gradients by parameter shift, central finite differences and a plain
 *     adjoint sweep with explicit dagger and derivative matrices.
 *
 * Conventions: qubit j is bit j of an index.  For targets t[0..k-1] the first
 * target is the most significant bit of G's index tau.  G is row-major,
 * interleaved (re, im), G[(tau * 2^k + tau') * 2 + {0,1}].
 * Compile with -ffp-contract=off so no product is fused into an FMA.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double re, im;
} ocx;

static ocx cx_mul(ocx a, ocx b)
{
    ocx r;
    r.re = a.re * b.re - a.im * b.im;
    r.im = a.re * b.im + a.im * b.re;
    return r;
}

static ocx cx_add(ocx a, ocx b)
{
    ocx r;
    r.re = a.re + b.re;
    r.im = a.im + b.im;
    return r;
}

static ocx cx_conj(ocx a)
{
    a.im = -a.im;
    return a;
}

/* ---------------------------------------------------------------- indices */

/* tau = the target bits of i, target t[j] going to bit (k-1-j) of tau. */
static uint64_t tau_of(uint64_t i, const int* t, int k)
{
    uint64_t tau = 0;
    for (int j = 0; j < k; ++j)
        tau |= ((i >> t[j]) & 1ULL) << (k - 1 - j);
    return tau;
}

/* i with its target bits replaced by the bits of tau (same ordering). */
static uint64_t with_tau(uint64_t i, const int* t, int k, uint64_t tau)
{
    for (int j = 0; j < k; ++j) {
        uint64_t bit = (tau >> (k - 1 - j)) & 1ULL;
        i = (i & ~(1ULL << t[j])) | (bit << t[j]);
    }
    return i;
}

static int check_qubits(int n, const int* t, int k, const int* ctl, int c)
{
    if (n < 1 || n > 40 || k < 1 || k > 10 || c < 0 || k + c > n)
        return -1;
    uint64_t seen = 0;
    for (int j = 0; j < k + c; ++j) {
        int q = j < k ? t[j] : ctl[j - k];
        if (q < 0 || q >= n || (seen >> q) & 1ULL)
            return -2;
        seen |= 1ULL << q;
    }
    return 0;
}

/* If G is exactly a 0/1 permutation matrix, fill src[tau] = the column holding
 * row tau's 1 and return 1; else return 0. */
static int as_permutation(const double* G, int dim, int* src)
{
    int* colseen = (int*)calloc((size_t)dim, sizeof(int));
    int ok = 1;
    for (int r = 0; r < dim && ok; ++r) {
        int ones = 0;
        for (int col = 0; col < dim; ++col) {
            double re = G[((size_t)r * dim + col) * 2], im = G[((size_t)r * dim + col) * 2 + 1];
            if (im != 0.0 || (re != 0.0 && re != 1.0)) {
                ok = 0;
                break;
            }
            if (re == 1.0) {
                ++ones;
                src[r] = col;
            }
        }
        if (ok && ones != 1)
            ok = 0;
        if (ok) {
            if (colseen[src[r]])
                ok = 0;
            colseen[src[r]] = 1;
        }
    }
    free(colseen);
    return ok;
}

/* ----------------------------------------------------------- eq. (1) core */

int orc_apply(int n, const double* in, double* out, const int* t, int k, const int* ctl, int c,
              const double* G)
{
    if (check_qubits(n, t, k, ctl, c) != 0 || in == out)
        return -1;
    const int dim = 1 << k;
    const uint64_t N = 1ULL << n;
    uint64_t cmask = 0;
    for (int j = 0; j < c; ++j)
        cmask |= 1ULL << ctl[j];
    int* src = (int*)malloc(sizeof(int) * (size_t)dim);
    const int perm = as_permutation(G, dim, src);
    const ocx* pin = (const ocx*)in;
    ocx* pout = (ocx*)out;
#pragma omp parallel for schedule(static)
    for (long long ii = 0; ii < (long long)N; ++ii) {
        uint64_t i = (uint64_t)ii;
        if ((i & cmask) != cmask) {
            memcpy(&pout[i], &pin[i], sizeof(ocx));
            continue;
        }
        uint64_t tau = tau_of(i, t, k);
        if (perm) {
            memcpy(&pout[i], &pin[with_tau(i, t, k, (uint64_t)src[tau])], sizeof(ocx));
            continue;
        }
        ocx acc = {0.0, 0.0};
        for (int tp = 0; tp < dim; ++tp) {
            ocx g = {G[((size_t)tau * dim + tp) * 2], G[((size_t)tau * dim + tp) * 2 + 1]};
            acc = cx_add(acc, cx_mul(g, pin[with_tau(i, t, k, (uint64_t)tp)]));
        }
        pout[i] = acc;
    }
    free(src);
    return 0;
}

/* Threads the OpenMP loops of this library use (for reports). */
int orc_threads(void)
{
    return omp_get_max_threads();
}

/* --------------------------------------------------------- pairwise sums */

static ocx dot_pairwise(const ocx* a, const ocx* b, uint64_t lo, uint64_t hi)
{
    if (hi - lo <= 32) {
        ocx s = {0.0, 0.0};
        for (uint64_t i = lo; i < hi; ++i)
            s = cx_add(s, cx_mul(cx_conj(a[i]), b[i]));
        return s;
    }
    uint64_t mid = lo + (hi - lo) / 2;
    return cx_add(dot_pairwise(a, b, lo, mid), dot_pairwise(a, b, mid, hi));
}

/* <a|b> over 2^n entries.  The range is cut into 64 aligned equal chunks (when
 * 2^n >= 2048) summed in parallel; because the recursion splits at halves this
 * is the same summation tree as a single pairwise pass. */
static ocx dot(const ocx* a, const ocx* b, int n)
{
    const uint64_t N = 1ULL << n;
    if (n < 11)
        return dot_pairwise(a, b, 0, N);
    ocx part[64];
    const uint64_t chunk = N / 64;
#pragma omp parallel for schedule(static)
    for (int p = 0; p < 64; ++p)
        part[p] = dot_pairwise(a, b, (uint64_t)p * chunk, (uint64_t)(p + 1) * chunk);
    for (int w = 1; w < 64; w *= 2)
        for (int p = 0; p < 64; p += 2 * w)
            part[p] = cx_add(part[p], part[p + w]);
    return part[0];
}

int orc_inner(int n, const double* a, const double* b, double* out2)
{
    ocx s = dot((const ocx*)a, (const ocx*)b, n);
    out2[0] = s.re;
    out2[1] = s.im;
    return 0;
}

/* dst = src over 2^n amplitudes (a plain copy, split over threads). */
static void copy_state(int n, double* dst, const double* src)
{
    const long long N2 = 2LL << n;
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < N2; ++i)
        dst[i] = src[i];
}

/* ------------------------------------------------------------ observables */

static const double PX[8] = {0, 0, 1, 0, 1, 0, 0, 0};
static const double PY[8] = {0, 0, 0, -1, 0, 1, 0, 0};
static const double PZ[8] = {1, 0, 0, 0, 0, 0, -1, 0};

/* dst = P_j src for the Pauli string (x, z), applied one qubit at a time. */
static void apply_pauli_string(int n, const double* src, double* dst, double* tmp, uint64_t x,
                               uint64_t z)
{
    copy_state(n, dst, src);
    for (int q = 0; q < n; ++q) {
        int xb = (int)((x >> q) & 1ULL), zb = (int)((z >> q) & 1ULL);
        if (!xb && !zb)
            continue;
        const double* m = xb && zb ? PY : (xb ? PX : PZ);
        orc_apply(n, dst, tmp, &q, 1, NULL, 0, m);
        copy_state(n, dst, tmp);
    }
}

/* E = sum_j coeff_j <psi|P_j|psi>; out2 = (Re E, Im E).  per_term (optional,
 * 2*nterms) receives <psi|P_j|psi> for each term. */
int orc_expect(int n, const double* psi, int nterms, const uint64_t* x, const uint64_t* z,
               const double* coeff, double* out2, double* per_term)
{
    const size_t bytes = (sizeof(double) * 2) << n;
    double* phi = (double*)malloc(bytes);
    double* tmp = (double*)malloc(bytes);
    if (!phi || !tmp) {
        free(phi);
        free(tmp);
        return -5;
    }
    double er = 0.0, ei = 0.0;
    for (int j = 0; j < nterms; ++j) {
        apply_pauli_string(n, psi, phi, tmp, x[j], z[j]);
        ocx e = dot((const ocx*)psi, (const ocx*)phi, n);
        if (per_term) {
            per_term[2 * j] = e.re;
            per_term[2 * j + 1] = e.im;
        }
        er += coeff[j] * e.re;
        ei += coeff[j] * e.im;
    }
    free(phi);
    free(tmp);
    out2[0] = er;
    out2[1] = ei;
    return 0;
}

/* lam = H psi = sum_j coeff_j P_j psi. */
int orc_apply_hamiltonian(int n, const double* psi, double* lam, int nterms, const uint64_t* x,
                             const uint64_t* z, const double* coeff)
{
    const size_t bytes = (sizeof(double) * 2) << n;
    const uint64_t N = 1ULL << n;
    double* phi = (double*)malloc(bytes);
    double* tmp = (double*)malloc(bytes);
    if (!phi || !tmp) {
        free(phi);
        free(tmp);
        return -5;
    }
    memset(lam, 0, bytes);
    for (int j = 0; j < nterms; ++j) {
        apply_pauli_string(n, psi, phi, tmp, x[j], z[j]);
#pragma omp parallel for schedule(static)
        for (long long i = 0; i < (long long)(2 * N); ++i)
            lam[i] += coeff[j] * phi[i];
    }
    free(phi);
    free(tmp);
    return 0;
}

int orc_norm2(int n, const double* psi, double* out)
{
    ocx s = dot((const ocx*)psi, (const ocx*)psi, n);
    out[0] = s.re;
    return 0;
}

/* ------------------------------------------------------ seeded random state */

/* SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014) evaluated at
 * state x: one golden-gamma step, then the two xor-shift-multiply rounds. */
static uint64_t splitmix64_at(uint64_t x)
{
    uint64_t zz = x + 0x9E3779B97F4A7C15ULL;
    zz = (zz ^ (zz >> 30)) * 0xBF58476D1CE4E5B9ULL;
    zz = (zz ^ (zz >> 27)) * 0x94D049BB133111EBULL;
    return zz ^ (zz >> 31);
}

uint64_t orc_splitmix64_at(uint64_t x)
{
    return splitmix64_at(x);
}

/* Counter-based stream of a seed.  The seed is first scrambled into a key,
 * the generator's first output from state `seed`; draw c is then the output
 * of the generator started at state `key` after c + 1 steps, i.e. the output
 * function at key + c * golden gamma.  Distinct seeds give unrelated keys, so
 * their streams are not reorderings of each other. */
static uint64_t stream_draw(uint64_t seed, uint64_t c)
{
    const uint64_t key = splitmix64_at(seed);
    return splitmix64_at(key + c * 0x9E3779B97F4A7C15ULL);
}

uint64_t orc_stream_draw(uint64_t seed, uint64_t c)
{
    return stream_draw(seed, c);
}

/* Unnormalised amplitude i: (u(i,0) - 1/2) + i (u(i,1) - 1/2) with
 * u(i,j) = top 53 bits of draw 2i+j of the seed's stream / 2^53. */
static ocx raw_amp(uint64_t seed, uint64_t i)
{
    ocx a;
    a.re = (double)(stream_draw(seed, 2 * i) >> 11) * 0x1.0p-53 - 0.5;
    a.im = (double)(stream_draw(seed, 2 * i + 1) >> 11) * 0x1.0p-53 - 0.5;
    return a;
}

/* sum_i |raw_i|^2 in a fixed order: 64 equal chunks (fewer for tiny n), each
 * summed in index order, then the chunk sums in chunk order -- so every call
 * returns the same bits whatever the thread timing. */
int orc_random_norm2(int n, uint64_t seed, double* out)
{
    const uint64_t N = 1ULL << n;
    const int nch = n >= 6 ? 64 : 1;
    const uint64_t len = N / (uint64_t)nch;
    double part[64];
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nch; ++c) {
        double s = 0.0;
        for (uint64_t i = (uint64_t)c * len; i < (uint64_t)(c + 1) * len; ++i) {
            ocx a = raw_amp(seed, i);
            s += a.re * a.re + a.im * a.im;
        }
        part[c] = s;
    }
    double s = 0.0;
    for (int c = 0; c < nch; ++c)
        s += part[c];
    out[0] = s;
    return 0;
}

/* Full normalised random state (scale = 1/sqrt(norm2) computed here). */
int orc_random_state(int n, uint64_t seed, double* psi)
{
    double s2;
    orc_random_norm2(n, seed, &s2);
    const double scale = 1.0 / sqrt(s2);
    const uint64_t N = 1ULL << n;
#pragma omp parallel for schedule(static)
    for (long long ii = 0; ii < (long long)N; ++ii) {
        ocx a = raw_amp(seed, (uint64_t)ii);
        psi[2 * ii] = a.re * scale;
        psi[2 * ii + 1] = a.im * scale;
    }
    return 0;
}

/* Amplitudes of the normalised random state at selected indices. */
int orc_random_amps(uint64_t seed, double scale, const uint64_t* idx, int m, double* out)
{
    for (int j = 0; j < m; ++j) {
        ocx a = raw_amp(seed, idx[j]);
        out[2 * j] = a.re * scale;
        out[2 * j + 1] = a.im * scale;
    }
    return 0;
}

/* eq. (1) evaluated only at the output indices idx[0..m-1], with the input
 * taken to be the normalised random state (seed, scale): one output at a time,
 * for states too large to hold twice in host memory. */
int orc_apply_sampled_random(int n, uint64_t seed, double scale, const int* t, int k, const int* ctl,
                             int c, const double* G, const uint64_t* idx, int m, double* out)
{
    if (check_qubits(n, t, k, ctl, c) != 0)
        return -1;
    const int dim = 1 << k;
    uint64_t cmask = 0;
    for (int j = 0; j < c; ++j)
        cmask |= 1ULL << ctl[j];
#pragma omp parallel for schedule(static)
    for (int j = 0; j < m; ++j) {
        uint64_t i = idx[j];
        ocx acc = {0.0, 0.0};
        if ((i & cmask) != cmask) {
            acc = raw_amp(seed, i);
            acc.re *= scale;
            acc.im *= scale;
        } else {
            uint64_t tau = tau_of(i, t, k);
            for (int tp = 0; tp < dim; ++tp) {
                ocx g = {G[((size_t)tau * dim + tp) * 2], G[((size_t)tau * dim + tp) * 2 + 1]};
                ocx a = raw_amp(seed, with_tau(i, t, k, (uint64_t)tp));
                a.re *= scale;
                a.im *= scale;
                acc = cx_add(acc, cx_mul(g, a));
            }
        }
        out[2 * j] = acc.re;
        out[2 * j + 1] = acc.im;
    }
    return 0;
}

/* ----------------------------------------------------------------- circuits */

enum { K_MATRIX = 0, K_H = 1, K_X = 2, K_Y = 3, K_Z = 4, K_RX = 5, K_RY = 6, K_RZ = 7, K_SWAP = 8 };

typedef struct {
    int nops;
    const int* kind;  /* [nops] */
    const int* k;     /* [nops] number of targets */
    const int* tgt;   /* [nops * 5] */
    const int* c;     /* [nops] number of controls */
    const int* ctl;   /* [nops * 4] */
    const int* param; /* [nops] parameter index or -1 */
    const long long* moff; /* [nops] offset (in doubles) into mats, or -1 */
    const double* mats;
} orc_circ;

static int is_rotation(int kind)
{
    return kind == K_RX || kind == K_RY || kind == K_RZ;
}

/* Gate matrix (row-major interleaved) for op o at angle theta. */
static void gate_matrix(const orc_circ* C, int o, double theta, double* G)
{
    const double r2 = 1.0 / sqrt(2.0);
    const double cth = cos(theta / 2.0), sth = sin(theta / 2.0);
    memset(G, 0, sizeof(double) * 8);
    switch (C->kind[o]) {
    case K_H:
        G[0] = r2; G[2] = r2; G[4] = r2; G[6] = -r2;
        break;
    case K_X:
        G[2] = 1.0; G[4] = 1.0;
        break;
    case K_Y:
        G[3] = -1.0; G[5] = 1.0;
        break;
    case K_Z:
        G[0] = 1.0; G[6] = -1.0;
        break;
    case K_RX: /* [[c, -i s], [-i s, c]] */
        G[0] = cth; G[3] = -sth; G[5] = -sth; G[6] = cth;
        break;
    case K_RY: /* [[c, -s], [s, c]] */
        G[0] = cth; G[2] = -sth; G[4] = sth; G[6] = cth;
        break;
    case K_RZ: /* diag(e^{-i theta/2}, e^{i theta/2}) */
        G[0] = cth; G[1] = -sth; G[6] = cth; G[7] = sth;
        break;
    default:
        break;
    }
}

/* d/dtheta of the rotation matrices above. */
static void gate_derivative(int kind, double theta, double* D)
{
    const double cth = cos(theta / 2.0), sth = sin(theta / 2.0);
    memset(D, 0, sizeof(double) * 8);
    switch (kind) {
    case K_RX: /* [[-s/2, -i c/2], [-i c/2, -s/2]] */
        D[0] = -0.5 * sth; D[3] = -0.5 * cth; D[5] = -0.5 * cth; D[6] = -0.5 * sth;
        break;
    case K_RY: /* [[-s/2, -c/2], [c/2, -s/2]] */
        D[0] = -0.5 * sth; D[2] = -0.5 * cth; D[4] = 0.5 * cth; D[6] = -0.5 * sth;
        break;
    case K_RZ: /* diag(-i/2 e^{-i theta/2}, i/2 e^{i theta/2}) */
        D[0] = -0.5 * sth; D[1] = -0.5 * cth; D[6] = -0.5 * sth; D[7] = 0.5 * cth;
        break;
    default:
        break;
    }
}

static const double SWAP4[32] = {1, 0, 0, 0, 0, 0, 0, 0,  0, 0, 0, 0, 1, 0, 0, 0,
                                 0, 0, 1, 0, 0, 0, 0, 0,  0, 0, 0, 0, 0, 0, 1, 0};

/* Conjugate transpose of a dim x dim matrix. */
static void dagger(const double* G, int dim, double* Gd)
{
    for (int r = 0; r < dim; ++r)
        for (int col = 0; col < dim; ++col) {
            Gd[((size_t)r * dim + col) * 2] = G[((size_t)col * dim + r) * 2];
            Gd[((size_t)r * dim + col) * 2 + 1] = -G[((size_t)col * dim + r) * 2 + 1];
        }
}

/* Matrix of op o (pointer into mats or filled into buf). */
static const double* op_matrix(const orc_circ* C, int o, const double* params, double* buf)
{
    if (C->kind[o] == K_MATRIX)
        return C->mats + C->moff[o];
    if (C->kind[o] == K_SWAP)
        return SWAP4;
    double theta = C->param[o] >= 0 ? params[C->param[o]] : 0.0;
    gate_matrix(C, o, theta, buf);
    return buf;
}

static int apply_op(int n, const orc_circ* C, int o, const double* params, int dag, const double* in,
                    double* out)
{
    double buf[8];
    double dbuf[32 * 32 * 2];
    const double* G = op_matrix(C, o, params, buf);
    int dim = 1 << C->k[o];
    if (dag) {
        if (dim > 32)
            return -3;
        dagger(G, dim, dbuf);
        G = dbuf;
    }
    return orc_apply(n, in, out, C->tgt + 5 * o, C->k[o], C->ctl + 4 * o, C->c[o], G);
}

/* psi = U_N..U_1 psi0 (psi0 NULL: |0..0>).  Each op maps the current state
 * into the other buffer; the two buffers then trade roles. */
static int run_circuit(int n, const orc_circ* C, const double* params, const double* psi0,
                       double* psi)
{
    const size_t bytes = (sizeof(double) * 2) << n;
    double* tmp = (double*)malloc(bytes);
    if (!tmp)
        return -5;
    if (psi0) {
        copy_state(n, psi, psi0);
    } else {
        memset(psi, 0, bytes);
        psi[0] = 1.0;
    }
    double* cur = psi;
    double* other = tmp;
    int rc = 0;
    for (int o = 0; o < C->nops && !rc; ++o) {
        rc = apply_op(n, C, o, params, 0, cur, other);
        double* t = cur;
        cur = other;
        other = t;
    }
    if (!rc && cur != psi)
        copy_state(n, psi, cur);
    free(tmp);
    return rc;
}

int orc_run(int n, int nops, const int* kind, const int* k, const int* tgt, const int* c,
            const int* ctl, const int* param, const long long* moff, const double* mats,
            const double* params, const double* psi0, double* psi)
{
    orc_circ C = {nops, kind, k, tgt, c, ctl, param, moff, mats};
    return run_circuit(n, &C, params, psi0, psi);
}

static int energy_of(int n, const orc_circ* C, const double* params, int nterms, const uint64_t* x,
                     const uint64_t* z, const double* coeff, double* psi, double* E)
{
    int rc = run_circuit(n, C, params, NULL, psi);
    if (rc)
        return rc;
    double e2[2];
    rc = orc_expect(n, psi, nterms, x, z, coeff, e2, NULL);
    *E = e2[0];
    return rc;
}

int orc_energy(int n, int nops, const int* kind, const int* k, const int* tgt, const int* c,
               const int* ctl, const int* param, const long long* moff, const double* mats,
               const double* params, int nterms, const uint64_t* x, const uint64_t* z,
               const double* coeff, double* E)
{
    orc_circ C = {nops, kind, k, tgt, c, ctl, param, moff, mats};
    double* psi = (double*)malloc((sizeof(double) * 2) << n);
    if (!psi)
        return -5;
    int rc = energy_of(n, &C, params, nterms, x, z, coeff, psi, E);
    free(psi);
    return rc;
}

/* Gradient entries for parameters which[0..m-1].  mode 0: parameter shift
 * [E(theta+pi/2) - E(theta-pi/2)]/2 (exact for exp(-i theta P/2); requires each
 * such parameter to drive only uncontrolled rotations); mode 1: central
 * finite difference with step h. */
int orc_grad(int n, int nops, const int* kind, const int* k, const int* tgt, const int* c,
             const int* ctl, const int* param, const long long* moff, const double* mats,
             const double* params, int nparams, int nterms, const uint64_t* x, const uint64_t* z,
             const double* coeff, const int* which, int m, int mode, double h, double* grad)
{
    orc_circ C = {nops, kind, k, tgt, c, ctl, param, moff, mats};
    if (mode == 0) {
        for (int j = 0; j < m; ++j)
            for (int o = 0; o < nops; ++o)
                if (param[o] == which[j] && (!is_rotation(kind[o]) || c[o] != 0))
                    return -3;
    }
    double* psi = (double*)malloc((sizeof(double) * 2) << n);
    double* th = (double*)malloc(sizeof(double) * (size_t)(nparams > 0 ? nparams : 1));
    if (!psi || !th) {
        free(psi);
        free(th);
        return -5;
    }
    const double step = mode == 0 ? M_PI / 2.0 : h;
    int rc = 0;
    for (int j = 0; j < m && !rc; ++j) {
        double ep, em;
        memcpy(th, params, sizeof(double) * (size_t)nparams);
        th[which[j]] = params[which[j]] + step;
        rc = energy_of(n, &C, th, nterms, x, z, coeff, psi, &ep);
        th[which[j]] = params[which[j]] - step;
        if (!rc)
            rc = energy_of(n, &C, th, nterms, x, z, coeff, psi, &em);
        grad[j] = mode == 0 ? 0.5 * (ep - em) : (ep - em) / (2.0 * h);
    }
    free(psi);
    free(th);
    return rc;
}

/* Adjoint-method gradient (Jones & Gacon, arXiv:2009.02823): forward state
 * phi = U_N..U_1|0>, lam = H phi, E = Re<phi|lam>; then for each op from last
 * to first: phi <- U^dagger phi; for rotations g += 2 Re <lam | dU phi> where
 * dU is the entrywise derivative of the (controlled) rotation, zero on the
 * control-off subspace; lam <- U^dagger lam. */
int orc_adjoint(int n, int nops, const int* kind, const int* k, const int* tgt, const int* c,
                const int* ctl, const int* param, const long long* moff, const double* mats,
                const double* params, int nparams, int nterms, const uint64_t* x,
                const uint64_t* z, const double* coeff, double* E, double* grad)
{
    orc_circ C = {nops, kind, k, tgt, c, ctl, param, moff, mats};
    const size_t bytes = (sizeof(double) * 2) << n;
    const uint64_t N = 1ULL << n;
    double* phi = (double*)malloc(bytes);
    double* lam = (double*)malloc(bytes);
    double* mu = (double*)malloc(bytes);
    if (!phi || !lam || !mu) {
        free(phi);
        free(lam);
        free(mu);
        return -5;
    }
    int rc = run_circuit(n, &C, params, NULL, phi);
    if (!rc)
        rc = orc_apply_hamiltonian(n, phi, lam, nterms, x, z, coeff);
    if (!rc) {
        ocx e = dot((const ocx*)phi, (const ocx*)lam, n);
        *E = e.re;
    }
    for (int p = 0; p < nparams; ++p)
        grad[p] = 0.0;
    /* phi, lam and mu are three buffers; after U^dagger maps one of phi, lam
     * into mu, the two pointers trade places (no copy). */
    for (int o = nops - 1; o >= 0 && !rc; --o) {
        double* t;
        rc = apply_op(n, &C, o, params, 1, phi, mu);
        if (rc)
            break;
        t = phi;
        phi = mu;
        mu = t;
        if (C.param[o] >= 0 && is_rotation(C.kind[o])) {
            double D[8];
            gate_derivative(C.kind[o], params[C.param[o]], D);
            rc = orc_apply(n, phi, mu, C.tgt + 5 * o, 1, C.ctl + 4 * o, C.c[o], D);
            if (rc)
                break;
            uint64_t cmask = 0;
            for (int j = 0; j < C.c[o]; ++j)
                cmask |= 1ULL << C.ctl[4 * o + j];
            if (cmask != 0) {
#pragma omp parallel for schedule(static)
                for (long long ii = 0; ii < (long long)N; ++ii)
                    if (((uint64_t)ii & cmask) != cmask) {
                        mu[2 * ii] = 0.0;
                        mu[2 * ii + 1] = 0.0;
                    }
            }
            ocx g = dot((const ocx*)lam, (const ocx*)mu, n);
            grad[C.param[o]] += 2.0 * g.re;
        }
        rc = apply_op(n, &C, o, params, 1, lam, mu);
        if (rc)
            break;
        t = lam;
        lam = mu;
        mu = t;
    }
    free(phi);
    free(lam);
    free(mu);
    return rc;
}

/* ------------------------------------------------------------ measurement */

/* Simulated measurement (Sec. 3: measurements are simulated by sampling from
 * the state).  Born rule: outcome i has probability |psi_i|^2 (no
 * normalisation is applied; the state's own norm is the total mass). */

/* Marginal distribution of the qubits q[0..m-1]: out[b] = sum of |psi_i|^2
 * over every i whose bits at q[0..m-1] spell b, q[0] being the most
 * significant bit of b (the same order as gate targets).  Plain loop over i in
 * index order. */
int orc_probabilities(int n, const double* psi, const int* q, int m, double* out)
{
    if (n < 1 || n > 40 || m < 1 || m > n)
        return -1;
    uint64_t seen = 0;
    for (int j = 0; j < m; ++j) {
        if (q[j] < 0 || q[j] >= n || ((seen >> q[j]) & 1ULL))
            return -1;
        seen |= 1ULL << q[j];
    }
    const uint64_t N = 1ULL << n;
    const uint64_t M = 1ULL << m;
    for (uint64_t b = 0; b < M; ++b)
        out[b] = 0.0;
    for (uint64_t i = 0; i < N; ++i) {
        const double p = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
        out[tau_of(i, q, m)] += p;
    }
    return 0;
}

/* Inverse-transform sampling of whole-register outcomes.  With the running
 * sums C_i = sum_{j <= i} |psi_j|^2 (taken in index order) and T = C_{N-1},
 * shot s maps its uniform u[s] to t = u[s] * T and returns the smallest i
 * with C_i > t.  If no such i exists (t >= T, which only rounding, u >= 1 or
 * a NaN can cause) it returns the smallest i with C_i == T, i.e. the last
 * outcome of nonzero probability (0 for the zero vector).  A negative u counts
 * as 0.  Outcomes of zero probability are never returned otherwise either:
 * C_i > t >= C_{i-1} means |psi_i|^2 > 0. */
int orc_sample(int n, const double* psi, const double* u, int64_t nshots, int64_t* out)
{
    if (n < 1 || n > 40 || nshots < 0)
        return -1;
    const uint64_t N = 1ULL << n;
    double* C = (double*)malloc(N * sizeof(double));
    if (!C)
        return -2;
    double run = 0.0;
    for (uint64_t i = 0; i < N; ++i) {
        run += psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
        C[i] = run;
    }
    const double T = C[N - 1];
    for (int64_t s = 0; s < nshots; ++s) {
        double t = u[s] * T;
        if (t < 0.0) /* u < 0 counts as u = 0 */
            t = 0.0;
        /* C is nondecreasing, so "the smallest i with C_i > t" is found by
         * bisection: lo is the answer once the range closes. */
        uint64_t lo = 0, hi = N;
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (C[mid] > t)
                hi = mid;
            else
                lo = mid + 1;
        }
        if (lo == N) {
            lo = 0;
            hi = N - 1;
            while (lo < hi) { /* smallest i with C_i >= T */
                const uint64_t mid = lo + (hi - lo) / 2;
                if (C[mid] >= T)
                    hi = mid;
                else
                    lo = mid + 1;
            }
        }
        out[s] = (int64_t)lo;
    }
    free(C);
    return 0;
}

/* Frequencies of measured outcomes: counts[b] = number of shots s whose
 * whole-register outcome samples[s] has bits q[0..m-1] spelling b (q[0] the
 * most significant bit of b, as for marginals).  Plain loop over shots. */
int orc_frequencies(int n, const int64_t* samples, int64_t nshots, const int* q, int m, int64_t* counts)
{
    if (n < 1 || n > 40 || m < 1 || m > n || nshots < 0)
        return -1;
    uint64_t seen = 0;
    for (int j = 0; j < m; ++j) {
        if (q[j] < 0 || q[j] >= n || ((seen >> q[j]) & 1ULL))
            return -1;
        seen |= 1ULL << q[j];
    }
    for (uint64_t b = 0; b < (1ULL << m); ++b)
        counts[b] = 0;
    for (int64_t s = 0; s < nshots; ++s)
        counts[tau_of((uint64_t)samples[s], q, m)] += 1;
    return 0;
}

/* Post-measurement state (Sec. 3: measurements; projective collapse): for the
 * outcome b of qubits q[0..m-1] (q[0] the most significant bit of b) with
 * probability p, out[i] = psi[i] / sqrt(p) where the bits of i at q spell b,
 * and 0 elsewhere.  p <= 0 (an impossible outcome) gives the zero vector. */
int orc_collapse(int n, const double* psi, double* out, const int* q, int m, uint64_t b, double p)
{
    if (n < 1 || n > 40 || m < 1 || m > n || (m < 64 && b >= (1ULL << m)))
        return -1;
    uint64_t seen = 0;
    for (int j = 0; j < m; ++j) {
        if (q[j] < 0 || q[j] >= n || ((seen >> q[j]) & 1ULL))
            return -1;
        seen |= 1ULL << q[j];
    }
    const uint64_t N = 1ULL << n;
    const double s = p > 0.0 ? 1.0 / sqrt(p) : 0.0;
    for (uint64_t i = 0; i < N; ++i) {
        const int keep = tau_of(i, q, m) == b;
        out[2 * i] = keep ? psi[2 * i] * s : 0.0;
        out[2 * i + 1] = keep ? psi[2 * i + 1] * s : 0.0;
    }
    return 0;
}

/* Seeded uniforms for sampling: u[s] = (draw s of the seed's stream >> 11) /
 * 2^53, the top 53 bits of the draw, in [0, 1). */
int orc_uniforms(uint64_t seed, int64_t count, double* u)
{
    if (count < 0)
        return -1;
    for (int64_t s = 0; s < count; ++s)
        u[s] = (double)(stream_draw(seed, (uint64_t)s) >> 11) * (1.0 / 9007199254740992.0);
    return 0;
}
