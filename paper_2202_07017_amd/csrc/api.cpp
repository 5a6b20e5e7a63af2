// Host side of libqsv.so: argument validation, canonical gate forms, kernel
// selection, the fusion planner, plans with HIP-graph replay, and the adjoint
// gradient driver.  Every public function validates before it enqueues.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "qsv.h"
#include "qsv_internal.h"
#include "qsv_expect.h"
#include "qsv_host.h"
#include "qsv_rpass.h"
#include "qsv_span.h"

using namespace qsv;

// ------------------------------------------------------------------ errors

namespace qsv {
thread_local std::string t_err = "no error";

qsv_status fail(qsv_status st, const char* fmt, ...)
{
    char buf[768];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return st;
}

qsv_status ok()
{
    t_err = "no error";
    return QSV_OK;
}

qsv_status enqueue_gate()
{
    const char* v = std::getenv("QSV_TEST_FAIL_LAUNCH");
    if (v && v[0] == '1' && v[1] == '\0')
        return fail(QSV_ERR_HIP, "kernel launch failed: unspecified launch failure "
                                 "(forced by QSV_TEST_FAIL_LAUNCH=1; nothing was enqueued)");
    return QSV_OK;
}

size_t amp_bytes(int dt)
{
    return dt == QSV_C64 ? 8 : 16;
}

qsv_status check_n_dt(int n, int dt)
{
    if (n < 1 || n > QSV_MAX_QUBITS)
        return fail(QSV_ERR_ARG, "n = %d outside [1, %d]", n, QSV_MAX_QUBITS);
    if (dt != QSV_C64 && dt != QSV_C128)
        return fail(QSV_ERR_ARG, "dtype %d is neither QSV_C64 (1) nor QSV_C128 (2)", dt);
    return QSV_OK;
}

qsv_status check_state(const void* psi, int n, int dt, const char* what)
{
    qsv_status st = check_n_dt(n, dt);
    if (st)
        return st;
    if (!psi)
        return fail(QSV_ERR_ARG, "%s is NULL", what);
    if (reinterpret_cast<uintptr_t>(psi) % 16)
        return fail(QSV_ERR_ARG, "%s is not 16-byte aligned", what);
    return QSV_OK;
}

qsv_status check_qubits(int n, const int* t, int k, int kmax, const int* c, int nc)
{
    if (k < 1 || k > kmax)
        return fail(QSV_ERR_ARG, "k = %d outside [1, %d]", k, kmax);
    if (nc < 0)
        return fail(QSV_ERR_ARG, "negative control count %d", nc);
    if (k + nc > n)
        return fail(QSV_ERR_ARG, "k + c = %d exceeds n = %d", k + nc, n);
    if (!t)
        return fail(QSV_ERR_ARG, "targets is NULL");
    if (nc > 0 && !c)
        return fail(QSV_ERR_ARG, "controls is NULL with c = %d", nc);
    uint64_t seen = 0;
    for (int j = 0; j < k + nc; ++j) {
        const int q = j < k ? t[j] : c[j - k];
        if (q < 0 || q >= n)
            return fail(QSV_ERR_QUBIT, "qubit %d outside [0, %d)", q, n);
        if ((seen >> q) & 1ull)
            return fail(QSV_ERR_QUBIT, "qubit %d appears twice among targets and controls", q);
        seen |= 1ull << q;
    }
    return QSV_OK;
}

qsv_status check_hamiltonian(const qsv_pauli_sum* H, int n)
{
    if (!H || H->nterms < 1 || !H->x_mask || !H->z_mask || !H->coeff)
        return fail(QSV_ERR_ARG, "Pauli sum is NULL, empty or has NULL arrays");
    const uint64_t lim = n >= 64 ? ~0ull : ((1ull << n) - 1);
    for (int j = 0; j < H->nterms; ++j)
        if ((H->x_mask[j] | H->z_mask[j]) & ~lim)
            return fail(QSV_ERR_QUBIT, "Pauli term %d acts on a qubit >= n = %d", j, n);
    return QSV_OK;
}

// ---------------------------------------------------- canonical gate forms

InsertSpec make_ins(std::vector<int> pos, uint64_t setmask)
{
    std::sort(pos.begin(), pos.end());
    InsertSpec s{};
    s.nins = (int)pos.size();
    s.setmask = setmask;
    for (size_t j = 0; j < pos.size(); ++j)
        s.low[j] = (1ull << pos[j]) - 1;
    return s;
}

// Targets sorted ascending; canonical tau bit j <-> ct[j].  The user's first
// target is the most significant bit of the user's tau.
void canonicalize(const int* t, int k, const double* G, int* ct, std::vector<double>& Gc)
{
    const int D = 1 << k;
    int order[QSV_MAX_TARGETS];
    for (int j = 0; j < k; ++j)
        order[j] = j;
    std::sort(order, order + k, [&](int a, int b) { return t[a] < t[b]; });
    for (int j = 0; j < k; ++j)
        ct[j] = t[order[j]];
    auto to_user = [&](int tc) {
        int tu = 0;
        for (int j = 0; j < k; ++j)
            if ((tc >> j) & 1)
                tu |= 1 << (k - 1 - order[j]);
        return tu;
    };
    Gc.assign((size_t)2 * D * D, 0.0);
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            const size_t u = ((size_t)to_user(r) * D + to_user(c)) * 2;
            Gc[((size_t)r * D + c) * 2] = G[u];
            Gc[((size_t)r * D + c) * 2 + 1] = G[u + 1];
        }
}

static uint64_t deposit(uint64_t v, const int* pos, int m, int shift)
{
    uint64_t o = 0;
    for (int j = 0; j < m; ++j)
        if ((v >> j) & 1ull)
            o |= 1ull << (pos[j] - shift);
    return o;
}

// Build the launch for eq. (1) with canonical (ct, Gc) and controls.
// `upload` receives bytes the kernel needs in device memory (set gdev to them).
Built build_launch(int n, int dt, const int* ct, int k, const int* ctl, int c, const double* Gc,
                   bool allow_mfma)
{
    Built b;
    GateLaunch& L = b.L;
    L.dt = dt;
    L.n = n;
    L.lowq = ct[0];
    for (int j = 0; j < c; ++j)
        L.lowq = std::min(L.lowq, ctl[j]);
    const int D = 1 << k;
    const size_t S = amp_bytes(dt);
    uint64_t cmask = 0;
    bool ctl0 = false;
    for (int j = 0; j < c; ++j) {
        cmask |= 1ull << ctl[j];
        ctl0 |= ctl[j] == 0;
    }
    auto G = [&](int r, int col, int part) { return Gc[((size_t)r * D + col) * 2 + part]; };

    bool diag = true, perm = true, ident = true;
    int src[32];
    for (int r = 0; r < D; ++r) {
        int ones = 0;
        for (int col = 0; col < D; ++col) {
            const double re = G(r, col, 0), im = G(r, col, 1);
            if (r != col && (re != 0.0 || im != 0.0))
                diag = false;
            if (im != 0.0 || (re != 0.0 && re != 1.0))
                perm = false;
            if (re == 1.0 && im == 0.0) {
                ++ones;
                src[r] = col;
            }
            if (r == col && (re != 1.0 || im != 0.0))
                ident = false;
        }
        if (ones != 1)
            perm = false;
    }
    if (perm) {
        int seen[32] = {0};
        for (int r = 0; r < D; ++r)
            if (seen[src[r]]++)
                perm = false;
    }
    if (diag && ident) {
        b.noop = true;
        return b;
    }
    std::vector<int> tgt(ct, ct + k), ctlv(ctl, ctl + c);
    if (perm) {
        L.type = L_PERM;
        std::vector<int> pos = tgt;
        pos.insert(pos.end(), ctlv.begin(), ctlv.end());
        const bool bit0 = std::find(pos.begin(), pos.end(), 0) != pos.end();
        const int shift = (dt == QSV_C64 && !bit0) ? 1 : 0;
        L.mode = shift ? W2 : W1;
        for (int& p : pos)
            p -= shift;
        L.ins = make_ins(pos, cmask >> shift);
        L.ngroups = 1ull << (n - shift - (int)pos.size());
        int m = 0;
        for (int r = 0; r < D; ++r)
            if (src[r] != r) {
                L.off[m] = deposit((uint64_t)r, ct, k, shift);
                L.off2[m] = deposit((uint64_t)src[r], ct, k, shift);
                ++m;
            }
        L.nmoved = m;
        if (k == 2 && c == 0 && src[0] == 0 && src[1] == 2 && src[2] == 1 && src[3] == 3) {
            L.swapq[0] = ct[0];
            L.swapq[1] = ct[1];
        }
        const double groups = std::ldexp(1.0, n - k - c);
        L.bytes = 2.0 * S * groups * m;
        return b;
    }
    if (diag) {
        L.type = L_DIAG;
        int nontriv = 0, tstar = 0;
        for (int r = 0; r < D; ++r)
            if (G(r, r, 0) != 1.0 || G(r, r, 1) != 0.0) {
                ++nontriv;
                tstar = r;
            }
        std::vector<int> pos = ctlv;
        uint64_t set = cmask;
        if (nontriv == 1) {
            pos.insert(pos.end(), tgt.begin(), tgt.end());
            set |= deposit((uint64_t)tstar, ct, k, 0);
            L.K = 0;
            L.g = {G(tstar, tstar, 0), G(tstar, tstar, 1)};
        } else {
            L.K = k;
            for (int j = 0; j < k; ++j)
                L.tpos[j] = ct[j];
            L.g.resize((size_t)2 * D);
            for (int r = 0; r < D; ++r) {
                L.g[2 * r] = G(r, r, 0);
                L.g[2 * r + 1] = G(r, r, 1);
            }
        }
        const bool bit0 = std::find(pos.begin(), pos.end(), 0) != pos.end();
        const int shift = (dt == QSV_C64 && !bit0) ? 1 : 0;
        L.mode = shift ? W2 : W1;
        for (int& p : pos)
            p -= shift;
        L.ins = make_ins(pos, set >> shift);
        L.ngroups = 1ull << (n - shift - (int)pos.size());
        const double touched = std::ldexp(1.0, n - (int)pos.size() - shift) * (shift ? 2 : 1);
        L.bytes = 2.0 * S * touched;
        L.flops = 6.0 * touched;
        return b;
    }
    // dense
    const char* nomfma = getenv("QSV_NO_MFMA");
    // An uncontrolled dense 2- or 3-qubit gate with a target among the three
    // lowest bits of the 16-byte unit index (complex128: qubits 0-2;
    // complex64, two amplitudes to a unit: qubits 1-3) gives each lane a
    // group of 2-8 contiguous units, so one load instruction of a wave
    // spreads over up to 8 times the bytes it uses.  Such a gate runs as the
    // 4-qubit block G (x) I (the added qubits the lowest free ones) on the
    // matrix cores, whose tiles are contiguous runs of >= 2 KiB: measured at
    // n = 30 and 32 it is never slower and up to 1.6 times faster (e.g.
    // complex128 (0,1,2) 3.95 -> 5.9 TB/s, complex64 (1,2,3) 3.8 -> 6.0).
    if (allow_mfma && c == 0 && (k == 2 || k == 3) && n >= 10 && !(nomfma && nomfma[0] == '1')) {
        const int lo = dt == QSV_C64 ? 1 : 0;
        bool low = false;
        for (int j = 0; j < k; ++j)
            low |= ct[j] >= lo && ct[j] < lo + 3;
        if (low) {
            int ct4[4];
            std::vector<int> all(ct, ct + k);
            for (int q = 0; (int)all.size() < 4; ++q)
                if (std::find(all.begin(), all.end(), q) == all.end())
                    all.push_back(q);
            std::sort(all.begin(), all.end());
            std::copy(all.begin(), all.end(), ct4);
            int idx[3];  // canonical tau bit of original target j inside ct4
            for (int j = 0; j < k; ++j)
                idx[j] = (int)(std::find(all.begin(), all.end(), ct[j]) - all.begin());
            int extra = 0;  // tau bits of the added qubits
            for (int j = 0; j < 4; ++j)
                if (std::find(ct, ct + k, ct4[j]) == ct + k)
                    extra |= 1 << j;
            auto orig = [&](int t4) {
                int t = 0;
                for (int j = 0; j < k; ++j)
                    t |= ((t4 >> idx[j]) & 1) << j;
                return t;
            };
            std::vector<double> G4((size_t)2 * 16 * 16, 0.0);
            for (int r = 0; r < 16; ++r)
                for (int col = 0; col < 16; ++col)
                    if ((r & extra) == (col & extra)) {
                        G4[((size_t)r * 16 + col) * 2] = G(orig(r), orig(col), 0);
                        G4[((size_t)r * 16 + col) * 2 + 1] = G(orig(r), orig(col), 1);
                    }
            Built b4 = build_launch(n, dt, ct4, 4, ctl, 0, G4.data(), true);
            b4.L.flops = 8.0 * D * std::ldexp(1.0, n);
            return b4;
        }
    }
    L.K = k;
    L.flops = 8.0 * D * std::ldexp(1.0, n - c);
    L.bytes = 2.0 * S * std::ldexp(1.0, n - c);
    if (allow_mfma && c == 0 && k >= 4 && n >= k + 6 && !(nomfma && nomfma[0] == '1')) {
        L.type = L_MFMA;
        std::vector<int> B = tgt;
        for (int q = 0, got = 0; got < 6; ++q)
            if (std::find(tgt.begin(), tgt.end(), q) == tgt.end()) {
                B.push_back(q);
                ++got;
            }
        std::sort(B.begin(), B.end());
        int Lr = 0;
        while (Lr < (int)B.size() && B[Lr] == Lr)
            ++Lr;
        L.L = Lr;
        auto rank = [&](int q) { return (int)(std::find(B.begin(), B.end(), q) - B.begin()); };
        for (int j = 0; j < k; ++j)
            L.tloc[j] = rank(ct[j]);
        int fj = 0;
        for (int q : B)
            if (std::find(tgt.begin(), tgt.end(), q) == tgt.end())
                L.floc[fj++] = rank(q);
        const int nch = 1 << ((int)B.size() - Lr);
        for (int cidx = 0; cidx < nch; ++cidx) {
            uint64_t o = 0;
            for (int m = 0; m < (int)B.size() - Lr; ++m)
                if ((cidx >> m) & 1)
                    o |= 1ull << B[Lr + m];
            L.choff[cidx] = o;
        }
        L.ins = make_ins(B, 0);
        L.ntiles = 1ull << (n - k - 6);
        L.ngroups = L.ntiles;
        // Three-product kernel by default (complex128 k = 5 with one tile per
        // workgroup ran 6-10% slower than the real embedding, with two 0-7%
        // faster and with four faster still, measured); QSV_MFMA_FORM=real
        // selects the embedding.
        const char* form = std::getenv("QSV_MFMA_FORM");
        L.mfma3 = 1;
        if (form && std::strcmp(form, "real") == 0)
            L.mfma3 = 0;
        else if (form && std::strcmp(form, "3m") == 0)
            L.mfma3 = 1;
        // Tiles per workgroup of the three-product kernel, measured at n = 28
        // and 30 over random and structured target sets: k = 5 takes four
        // (the loads of the next tile run under the current one's products;
        // complex128 5-18% faster than two on nearly every set, complex64 4%
        // on average at n = 30 and even at n = 28), k = 4 two when its
        // targets lie in a window of 8 qubits (1-5% faster) and one
        // otherwise (the prefetch then costs about as much as it hides).
        // QSV_MFMA_TPB=1|2|4 forces a count (comparisons).
        // Small states keep at least 2048 workgroups (eight per CU): at n = 20
        // four tiles per workgroup left 128 of them and the fused U(2)+CZ
        // circuit ran 0.34 -> 0.43 ms.
        const int span = *std::max_element(tgt.begin(), tgt.end()) - *std::min_element(tgt.begin(), tgt.end());
        L.mfma_tpb = k == 5 ? 4 : (span < 2 * k ? 2 : 1);
        while (L.mfma_tpb > 1 && L.ntiles / (uint64_t)L.mfma_tpb < 2048)
            L.mfma_tpb /= 2;
        if (const char* e = std::getenv("QSV_MFMA_TPB")) {
            const int v = std::atoi(e);
            if (v == 1 || v == 2 || v == 4)
                L.mfma_tpb = v;
        }
        if (L.mfma3)
            mfma3_fragments(Gc, k, dt, b.upload);
        else
            mfma_fragments(Gc, k, dt, b.upload);
        return b;
    }
    L.type = L_DENSE;
    std::vector<int> pos;
    int shift = 0;
    if (dt == QSV_C64 && ct[0] == 0) {
        L.mode = INTRA;
        shift = 1;
        for (int j = 1; j < k; ++j)
            pos.push_back(ct[j] - 1);
        for (int q : ctlv)
            pos.push_back(q - 1);
        for (int v = 0; v < D / 2; ++v)
            L.off[v] = deposit((uint64_t)v, ct + 1, k - 1, 1);
    } else if (dt == QSV_C64 && !ctl0) {
        L.mode = W2;
        shift = 1;
        for (int q : tgt)
            pos.push_back(q - 1);
        for (int q : ctlv)
            pos.push_back(q - 1);
        for (int v = 0; v < D; ++v)
            L.off[v] = deposit((uint64_t)v, ct, k, 1);
    } else {
        L.mode = W1;
        pos = tgt;
        pos.insert(pos.end(), ctlv.begin(), ctlv.end());
        for (int v = 0; v < D; ++v)
            L.off[v] = deposit((uint64_t)v, ct, k, 0);
    }
    L.ins = make_ins(pos, cmask >> shift);
    L.ngroups = 1ull << (n - shift - (int)pos.size());
    if (k <= 3) {
        L.g.assign(Gc, Gc + (size_t)2 * D * D);
    } else {
        const size_t cnt = (size_t)2 * D * D;
        b.upload.resize(cnt * (dt == QSV_C64 ? 4 : 8));
        for (size_t j = 0; j < cnt; ++j) {
            if (dt == QSV_C64)
                reinterpret_cast<float*>(b.upload.data())[j] = (float)Gc[j];
            else
                reinterpret_cast<double*>(b.upload.data())[j] = Gc[j];
        }
    }
    return b;
}

// Launch for an unbound rotation exp(-i theta P/2) on `target` with controls.
GateLaunch rotation_launch(int n, int dt, int rot, int target, const int* ctl, int c, int pidx)
{
    GateLaunch L;
    L.dt = dt;
    L.n = n;
    L.rot = rot;
    L.pidx = pidx;
    L.lowq = target;
    for (int j = 0; j < c; ++j)
        L.lowq = std::min(L.lowq, ctl[j]);
    const size_t S = amp_bytes(dt);
    uint64_t cmask = 0;
    bool ctl0 = false;
    std::vector<int> ctlv(ctl, ctl + c);
    for (int q : ctlv) {
        cmask |= 1ull << q;
        ctl0 |= q == 0;
    }
    L.bytes = 2.0 * S * std::ldexp(1.0, n - c);
    if (rot == ROT_Z) {
        L.type = L_DIAG;
        L.K = 1;
        L.tpos[0] = target;
        const int shift = (dt == QSV_C64 && !ctl0) ? 1 : 0;
        L.mode = shift ? W2 : W1;
        std::vector<int> pos = ctlv;
        for (int& p : pos)
            p -= shift;
        L.ins = make_ins(pos, cmask >> shift);
        L.ngroups = 1ull << (n - shift - c);
        L.flops = 6.0 * std::ldexp(1.0, n - c);
        return L;
    }
    L.type = L_DENSE;
    L.K = 1;
    L.flops = 16.0 * std::ldexp(1.0, n - c);
    std::vector<int> pos;
    int shift = 0;
    if (dt == QSV_C64 && target == 0) {
        L.mode = INTRA;
        shift = 1;
        for (int q : ctlv)
            pos.push_back(q - 1);
        L.off[0] = 0;
    } else if (dt == QSV_C64 && !ctl0) {
        L.mode = W2;
        shift = 1;
        pos.push_back(target - 1);
        for (int q : ctlv)
            pos.push_back(q - 1);
        L.off[0] = 0;
        L.off[1] = 1ull << (target - 1);
    } else {
        L.mode = W1;
        pos.push_back(target);
        pos.insert(pos.end(), ctlv.begin(), ctlv.end());
        L.off[0] = 0;
        L.off[1] = 1ull << target;
    }
    L.ins = make_ins(pos, cmask >> shift);
    L.ngroups = 1ull << (n - shift - (int)pos.size());
    return L;
}

// -------------------------------------------------------- device staging

namespace {
// Per (device, stream) ring of device slots for the tables of single calls
// (qsv_apply_gate / qsv_apply_fused with k >= 4).  A slot is filled by a
// staging kernel on the stream, so its reuse is ordered after the kernel that
// read it, and no host thread ever waits for the device.
constexpr int kStageSlots = 8;
constexpr size_t kStageSlotBytes = 32768;  // the largest table: k = 5 complex128 matrix-core fragments
struct StageRing {
    unsigned char* dev = nullptr;
    int next = 0;
};
std::mutex g_stage_mu;
std::map<std::pair<int, hipStream_t>, StageRing> g_stage;
}  // namespace

qsv_status stage_upload(const void* host, size_t bytes, hipStream_t s, const void** dev_out)
{
    if (bytes > kStageSlotBytes)
        return fail(QSV_ERR_UNSUPPORTED, "staged table of %zu bytes exceeds the %zu-byte slot", bytes,
                    kStageSlotBytes);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    unsigned char* slot = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        StageRing& r = g_stage[{dev, s}];
        if (!r.dev) {
            void* p = nullptr;
            if (hipMalloc(&p, kStageSlots * kStageSlotBytes) != hipSuccess)
                return fail(QSV_ERR_NOMEM, "staging ring of %zu bytes", kStageSlots * kStageSlotBytes);
            r.dev = static_cast<unsigned char*>(p);
        }
        slot = r.dev + (size_t)r.next * kStageSlotBytes;
        r.next = (r.next + 1) % kStageSlots;
    }
    // pad to a whole number of 16-byte words
    const size_t padded = (bytes + 15) & ~(size_t)15;
    if (padded != bytes) {
        std::vector<unsigned char> tmp(padded, 0);
        std::memcpy(tmp.data(), host, bytes);
        e = launch_stage(slot, tmp.data(), padded, s);
    } else {
        e = launch_stage(slot, host, bytes, s);
    }
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "staging launch: %s", hipGetErrorString(e));
    *dev_out = slot;
    return QSV_OK;
}

qsv_status launch_checked(const GateLaunch& L, void* psi, void* psi2, hipStream_t s)
{
    hipError_t e;
    if (L.type == L_DIAGRUN)
        e = psi2 ? hipErrorInvalidValue : launch_diag_run(L, psi, s);
    else if (L.type == L_QPERM)
        e = launch_qperm(L, psi, psi2, s);
    else
        e = launch_gate(L, psi, psi2, s);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return QSV_OK;
}

// Group a Pauli sum into diagonal chunks and per-x-mask chunks.
void group_terms(const qsv_pauli_sum* H, std::vector<TermChunk>& diag,
                 std::vector<std::pair<uint64_t, TermChunk>>& pairs)
{
    std::map<uint64_t, std::vector<int>> byx;
    std::vector<int> order;
    for (int j = 0; j < H->nterms; ++j) {
        if (byx.find(H->x_mask[j]) == byx.end())
            order.push_back(j);
        byx[H->x_mask[j]].push_back(j);
    }
    for (int first : order) {
        const uint64_t x = H->x_mask[first];
        const std::vector<int>& js = byx[x];
        for (size_t s0 = 0; s0 < js.size(); s0 += kMaxTermsPerLaunch) {
            TermChunk t{};
            for (size_t s1 = s0; s1 < js.size() && s1 < s0 + kMaxTermsPerLaunch; ++s1) {
                const int j = js[s1];
                t.z[t.nt] = H->z_mask[j];
                t.c[t.nt] = H->coeff[j];
                t.ylo[t.nt] = __builtin_popcountll(H->x_mask[j] & H->z_mask[j]) & 3;
                ++t.nt;
            }
            if (x == 0)
                diag.push_back(t);
            else
                pairs.push_back({x, t});
        }
    }
}

// Split a Pauli sum into tiled passes (n >= kTileQubits).  Pass 0 uses the
// low 12 qubits and takes every diagonal term plus every term whose x mask
// lies there; later passes use qubits [0, L) with L >= 6 plus up to 12 - L
// higher qubits chosen greedily from the x masks left.  A term whose x mask
// has more than 6 qubits above 5 goes to `leftover` (per-mask pair kernel).
void plan_tiles(const qsv_pauli_sum* H, int n, std::vector<TileExpK>& out,
                std::vector<std::pair<uint64_t, TermChunk>>& leftover)
{
    struct T {
        uint64_t x, z;
        double c;
        int ylo;
    };
    std::vector<T> all;
    for (int j = 0; j < H->nterms; ++j)
        all.push_back(T{H->x_mask[j], H->z_mask[j], H->coeff[j],
                        __builtin_popcountll(H->x_mask[j] & H->z_mask[j]) & 3});
    std::vector<std::pair<uint32_t, std::vector<T>>> passes;  // (tile mask, terms)
    const uint64_t low12 = (1ull << kTileQubits) - 1;
    std::vector<T> p0, rest;
    for (const T& t : all)
        (((t.x & ~low12) == 0) ? p0 : rest).push_back(t);
    passes.push_back({(uint32_t)low12, p0});
    std::vector<bool> used(rest.size(), false);
    size_t left = rest.size();
    while (left > 0) {
        uint64_t Hm = 0;
        std::vector<T> take;
        for (size_t j = 0; j < rest.size(); ++j) {
            if (used[j])
                continue;
            const uint64_t hb = rest[j].x & ~0x3Full;
            if (__builtin_popcountll(Hm | hb) <= kTileQubits - 6) {
                Hm |= hb;
                take.push_back(rest[j]);
                used[j] = true;
                --left;
            }
        }
        if (take.empty()) {  // the first unused term cannot fit any tile
            for (size_t j = 0; j < rest.size(); ++j)
                if (!used[j]) {
                    TermChunk tc{};
                    tc.nt = 1;
                    tc.z[0] = rest[j].z;
                    tc.c[0] = rest[j].c;
                    tc.ylo[0] = rest[j].ylo;
                    leftover.push_back({rest[j].x, tc});
                    used[j] = true;
                    --left;
                    break;
                }
            continue;
        }
        uint64_t B = 0x3Full | Hm;
        for (int b = 6; b < n && __builtin_popcountll(B) < kTileQubits; ++b)
            B |= 1ull << b;
        passes.push_back({(uint32_t)B, take});
    }
    for (auto& pr : passes) {
        const uint64_t B = pr.first;
        std::vector<int> pos;
        for (int b = 0; b < 64; ++b)
            if ((B >> b) & 1)
                pos.push_back(b);
        auto compress = [&](uint64_t v) {
            uint32_t o = 0;
            for (size_t j = 0; j < pos.size(); ++j)
                if ((v >> pos[j]) & 1)
                    o |= 1u << j;
            return o;
        };
        int L = 0;
        while (L < (int)pos.size() && pos[L] == L)
            ++L;
        // diagonal classes (see TileExpK): 0 static straddler, 1 tile-signed
        // with a local mask, 2 wholly outside, 3 static table term
        std::vector<XTerm> dcls[4], pairs;
        for (const T& t : pr.second) {
            XTerm x{};
            x.z = t.z;
            x.c = t.c;
            x.zloc = compress(t.z);
            x.ylo = t.ylo;
            if (t.x == 0) {
                x.kind = 0;
                const bool lo = (x.zloc & 63) != 0, hi = (x.zloc >> 6) != 0;
                x.dpart = (lo && hi ? 3 : (hi ? 2 : 1));
                const bool inside = (t.z & ~B) == 0;
                const int cls = inside ? (x.dpart == 3 ? 0 : 3) : (x.zloc ? 1 : 2);
                dcls[cls].push_back(x);
            } else {
                x.xloc = compress(t.x);
                x.kind = (t.z == 0 && t.ylo == 0) ? 2 : 1;
                pairs.push_back(x);
            }
        }
        // launches of <= kMaxTileTerms terms: diagonal terms ride with the
        // first launch(es), pair terms fill the rest
        std::vector<XTerm> diag;
        std::vector<int> dclass;
        for (int cls = 0; cls < 4; ++cls)
            for (const XTerm& x : dcls[cls]) {
                diag.push_back(x);
                dclass.push_back(cls);
            }
        size_t di = 0, pi = 0;
        bool first = true;
        while (first || di < diag.size() || pi < pairs.size()) {
            first = false;
            TileExpK k{};
            k.ntiles = 1ull << (n - kTileQubits);
            k.ins = make_ins(pos, 0);
            k.L = L;
            const int nch = 1 << (kTileQubits - L);
            for (int c = 0; c < nch; ++c) {
                uint64_t o = 0;
                for (int m = 0; m < kTileQubits - L; ++m)
                    if ((c >> m) & 1)
                        o |= 1ull << pos[L + m];
                k.choff[c] = o;
            }
            int nt = 0;
            int cnt[4] = {0, 0, 0, 0};
            while (di < diag.size() && nt < kMaxTileTerms) {
                ++cnt[dclass[di]];
                k.t[nt++] = diag[di++];
            }
            k.nx = cnt[0];
            k.nd = k.nx + cnt[1];
            k.no = k.nd + cnt[2];
            k.pstart = nt;
            k.ndiag = nt;
            while (pi < pairs.size() && nt < kMaxTileTerms)
                k.t[nt++] = pairs[pi++];
            k.nt = nt;
            // pure X strings first (their loop needs no phase)
            std::stable_partition(k.t + k.pstart, k.t + k.nt, [](const XTerm& x) { return x.kind == 2; });
            k.pxend = k.pstart;
            while (k.pxend < k.nt && k.t[k.pxend].kind == 2)
                ++k.pxend;
            out.push_back(k);
        }
    }
}

// The passes of <psi|H|psi> for n >= kTileQubits, the cheapest of three
// plans:
//   R1  register-tile passes for the strings they take, LDS-tile passes for
//       the rest whose x masks fit a 12-qubit tile, span passes for the
//       others;
//   R2  register-tile passes, span passes for all the rest;
//   S   span passes for every string (five x masks with a qubit above 5 per
//       pass, strings on qubits 0..5 and diagonal strings spread over them).
// The cost of a pass is its time relative to a register pass of single X
// strings, measured at n = 30 (ExpPlan::cost).  QSV_EXPECT_PLAN=reg or
// =span restricts the choice to R1/R2 or S (comparisons); QSV_NO_SPAN_PASS=1
// leaves R1 with one pass per x mask for what no tile holds.
struct ExpPlan {
    std::vector<RegPassK> regs;
    std::vector<TileExpK> tiles;
    std::vector<SpanPassK> spans;
    std::vector<std::pair<uint64_t, TermChunk>> pairs;
    // complex64 passes are partly bound by their FP64 arithmetic, complex128
    // ones by the state read: register passes with transposed roles and
    // general strings 2.2 (1.45), with general strings 1.05 (1.02), with
    // transposed roles 1.1 (1.0); LDS-tile passes 1.7 (1.3); per-mask passes
    // 1.15; a span pass grows with its arithmetic L (direction strings 1,
    // lane strings 2.5, diagonal strings 0.1 plus 2 for their transform):
    // complex64 0.78 + 0.1 L ms against 1.3 ms, complex128 2.45 + 0.025 L
    // ms against 2.6 ms
    double cost(int dt) const
    {
        const bool c64 = dt == C64;
        double c = (c64 ? 1.7 : 1.3) * (double)tiles.size() + 1.15 * (double)pairs.size();
        for (const RegPassK& k : regs) {
            const bool tr = k.nt > k.n1, gen = k.n1 > k.ns1 || k.nc > k.ns2 || k.nt > k.nc;
            c += (tr && gen) ? (c64 ? 2.2 : 1.45) : gen ? (c64 ? 1.05 : 1.02) : tr ? (c64 ? 1.1 : 1.0) : 1.0;
        }
        for (const SpanPassK& k : spans) {
            const int ndir = k.koff[2 * kSpanDirs], nlane = k.koff[kSpanGroups] - ndir,
                      ndiag = k.nt - k.koff[kSpanGroups];
            const double L = ndir + 2.5 * nlane + 0.1 * ndiag + (ndiag ? 2.0 : 0.0);
            c += c64 ? std::max(0.97, (0.78 + 0.1 * L) / 1.3) : (2.45 + 0.025 * L) / 2.6;
        }
        return c;
    }
};

struct SubSum {  // the strings idx of H as a Pauli sum of their own
    std::vector<uint64_t> x, z;
    std::vector<double> c;
    SubSum() = default;
    SubSum(const qsv_pauli_sum* H, const std::vector<int>& idx)
    {
        for (int j : idx) {
            x.push_back(H->x_mask[j]);
            z.push_back(H->z_mask[j]);
            c.push_back(H->coeff[j]);
        }
    }
    qsv_pauli_sum sum() const { return qsv_pauli_sum{(int)x.size(), x.data(), z.data(), c.data()}; }
};

void plan_expectation(const qsv_pauli_sum* H, int n, int dt, ExpPlan& P)
{
    const char* nospan = std::getenv("QSV_NO_SPAN_PASS");
    const bool span = !(nospan && nospan[0] == '1');
    const char* force = std::getenv("QSV_EXPECT_PLAN");
    const bool want_r = span && force && std::strcmp(force, "reg") == 0;
    const bool want_s = span && force && std::strcmp(force, "span") == 0;
    std::vector<ExpPlan> plans;
    if (!want_s) {
        std::vector<int> rest;
        std::vector<RegPassK> regs;
        plan_reg_passes(H, n, regs, rest);
        const SubSum R(H, rest);
        const qsv_pauli_sum Hr = R.sum();
        ExpPlan A;  // R1
        A.regs = regs;
        if (!rest.empty()) {
            std::vector<std::pair<uint64_t, TermChunk>> leftover;
            plan_tiles(&Hr, n, A.tiles, leftover);
            if (!span || leftover.empty()) {
                A.pairs.swap(leftover);
            } else {
                SubSum L;
                for (const auto& pr : leftover)
                    for (int k = 0; k < pr.second.nt; ++k) {
                        L.x.push_back(pr.first);
                        L.z.push_back(pr.second.z[k]);
                        L.c.push_back(pr.second.c[k]);
                    }
                const qsv_pauli_sum Hl = L.sum();
                plan_span_passes(&Hl, n, A.spans);
            }
        }
        plans.push_back(A);
        if (span && !rest.empty()) {
            ExpPlan B;  // R2
            B.regs = regs;
            plan_span_passes(&Hr, n, B.spans);
            plans.push_back(B);
        }
    }
    if (span && !want_r) {
        ExpPlan S;
        plan_span_passes(H, n, S.spans);
        plans.push_back(S);
    }
    size_t best = 0;
    for (size_t i = 1; i < plans.size(); ++i)
        if (plans[i].cost(dt) < plans[best].cost(dt))
            best = i;
    P = plans[best];
}

qsv_status enqueue_expectation(const void* psi, int n, int dt, const qsv_pauli_sum* H, double* out,
                               double* work, int ncomp, hipStream_t s)
{
    int acc = 0;
    const int nb = reduce_blocks(n, dt);
    if (n >= kTileQubits) {
        ExpPlan P;
        plan_expectation(H, n, dt, P);
        for (const RegPassK& k : P.regs) {
            hipError_t e = launch_reg_pass(k, psi, dt, work, nb, acc, s);
            if (e != hipSuccess)
                return fail(QSV_ERR_HIP, "expectation launch: %s", hipGetErrorString(e));
            acc = 1;
        }
        for (const TileExpK& k : P.tiles) {
            hipError_t e = launch_tile_pass(k, psi, nullptr, dt, false, work, nb, acc, s);
            if (e != hipSuccess)
                return fail(QSV_ERR_HIP, "expectation launch: %s", hipGetErrorString(e));
            acc = 1;
        }
        for (const SpanPassK& k : P.spans) {
            hipError_t e = launch_span_pass(k, psi, dt, work, nb, acc, s);
            if (e != hipSuccess)
                return fail(QSV_ERR_HIP, "expectation launch: %s", hipGetErrorString(e));
            acc = 1;
        }
        for (const auto& pr : P.pairs) {
            hipError_t e = launch_expect_pair(psi, n, dt, pr.first, pr.second, work, acc, s);
            if (e != hipSuccess)
                return fail(QSV_ERR_HIP, "expectation launch: %s", hipGetErrorString(e));
            acc = 1;
        }
    } else {
        std::vector<TermChunk> diag;
        std::vector<std::pair<uint64_t, TermChunk>> pairs;
        group_terms(H, diag, pairs);
        for (const TermChunk& t : diag) {
            hipError_t e = launch_expect_diag(psi, n, dt, t, work, acc, s);
            if (e != hipSuccess)
                return fail(QSV_ERR_HIP, "expectation launch: %s", hipGetErrorString(e));
            acc = 1;
        }
        for (const auto& pr : pairs) {
            hipError_t e = launch_expect_pair(psi, n, dt, pr.first, pr.second, work, acc, s);
            if (e != hipSuccess)
                return fail(QSV_ERR_HIP, "expectation launch: %s", hipGetErrorString(e));
            acc = 1;
        }
    }
    hipError_t e = launch_finalize(work, nb, ncomp, out, s);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "finalize launch: %s", hipGetErrorString(e));
    return QSV_OK;
}

qsv_status enqueue_hpsi(const void* psi, void* lam, int n, int dt, const qsv_pauli_sum* H,
                        hipStream_t s)
{
    if (n >= kTileQubits) {
        std::vector<TileExpK> tiles;
        std::vector<std::pair<uint64_t, TermChunk>> leftover;
        plan_tiles(H, n, tiles, leftover);
        int acc = 0;
        for (const TileExpK& k : tiles) {
            hipError_t e = launch_tile_pass(k, psi, lam, dt, true, nullptr, 0, acc, s);
            if (e != hipSuccess)
                return fail(QSV_ERR_HIP, "H psi launch: %s", hipGetErrorString(e));
            acc = 1;
        }
        for (const auto& pr : leftover) {
            hipError_t e = launch_hpsi_pair(psi, lam, n, dt, pr.first, pr.second, s);
            if (e != hipSuccess)
                return fail(QSV_ERR_HIP, "H psi launch: %s", hipGetErrorString(e));
        }
        return QSV_OK;
    }
    std::vector<TermChunk> diag;
    std::vector<std::pair<uint64_t, TermChunk>> pairs;
    group_terms(H, diag, pairs);
    if (diag.empty())
        diag.push_back(TermChunk{});  // lam = 0 * psi
    int acc = 0;
    for (const TermChunk& t : diag) {
        hipError_t e = launch_hpsi_diag(psi, lam, n, dt, t, acc, s);
        if (e != hipSuccess)
            return fail(QSV_ERR_HIP, "H psi launch: %s", hipGetErrorString(e));
        acc = 1;
    }
    for (const auto& pr : pairs) {
        hipError_t e = launch_hpsi_pair(psi, lam, n, dt, pr.first, pr.second, s);
        if (e != hipSuccess)
            return fail(QSV_ERR_HIP, "H psi launch: %s", hipGetErrorString(e));
    }
    return QSV_OK;
}

}  // namespace qsv

// ============================================================== C ABI

extern "C" {

const char* qsv_last_error(void)
{
    return t_err.c_str();
}

const char* qsv_version(void)
{
    return "qsv 0.1 gfx950";
}

qsv_status qsv_state_bytes(int n, qsv_dtype dt, size_t* bytes)
{
    qsv_status st = check_n_dt(n, dt);
    if (st)
        return st;
    if (!bytes)
        return fail(QSV_ERR_ARG, "bytes is NULL");
    *bytes = amp_bytes(dt) << n;
    return ok();
}

qsv_status qsv_state_alloc(int n, qsv_dtype dt, void** psi)
{
    qsv_status st = check_n_dt(n, dt);
    if (st)
        return st;
    if (!psi)
        return fail(QSV_ERR_ARG, "psi is NULL");
    hipError_t e = hipMalloc(psi, amp_bytes(dt) << n);
    if (e != hipSuccess)
        return fail(QSV_ERR_NOMEM, "hipMalloc of %zu bytes: %s", amp_bytes(dt) << n,
                    hipGetErrorString(e));
    return ok();
}

qsv_status qsv_state_free(void* psi)
{
    if (!psi)
        return ok();
    hipError_t e = hipFree(psi);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "hipFree: %s", hipGetErrorString(e));
    return ok();
}

qsv_status qsv_init_basis(void* psi, int n, qsv_dtype dt, uint64_t index, void* stream)
{
    qsv_status st = check_state(psi, n, dt, "psi");
    if (st)
        return st;
    if (index >> n)
        return fail(QSV_ERR_ARG, "basis index %llu >= 2^%d", (unsigned long long)index, n);
    if ((st = enqueue_gate()))
        return st;
    hipError_t e = launch_init_basis(psi, n, dt, index, (hipStream_t)stream);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "init launch: %s", hipGetErrorString(e));
    return ok();
}

qsv_status qsv_reduce_workspace_bytes(size_t* bytes)
{
    if (!bytes)
        return fail(QSV_ERR_ARG, "bytes is NULL");
    *bytes = kReduceWorkBytes;
    return ok();
}

qsv_status qsv_init_random(void* psi, int n, qsv_dtype dt, uint64_t seed, void* work, void* stream)
{
    qsv_status st = check_state(psi, n, dt, "psi");
    if (st)
        return st;
    if (!work)
        return fail(QSV_ERR_ARG, "work is NULL");
    if ((st = enqueue_gate()))
        return st;
    hipError_t e = launch_init_random(psi, n, dt, seed, static_cast<double*>(work), (hipStream_t)stream);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "init launch: %s", hipGetErrorString(e));
    return ok();
}

qsv_status qsv_apply_gate(void* psi, int n, qsv_dtype dt, const int* targets, int k,
                          const int* controls, int c, const double* G, void* stream)
{
    qsv_status st = check_state(psi, n, dt, "psi");
    if (st)
        return st;
    if ((st = check_qubits(n, targets, k, QSV_MAX_TARGETS, controls, c)))
        return st;
    if (!G)
        return fail(QSV_ERR_ARG, "G is NULL");
    if (k + c > kMaxIns)
        return fail(QSV_ERR_UNSUPPORTED, "k + c = %d exceeds %d", k + c, kMaxIns);
    if ((st = enqueue_gate()))
        return st;
    int ct[QSV_MAX_TARGETS];
    std::vector<double> Gc;
    canonicalize(targets, k, G, ct, Gc);
    Built b = build_launch(n, dt, ct, k, controls, c, Gc.data(), true);
    if (b.noop)
        return ok();
    hipStream_t s = (hipStream_t)stream;
    if (!b.upload.empty()) {
        const void* d = nullptr;
        if ((st = stage_upload(b.upload.data(), b.upload.size(), s, &d)))
            return st;
        b.L.gdev = d;
    }
    if ((st = launch_checked(b.L, psi, nullptr, s)))
        return st;
    return ok();
}

qsv_status qsv_apply_fused(void* psi, int n, qsv_dtype dt, const qsv_block* blocks, int nblocks,
                           void* stream)
{
    qsv_status st = check_state(psi, n, dt, "psi");
    if (st)
        return st;
    if (nblocks < 0 || (nblocks > 0 && !blocks))
        return fail(QSV_ERR_ARG, "bad block list");
    for (int j = 0; j < nblocks; ++j) {
        if ((st = check_qubits(n, blocks[j].targets, blocks[j].k, QSV_MAX_TARGETS, nullptr, 0)))
            return st;
        if (!blocks[j].M)
            return fail(QSV_ERR_ARG, "block %d has a NULL matrix", j);
    }
    if ((st = enqueue_gate()))
        return st;
    hipStream_t s = (hipStream_t)stream;
    for (int j = 0; j < nblocks; ++j) {
        int ct[QSV_MAX_TARGETS];
        std::vector<double> Gc;
        canonicalize(blocks[j].targets, blocks[j].k, blocks[j].M, ct, Gc);
        Built b = build_launch(n, dt, ct, blocks[j].k, nullptr, 0, Gc.data(), true);
        if (b.noop)
            continue;
        if (!b.upload.empty()) {
            const void* d = nullptr;
            if ((st = stage_upload(b.upload.data(), b.upload.size(), s, &d)))
                return st;
            b.L.gdev = d;
        }
        if ((st = launch_checked(b.L, psi, nullptr, s)))
            return st;
    }
    return ok();
}

qsv_status qsv_norm2(const void* psi, int n, qsv_dtype dt, double* out_dev, void* work, void* stream)
{
    qsv_status st = check_state(psi, n, dt, "psi");
    if (st)
        return st;
    if (!out_dev || !work)
        return fail(QSV_ERR_ARG, "out_dev or work is NULL");
    if ((st = enqueue_gate()))
        return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_norm2(psi, n, dt, static_cast<double*>(work), 0, s);
    if (e == hipSuccess)
        e = launch_finalize(static_cast<double*>(work), reduce_blocks(n, dt), 1, out_dev, s);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "norm launch: %s", hipGetErrorString(e));
    return ok();
}

qsv_status qsv_expectation(const void* psi, int n, qsv_dtype dt, const qsv_pauli_sum* H,
                           double* out_dev, void* work, void* stream)
{
    qsv_status st = check_state(psi, n, dt, "psi");
    if (st)
        return st;
    if ((st = check_hamiltonian(H, n)))
        return st;
    if (!out_dev || !work)
        return fail(QSV_ERR_ARG, "out_dev or work is NULL");
    if ((st = enqueue_gate()))
        return st;
    if ((st = enqueue_expectation(psi, n, dt, H, out_dev, static_cast<double*>(work), 2,
                                  (hipStream_t)stream)))
        return st;
    return ok();
}

qsv_status qsv_expectation_launches(const qsv_pauli_sum* H, int n, qsv_dtype dt, int* nlaunches)
{
    qsv_status st = check_n_dt(n, dt);
    if (st)
        return st;
    if ((st = check_hamiltonian(H, n)))
        return st;
    if (!nlaunches)
        return fail(QSV_ERR_ARG, "nlaunches is NULL");
    int count = 1;  // the finalize
    if (n >= kTileQubits) {
        ExpPlan P;
        plan_expectation(H, n, dt, P);
        count += (int)(P.regs.size() + P.tiles.size() + P.spans.size() + P.pairs.size());
    } else {
        std::vector<TermChunk> diag;
        std::vector<std::pair<uint64_t, TermChunk>> pairs;
        group_terms(H, diag, pairs);
        count += (int)(diag.size() + pairs.size());
    }
    *nlaunches = count;
    return ok();
}

qsv_status qsv_expectation_noalloc(const void* psi, int n, qsv_dtype dt, const qsv_pauli_sum* H,
                                   double* out_dev, void* stream)
{
    qsv_status st = check_state(psi, n, dt, "psi");
    if (st)
        return st;
    if ((st = check_hamiltonian(H, n)))
        return st;
    if (!out_dev)
        return fail(QSV_ERR_ARG, "out_dev is NULL");
    // partial sums: re and im per reduction slot
    const size_t need = 2 * sizeof(double) * (size_t)reduce_blocks(n, dt);
    if (need > kStaticScratchBytes)
        return fail(QSV_ERR_UNSUPPORTED, "n = %d needs %zu bytes of partial sums, the static "
                    "scratch holds %zu", n, need, kStaticScratchBytes);
    if ((st = enqueue_gate()))
        return st;
    double* scr = nullptr;
    const hipError_t e = static_scratch(&scr);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "static scratch address: %s", hipGetErrorString(e));
    if ((st = enqueue_expectation(psi, n, dt, H, out_dev, scr, 2, (hipStream_t)stream)))
        return st;
    return ok();
}

qsv_status qsv_inner(const void* a, const void* b, int n, qsv_dtype dt, double* out_dev, void* work,
                     void* stream)
{
    qsv_status st = check_state(a, n, dt, "a");
    if (st)
        return st;
    if ((st = check_state(b, n, dt, "b")))
        return st;
    if (!out_dev || !work)
        return fail(QSV_ERR_ARG, "out_dev or work is NULL");
    if ((st = enqueue_gate()))
        return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_inner(a, b, n, dt, static_cast<double*>(work), 0, s);
    if (e == hipSuccess)
        e = launch_finalize(static_cast<double*>(work), reduce_blocks(n, dt), 2, out_dev, s);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "inner launch: %s", hipGetErrorString(e));
    return ok();
}

qsv_status qsv_apply_pauli_sum(const void* psi, void* out, int n, qsv_dtype dt,
                               const qsv_pauli_sum* H, void* stream)
{
    qsv_status st = check_state(psi, n, dt, "psi");
    if (st)
        return st;
    if ((st = check_state(out, n, dt, "out")))
        return st;
    if (psi == out)
        return fail(QSV_ERR_ARG, "psi and out must be distinct");
    if ((st = check_hamiltonian(H, n)))
        return st;
    if ((st = enqueue_gate()))
        return st;
    if ((st = enqueue_hpsi(psi, out, n, dt, H, (hipStream_t)stream)))
        return st;
    return ok();
}

}  // extern "C"

// ------------------------------------------------------------ measurement

qsv_status qsv_measure_workspace_bytes(int n, qsv_dtype dt, size_t* bytes)
{
    qsv_status st = check_n_dt(n, dt);
    if (st)
        return st;
    if (!bytes)
        return fail(QSV_ERR_ARG, "bytes is NULL");
    const size_t a = sample_workspace_doubles(n), b = marginal_workspace_doubles();
    *bytes = (a > b ? a : b) * sizeof(double);
    return ok();
}

qsv_status qsv_probabilities(const void* psi, int n, qsv_dtype dt, const int* qubits, int m,
                             double* out_dev, void* work, void* stream)
{
    qsv_status st = check_state(psi, n, dt, "psi");
    if (st)
        return st;
    if ((st = check_qubits(n, qubits, m, n, nullptr, 0)))
        return st;
    if (!out_dev || !work)
        return fail(QSV_ERR_ARG, "out_dev or work is NULL");
    if ((st = enqueue_gate()))
        return st;
    hipError_t e = launch_marginal(psi, n, dt, qubits, m, out_dev, static_cast<double*>(work),
                                   (hipStream_t)stream);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "probabilities launch: %s", hipGetErrorString(e));
    return ok();
}

qsv_status qsv_sample(const void* psi, int n, qsv_dtype dt, const double* u_dev, int64_t nshots,
                      int64_t* out_dev, void* work, void* stream)
{
    qsv_status st = check_state(psi, n, dt, "psi");
    if (st)
        return st;
    if (nshots < 0)
        return fail(QSV_ERR_ARG, "nshots = %lld is negative", (long long)nshots);
    if (nshots == 0)
        return ok();
    if (!u_dev || !out_dev || !work)
        return fail(QSV_ERR_ARG, "u_dev, out_dev or work is NULL");
    if ((st = enqueue_gate()))
        return st;
    hipError_t e = launch_sample(psi, n, dt, u_dev, 0, 0, nshots, out_dev, static_cast<double*>(work),
                                 (hipStream_t)stream);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "sample launch: %s", hipGetErrorString(e));
    return ok();
}

qsv_status qsv_frequencies(const int64_t* samples_dev, int64_t nshots, int n, const int* qubits, int m,
                           int64_t* counts_dev, void* stream)
{
    if (n < 1 || n > QSV_MAX_QUBITS)
        return fail(QSV_ERR_ARG, "n = %d outside [1, %d]", n, QSV_MAX_QUBITS);
    qsv_status st = check_qubits(n, qubits, m, n, nullptr, 0);
    if (st)
        return st;
    if (m > 30)
        return fail(QSV_ERR_UNSUPPORTED, "m = %d measured qubits: at most 30 (2^m counters)", m);
    if (nshots < 0)
        return fail(QSV_ERR_ARG, "nshots = %lld is negative", (long long)nshots);
    if (!counts_dev || (nshots > 0 && !samples_dev))
        return fail(QSV_ERR_ARG, "samples_dev or counts_dev is NULL");
    if ((st = enqueue_gate()))
        return st;
    hipError_t e = launch_frequencies(samples_dev, nshots, n, qubits, m, counts_dev, (hipStream_t)stream);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "frequencies launch: %s", hipGetErrorString(e));
    return ok();
}

qsv_status qsv_collapse(void* psi, int n, qsv_dtype dt, const int* qubits, int m, uint64_t outcome,
                        const double* prob_dev, void* stream)
{
    qsv_status st = check_state(psi, n, dt, "psi");
    if (st)
        return st;
    if ((st = check_qubits(n, qubits, m, n, nullptr, 0)))
        return st;
    if (m < 64 && outcome >> m)
        return fail(QSV_ERR_ARG, "outcome %llu needs more than m = %d bits", (unsigned long long)outcome, m);
    if (!prob_dev)
        return fail(QSV_ERR_ARG, "prob_dev is NULL");
    if ((st = enqueue_gate()))
        return st;
    hipError_t e = launch_collapse(psi, n, dt, qubits, m, outcome, prob_dev, (hipStream_t)stream);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "collapse launch: %s", hipGetErrorString(e));
    return ok();
}

qsv_status qsv_sample_seeded(const void* psi, int n, qsv_dtype dt, uint64_t seed, int64_t nshots,
                             int64_t* out_dev, void* work, void* stream)
{
    qsv_status st = check_state(psi, n, dt, "psi");
    if (st)
        return st;
    if (nshots < 0)
        return fail(QSV_ERR_ARG, "nshots = %lld is negative", (long long)nshots);
    if (nshots == 0)
        return ok();
    if (!out_dev || !work)
        return fail(QSV_ERR_ARG, "out_dev or work is NULL");
    if ((st = enqueue_gate()))
        return st;
    hipError_t e = launch_sample(psi, n, dt, nullptr, seed, 1, nshots, out_dev, static_cast<double*>(work),
                                 (hipStream_t)stream);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "sample launch: %s", hipGetErrorString(e));
    return ok();
}
