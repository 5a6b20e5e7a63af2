// Host side of the batched mode: validation, the cache-blocking pass
// scheduler, device tables, graph replay and the autotuner.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "qsv.h"
#include "qsv_batch.h"
#include "qsv_host.h"
#include "qsv_tileprog.h"

using namespace qsv;

namespace {

struct HInst {
    int n = 0;
    int nparam = 0;
    std::vector<HGate> ops;
    std::vector<BTerm> terms;
};

}  // namespace

struct qsv_batch_plan {
    int dt = 0;
    int ninst = 0;
    std::vector<HInst> inst;
    std::vector<double> mats;  // fixed 2x2 matrices, 8 doubles each
    std::vector<long long> param_off;
    std::vector<int> order;
    long long work_bytes = 0;
    std::vector<long long> work_off;
    // large instances (n >= split) run as single-instance adjoint plans, on
    // kLargeStreams side streams at once (each stream with its own workspace
    // region of big_bytes, starting at big_off)
    std::vector<qsv_adjoint_plan*> sub;  // per instance with n >= kSplitMin, else nullptr
    long long big_off = 0;
    long long big_bytes = 0;
    int split = 99;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev;  // fork, then one join per side stream
    ~qsv_batch_plan()
    {
        for (qsv_adjoint_plan* p : sub)
            if (p)
                qsv_adjoint_plan_destroy(p);
        for (hipEvent_t e : ev)
            if (e)
                hipEventDestroy(e);
        for (hipStream_t q : side)
            if (q)
                hipStreamDestroy(q);
    }
    // configuration
    int m = 0, threads = 0, blocks = 0;
    int cfg_m = -1;
    int nsmall = 0;
    DevPack dev;
    size_t o_inst = 0, o_order = 0, o_pass = 0, o_steps = 0, o_pops = 0, o_mats = 0, o_terms = 0;
    GraphCache graph;
    std::string key;
};

namespace {

constexpr int kWorkMinQubits = 11;  // instances with n >= this get a workspace region
constexpr int kSplitMin = 16;       // smallest size the large tier may take
// Side streams of the large tier: they run beside the persistent kernel and
// beside each other (the small large-tier instances leave most of the GPU
// idle on their own).
constexpr int kLargeStreams = 3;

qsv_status configure(qsv_batch_plan* P, int m, int threads, int split)
{
    if (P->cfg_m == m && P->threads == threads && P->split == split && P->dev.mem)
        return QSV_OK;
    P->split = split;
    std::vector<int> small;
    for (int i : P->order)
        if (P->inst[i].n < split || !P->sub[i])
            small.push_back(i);
    P->graph.reset();
    P->dev.reset();
    std::vector<BInst> bi(P->ninst);
    std::vector<DPass> passes;
    std::vector<DStep> steps;
    std::vector<DOp> dops;
    std::vector<BTerm> terms;
    for (int i = 0; i < P->ninst; ++i) {
        const HInst& I = P->inst[i];
        TileProgram tp;
        compile_tile_program(I.ops, I.n, m, kMaxPassOps, tp);
        BInst& b = bi[i];
        b.n = I.n;
        b.npass = (int)tp.passes.size();
        b.pass_off = (int)passes.size();
        b.nterm = (int)I.terms.size();
        b.term_off = (int)terms.size();
        b.nparam = I.nparam;
        b.param_off = P->param_off[i];
        b.work_off = P->work_off[i];
        for (DPass q : tp.passes) {
            q.step_off += (int)steps.size();
            q.op_off += (int)dops.size();
            passes.push_back(q);
        }
        steps.insert(steps.end(), tp.steps.begin(), tp.steps.end());
        dops.insert(dops.end(), tp.ops.begin(), tp.ops.end());
        terms.insert(terms.end(), I.terms.begin(), I.terms.end());
    }
    P->o_inst = P->dev.add(table_bytes(bi));
    P->o_order = P->dev.add(table_bytes(small));
    P->nsmall = (int)small.size();
    P->o_pass = P->dev.add(table_bytes(passes));
    P->o_steps = P->dev.add(table_bytes(steps));
    P->o_pops = P->dev.add(table_bytes(dops));
    P->o_mats = P->dev.add(table_bytes(P->mats, 8));
    P->o_terms = P->dev.add(table_bytes(terms));
    qsv_status st = P->dev.commit();
    if (st)
        return st;
    const int res = batch_resident_blocks(P->dt, m, threads);
    if (res <= 0)
        return fail(QSV_ERR_UNSUPPORTED, "batch kernel does not fit (m = %d, %d threads)", m, threads);
    P->blocks = std::max(1, std::min(res, P->nsmall));
    P->m = m;
    P->threads = threads;
    P->cfg_m = m;
    return QSV_OK;
}

BatchArgs batch_args(const qsv_batch_plan* P, const double* params, void* work, double* energies,
                     double* grads)
{
    BatchArgs a{};
    a.inst = static_cast<const BInst*>(P->dev.at(P->o_inst));
    a.order = static_cast<const int*>(P->dev.at(P->o_order));
    a.ninst = P->nsmall;
    a.m = P->m;
    a.apt = ((1 << P->m) / P->threads) >= 16 ? 16 : 8;
    a.passes = static_cast<const DPass*>(P->dev.at(P->o_pass));
    a.steps = static_cast<const DStep*>(P->dev.at(P->o_steps));
    a.ops = static_cast<const DOp*>(P->dev.at(P->o_pops));
    a.mats = static_cast<const double*>(P->dev.at(P->o_mats));
    a.terms = static_cast<const BTerm*>(P->dev.at(P->o_terms));
    a.params = params;
    a.grads = grads;
    a.energies = energies;
    a.work = static_cast<char*>(work);
    a.counter = static_cast<int*>(work);
    return a;
}

// The persistent kernel (instances below the split) on s.
qsv_status enqueue_small(qsv_batch_plan* P, const double* params, void* work, double* energies,
                         double* grads, hipStream_t s)
{
    if (P->nsmall == 0)
        return QSV_OK;
    hipError_t e = launch_batch(batch_args(P, params, work, energies, grads), P->dt, P->threads,
                                P->blocks, s);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "batch launch: %s", hipGetErrorString(e));
    return QSV_OK;
}

// Large tier: side streams forked from s (fork_large, before anything else
// of the call is enqueued on s) and joined back into s (join_large, also
// after an error: a capture needs it); instances assigned largest first to
// the least loaded stream, each stream with its own workspace region.
int large_streams(const qsv_batch_plan* P)
{
    int nl = 0;
    for (int i = 0; i < P->ninst; ++i)
        nl += (P->inst[i].n >= P->split && P->sub[i]) ? 1 : 0;
    return std::min((int)P->side.size(), nl);
}

qsv_status fork_large(qsv_batch_plan* P, int ns, hipStream_t s)
{
    if (ns == 0)
        return QSV_OK;
    hipError_t e = hipEventRecord(P->ev[0], s);
    for (int k = 0; k < ns && e == hipSuccess; ++k)
        e = hipStreamWaitEvent(P->side[k], P->ev[0], 0);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "large-tier fork: %s", hipGetErrorString(e));
    return QSV_OK;
}

qsv_status enqueue_large(qsv_batch_plan* P, int ns, const double* params, void* work,
                         double* energies, double* grads)
{
    std::vector<double> load(ns > 0 ? ns : 1, 0.0);
    for (int i : P->order) {
        if (P->inst[i].n < P->split || !P->sub[i])
            continue;
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[k] += std::ldexp((double)P->inst[i].ops.size() + 1, P->inst[i].n);
        qsv_status st = adjoint_enqueue_direct(P->sub[i], params + P->param_off[i],
                                               static_cast<char*>(work) + P->big_off + k * P->big_bytes,
                                               energies + i, grads + P->param_off[i], P->side[k]);
        if (st)
            return st;
    }
    return QSV_OK;
}

qsv_status join_large(qsv_batch_plan* P, int ns, hipStream_t s, qsv_status st)
{
    for (int k = 0; k < ns; ++k) {
        hipError_t j = hipEventRecord(P->ev[1 + k], P->side[k]);
        if (j == hipSuccess)
            j = hipStreamWaitEvent(s, P->ev[1 + k], 0);
        if (j != hipSuccess && !st)
            st = fail(QSV_ERR_HIP, "large-tier join: %s", hipGetErrorString(j));
    }
    return st;
}

// Everything, directly on s (the autotuner).  with_large = false leaves out
// the large tier (persistent-kernel shapes are timed on their own).
qsv_status enqueue(qsv_batch_plan* P, const double* params, void* work, double* energies,
                   double* grads, hipStream_t s, bool with_large = true)
{
    const int ns = with_large ? large_streams(P) : 0;
    qsv_status st = fork_large(P, ns, s);
    if (st)
        return st;
    st = enqueue_small(P, params, work, energies, grads, s);
    if (!st && ns > 0)
        st = enqueue_large(P, ns, params, work, energies, grads);
    return join_large(P, ns, s, st);
}

// (tile qubits, threads) with 8 or 16 amplitudes per thread in a tile step
std::vector<std::pair<int, int>> candidates(int dt)
{
    if (dt == QSV_C64)
        return {{12, 512}, {12, 256}, {11, 256}, {13, 512}};
    return {{11, 256}, {12, 512}, {10, 128}};
}

std::vector<int> split_candidates()
{
    return {17, 19, 21, 99};
}

bool read_cache(const std::string& key, int* m, int* threads, int* split)
{
    const char* path = getenv("QSV_TUNE_CACHE");
    if (!path)
        return false;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        // one entry per line:  "key": [m, threads, ms],
        const size_t q0 = line.find('"'), q1 = line.find('"', q0 + 1);
        if (q0 == std::string::npos || q1 == std::string::npos || line.substr(q0 + 1, q1 - q0 - 1) != key)
            continue;
        int a = 0, b = 0, c = 0;
        if (sscanf(line.c_str() + line.find('[', q1), "[%d, %d, %d", &a, &b, &c) == 3) {
            *m = a;
            *threads = b;
            *split = c;
            return true;
        }
    }
    return false;
}

void write_cache(const std::string& key, int m, int threads, int split, double ms)
{
    const char* path = getenv("QSV_TUNE_CACHE");
    if (!path)
        return;
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (std::getline(f, line))
            if (line.find('"') != std::string::npos && line.find("\"" + key + "\"") == std::string::npos)
                keep.push_back(line.back() == ',' ? line.substr(0, line.size() - 1) : line);
    }
    char buf[256];
    snprintf(buf, sizeof buf, "  \"%s\": [%d, %d, %d, %.3f]", key.c_str(), m, threads, split, ms);
    keep.push_back(buf);
    std::ofstream o(path);
    o << "{\n";
    for (size_t j = 0; j < keep.size(); ++j)
        o << keep[j] << (j + 1 < keep.size() ? ",\n" : "\n");
    o << "}\n";
}

}  // namespace

extern "C" {

qsv_status qsv_batch_plan_create(const qsv_circuit* circs, const qsv_pauli_sum* Hs, int ninst,
                                 qsv_dtype dt, qsv_batch_plan** plan, size_t* work_bytes)
{
    if (!circs || !Hs || ninst < 1 || !plan || !work_bytes)
        return fail(QSV_ERR_ARG, "NULL circuit list, Hamiltonian list, plan or size, or ninst < 1");
    qsv_status st = check_n_dt(1, dt);
    if (st)
        return st;
    std::unique_ptr<qsv_batch_plan> P(new qsv_batch_plan);
    P->dt = dt;
    P->ninst = ninst;
    P->inst.resize(ninst);
    P->param_off.resize(ninst + 1, 0);
    P->work_off.assign(ninst, 0);
    long long woff = 256;  // the queue counter lives at offset 0
    std::ostringstream sig;
    sig << "gfx950/" << (dt == QSV_C64 ? "c64" : "c128") << "/" << ninst;
    unsigned long long h = 1469598103934665603ull;
    for (int i = 0; i < ninst; ++i) {
        const qsv_circuit* C = &circs[i];
        if ((st = check_circuit(C, QSV_BATCH_MAX_QUBITS)))
            return fail(st, "instance %d: %s", i, qsv_last_error());
        if ((st = check_hamiltonian(&Hs[i], C->n)))
            return fail(st, "instance %d: %s", i, qsv_last_error());
        if (C->n < 3)
            return fail(QSV_ERR_UNSUPPORTED, "instance %d: batch instances need n >= 3", i);
        HInst& I = P->inst[i];
        I.n = C->n;
        I.nparam = C->nparams;
        for (int o = 0; o < C->nops; ++o) {
            const qsv_op& op = C->ops[o];
            if (op.k != 1 || op.c > 2 || op.kind == QSV_OP_SWAP)
                return fail(QSV_ERR_UNSUPPORTED,
                            "instance %d op %d: batches take single-target gates with <= 2 controls",
                            i, o);
            HGate x{};
            x.t = op.targets[0];
            x.nc = op.c;
            x.c0 = op.c > 0 ? op.controls[0] : 0;
            x.c1 = op.c > 1 ? op.controls[1] : 0;
            x.param = -1;
            x.mat = -1;
            if (op.kind == QSV_OP_RX || op.kind == QSV_OP_RY || op.kind == QSV_OP_RZ) {
                x.kind = op.kind;
                x.param = op.param;
            } else {
                x.kind = 0;
                x.mat = (int)(P->mats.size() / 8);
                std::vector<double> m = op_matrix(op, 0.0);
                P->mats.insert(P->mats.end(), m.begin(), m.end());
            }
            I.ops.push_back(x);
        }
        for (int t = 0; t < Hs[i].nterms; ++t) {
            BTerm b{};
            b.x = Hs[i].x_mask[t];
            b.z = Hs[i].z_mask[t];
            b.c = Hs[i].coeff[t];
            b.ylo = __builtin_popcountll(b.x & b.z) & 3;
            I.terms.push_back(b);
        }
        P->param_off[i + 1] = P->param_off[i] + C->nparams;
        if (I.n >= kWorkMinQubits) {
            P->work_off[i] = woff;
            woff += (long long)(2 * amp_bytes(dt)) << I.n;
            woff = (woff + 255) & ~255ll;
        }
        h = (h ^ (unsigned long long)(I.n * 1000003 + C->nops)) * 1099511628211ull;
    }
    sig << "/" << std::hex << h;
    P->key = sig.str();
    // the large tier: an adjoint plan per instance of >= kSplitMin qubits; up
    // to kLargeStreams of them run at once, each in a workspace region of its
    // stream
    P->sub.assign(ninst, nullptr);
    size_t big = 0;
    int nlarge = 0;
    for (int i = 0; i < ninst; ++i) {
        if (P->inst[i].n < kSplitMin)
            continue;
        size_t wb = 0;
        qsv_adjoint_plan* ap = nullptr;
        if ((st = qsv_adjoint_plan_create(&circs[i], &Hs[i], dt, 5, &ap, &wb)))
            return fail(st, "instance %d: %s", i, qsv_last_error());
        P->sub[i] = ap;
        big = std::max(big, wb);
        ++nlarge;
    }
    P->big_off = woff;
    P->big_bytes = (long long)((big + 255) & ~size_t(255));
    if (nlarge > 0) {
        const int ns = std::min(nlarge, kLargeStreams);
        woff += ns * P->big_bytes;
        P->side.assign(ns, nullptr);
        P->ev.assign(1 + ns, nullptr);
        for (hipStream_t& q : P->side)
            if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess)
                return fail(QSV_ERR_HIP, "large-tier stream creation failed");
        for (hipEvent_t& q : P->ev)
            if (hipEventCreateWithFlags(&q, hipEventDisableTiming) != hipSuccess)
                return fail(QSV_ERR_HIP, "large-tier event creation failed");
    }
    P->work_bytes = woff;
    // largest estimated work first
    P->order.resize(ninst);
    for (int i = 0; i < ninst; ++i)
        P->order[i] = i;
    std::stable_sort(P->order.begin(), P->order.end(), [&](int a, int b) {
        const double ca = std::ldexp((double)P->inst[a].ops.size() + 1, P->inst[a].n);
        const double cb = std::ldexp((double)P->inst[b].ops.size() + 1, P->inst[b].n);
        return ca > cb;
    });
    int m = dt == QSV_C64 ? 12 : 11, threads = 512, split = 19;
    read_cache(P->key, &m, &threads, &split);
    if (const char* e = getenv("QSV_BATCH_SHAPE")) {  // "m,threads[,split]" (tests of every shape)
        int a = 0, b = 0, c = split;
        if (sscanf(e, "%d,%d,%d", &a, &b, &c) >= 2 && a >= 3 && a <= 14 &&
            (b == 128 || b == 256 || b == 512) && ((1 << a) / b == 8 || (1 << a) / b == 16)) {
            m = a;
            threads = b;
            split = c;
        }
    }
    P->m = m;
    P->threads = threads;
    P->split = split;
    *work_bytes = (size_t)P->work_bytes;
    *plan = P.release();
    return ok();
}

qsv_status qsv_batch_offsets(const qsv_batch_plan* plan, int64_t* offsets)
{
    if (!plan || !offsets)
        return fail(QSV_ERR_ARG, "plan or offsets is NULL");
    for (int i = 0; i <= plan->ninst; ++i)
        offsets[i] = plan->param_off[i];
    return ok();
}

qsv_status qsv_batch_run(qsv_batch_plan* plan, const double* params_dev, void* work,
                         double* energies_dev, double* grads_dev, void* stream)
{
    if (!plan || !work || !energies_dev || (plan->param_off.back() > 0 && (!params_dev || !grads_dev)))
        return fail(QSV_ERR_ARG, "NULL plan, work, energies, gradients or parameters");
    if (reinterpret_cast<uintptr_t>(work) % 256)
        return fail(QSV_ERR_ARG, "work is not 256-byte aligned");
    qsv_status st = enqueue_gate();
    if (st)
        return st;
    st = configure(plan, plan->m, plan->threads, plan->split);
    if (st) {
        // the requested tile does not fit this device: take the first candidate that does
        for (auto c : candidates(plan->dt))
            if ((st = configure(plan, c.first, c.second, plan->split)) == QSV_OK)
                break;
        if (st)
            return st;
    }
    hipStream_t s = (hipStream_t)stream;
    // The persistent kernel replays through a graph; the large tier is
    // launched directly on the side streams: replaying independent branches
    // of one graph ran them one after another on this runtime (measured),
    // launched directly they overlap (2 streams: 338 -> 264 ms per batch of
    // the 1024-instance workload).
    const int ns = large_streams(plan);
    if ((st = fork_large(plan, ns, s)))
        return st;
    std::vector<const void*> key = {params_dev, work, energies_dev, grads_dev};
    st = run_graph(plan->graph, key, s, [&](hipStream_t cs) {
        return enqueue_small(plan, params_dev, work, energies_dev, grads_dev, cs);
    });
    if (!st && ns > 0)
        st = enqueue_large(plan, ns, params_dev, work, energies_dev, grads_dev);
    st = join_large(plan, ns, s, st);
    if (st)
        return st;
    return ok();
}

qsv_status qsv_batch_tune(qsv_batch_plan* plan, const double* params_dev, void* work,
                          double* energies_dev, double* grads_dev, void* stream, int* chosen)
{
    if (!plan || !work || !energies_dev)
        return fail(QSV_ERR_ARG, "NULL plan, work or energies");
    if (qsv_status gst = enqueue_gate())
        return gst;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(QSV_ERR_HIP, "event creation failed");
    // time one configuration: a warm-up run, then the mean of two (the
    // large tier left out while tile shapes are compared: it does not depend
    // on them, and its time would only add noise)
    auto measure = [&](int m, int t, int split, bool with_large, double* ms) -> bool {
        hipStreamSynchronize(s);
        if (configure(plan, m, t, split) != QSV_OK)
            return false;
        if (enqueue(plan, params_dev, work, energies_dev, grads_dev, s, with_large) != QSV_OK)
            return false;
        hipEventRecord(e0, s);
        for (int r = 0; r < 2; ++r)
            if (enqueue(plan, params_dev, work, energies_dev, grads_dev, s, with_large) != QSV_OK)
                return false;
        hipEventRecord(e1, s);
        hipEventSynchronize(e1);
        float f = 0.f;
        hipEventElapsedTime(&f, e0, e1);
        *ms = f / 2;
        return true;
    };
    double best = 1e300;
    int bm = plan->m, bt = plan->threads, bs = plan->split;
    // 1) tile shape at the current split (persistent kernel alone), 2) split
    // at the best shape (whole batch)
    for (auto c : candidates(plan->dt)) {
        double ms;
        if (measure(c.first, c.second, bs, false, &ms) && ms < best) {
            best = ms;
            bm = c.first;
            bt = c.second;
        }
    }
    best = 1e300;
    for (int sp : split_candidates()) {
        double ms;
        if (measure(bm, bt, sp, true, &ms) && ms < best) {
            best = ms;
            bs = sp;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipStreamSynchronize(s);
    qsv_status st = configure(plan, bm, bt, bs);
    if (st)
        return st;
    write_cache(plan->key, bm, bt, bs, best);
    if (chosen) {
        chosen[0] = bm;
        chosen[1] = bt;
        chosen[2] = bs;
    }
    return ok();
}

qsv_status qsv_batch_plan_destroy(qsv_batch_plan* plan)
{
    delete plan;
    return ok();
}

}  // extern "C"
