// Host-side helpers shared by the C-ABI translation units of libqsv.so.
#pragma once

#include <cstdlib>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "qsv.h"
#include "qsv_internal.h"

namespace qsv {

constexpr size_t kReduceWorkBytes = 32768;  // >= 2 x 1024 partials + scale slot

struct Built {
    GateLaunch L;
    std::vector<unsigned char> upload;  // device bytes the launch needs (gdev)
    bool noop = false;
};

qsv_status fail(qsv_status st, const char* fmt, ...);
qsv_status ok();
// Test hook of the launch error path: QSV_OK, or -- with QSV_TEST_FAIL_LAUNCH=1
// in the environment -- QSV_ERR_HIP with the message a failed launch gives.
// Every entry point calls it after validation and before its first enqueue.
qsv_status enqueue_gate();
size_t amp_bytes(int dt);
qsv_status check_n_dt(int n, int dt);
qsv_status check_state(const void* psi, int n, int dt, const char* what);
qsv_status check_qubits(int n, const int* t, int k, int kmax, const int* c, int nc);
qsv_status check_hamiltonian(const qsv_pauli_sum* H, int n);
InsertSpec make_ins(std::vector<int> pos, uint64_t setmask);
void canonicalize(const int* t, int k, const double* G, int* ct, std::vector<double>& Gc);
Built build_launch(int n, int dt, const int* ct, int k, const int* ctl, int c, const double* Gc,
                   bool allow_mfma);
GateLaunch rotation_launch(int n, int dt, int rot, int target, const int* ctl, int c, int pidx);
qsv_status stage_upload(const void* host, size_t bytes, hipStream_t s, const void** dev_out);
qsv_status launch_checked(const GateLaunch& L, void* psi, void* psi2, hipStream_t s);
void group_terms(const qsv_pauli_sum* H, std::vector<TermChunk>& diag,
                 std::vector<std::pair<uint64_t, TermChunk>>& pairs);
qsv_status enqueue_expectation(const void* psi, int n, int dt, const qsv_pauli_sum* H, double* out,
                               double* work, int ncomp, hipStream_t s);
qsv_status enqueue_hpsi(const void* psi, void* lam, int n, int dt, const qsv_pauli_sum* H,
                        hipStream_t s);
qsv_status check_circuit(const qsv_circuit* C, int max_n);
// Enqueue a full adjoint evaluation of a plan directly on `s` (no graph).
qsv_status adjoint_enqueue_direct(qsv_adjoint_plan* P, const double* params, void* work,
                                  double* energy, double* grad, hipStream_t s);
size_t adjoint_work_bytes(const qsv_adjoint_plan* P);
std::vector<double> op_matrix(const qsv_op& op, double theta);

// --------------------------------------------------------- graph caching

struct GraphCache {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const void*> key;
    ~GraphCache() { reset(); }
    void reset()
    {
        if (exec)
            hipGraphExecDestroy(exec);
        if (graph)
            hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        key.clear();
    }
};

inline bool graphs_enabled()
{
    const char* e = getenv("QSV_NO_GRAPH");
    return !(e && e[0] == '1');
}

// Run `enqueue` directly, or through a cached graph keyed by `key`.
template <typename F>
qsv_status run_graph(GraphCache& gc, const std::vector<const void*>& key, hipStream_t s,
                            F enqueue)
{
    if (!graphs_enabled())
        return enqueue(s);
    if (!gc.exec || gc.key != key) {
        gc.reset();
        hipStream_t cs;
        hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess)
            return fail(QSV_ERR_HIP, "capture stream: %s", hipGetErrorString(e));
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            hipStreamDestroy(cs);
            return fail(QSV_ERR_HIP, "begin capture: %s", hipGetErrorString(e));
        }
        qsv_status st = enqueue(cs);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        hipStreamDestroy(cs);
        if (st) {
            if (g)
                hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess)
            return fail(QSV_ERR_HIP, "end capture: %s", hipGetErrorString(e));
        gc.graph = g;
        e = hipGraphInstantiate(&gc.exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            gc.reset();
            return fail(QSV_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
        }
        gc.key = key;
    }
    hipError_t e = hipGraphLaunch(gc.exec, s);
    if (e != hipSuccess)
        return fail(QSV_ERR_HIP, "graph launch: %s", hipGetErrorString(e));
    return QSV_OK;
}

// Bytes of a host table for upload, at least min_elems elements (zero-filled
// beyond the table, so empty tables still give a valid device pointer).
template <typename T>
std::vector<unsigned char> table_bytes(const std::vector<T>& v, size_t min_elems = 1)
{
    std::vector<unsigned char> out((v.size() > min_elems ? v.size() : min_elems) * sizeof(T), 0);
    if (!v.empty())
        std::memcpy(out.data(), v.data(), v.size() * sizeof(T));
    return out;
}

// Device memory owned by a plan: all uploads packed at 256-byte offsets.
struct DevPack {
    void* mem = nullptr;
    size_t bytes = 0;
    std::vector<std::pair<size_t, std::vector<unsigned char>>> pending;
    size_t add(std::vector<unsigned char> data)
    {
        const size_t off = (bytes + 255) & ~size_t(255);
        bytes = off + data.size();
        pending.push_back({off, std::move(data)});
        return off;
    }
    qsv_status commit()
    {
        if (bytes == 0)
            return QSV_OK;
        if (hipMalloc(&mem, bytes) != hipSuccess)
            return fail(QSV_ERR_NOMEM, "plan device allocation of %zu bytes failed", bytes);
        std::vector<unsigned char> host(bytes, 0);
        for (auto& p : pending)
            std::memcpy(host.data() + p.first, p.second.data(), p.second.size());
        hipError_t e = hipMemcpy(mem, host.data(), bytes, hipMemcpyHostToDevice);
        pending.clear();
        if (e != hipSuccess)
            return fail(QSV_ERR_HIP, "plan upload: %s", hipGetErrorString(e));
        return QSV_OK;
    }
    const void* at(size_t off) const { return static_cast<const char*>(mem) + off; }
    void reset()
    {
        if (mem)
            hipFree(mem);
        mem = nullptr;
        bytes = 0;
        pending.clear();
    }
    ~DevPack() { reset(); }
};

}  // namespace qsv
