// Host-side helpers shared by the C-ABI translation units of libqsv.so.
#pragma once

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

}  // namespace qsv
