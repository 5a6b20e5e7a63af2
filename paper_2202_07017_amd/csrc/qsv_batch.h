// Device tables of the batched persistent kernel (shared by the host planner
// in batch.cpp and the kernel in kernels_batch.hip).
#pragma once

#include "qsv_internal.h"

namespace qsv {

constexpr int kMaxPassOps = 128;  // gates staged per pass

struct BInst {
    int n;
    int npass;
    int pass_off;
    int nterm;
    int term_off;
    int nparam;
    long long param_off;  // into params / grads
    long long work_off;   // byte offset of (psi, lambda) in the workspace (n > m only)
};

struct BPass {
    uint32_t bmask;  // tile qubits (n <= m: all qubits)
    int nops;
    int op_off;
    int pad;
};

struct BPOp {
    uint8_t kind;  // 0 = fixed matrix (mat), 5 / 6 / 7 = RX / RY / RZ (param)
    uint8_t tloc;  // target, as a local (tile) bit position
    uint8_t nc;    // number of controls (0..2)
    uint8_t c0, c1;
    uint8_t pad[3];
    int32_t param;
    int32_t mat;
};

struct BTerm {
    uint64_t x, z;
    double c;
    int ylo;
    int pad;
};

struct BatchArgs {
    const BInst* inst;
    const int* order;
    int ninst;
    int m;
    const BPass* passes;
    const BPOp* pops;
    const double* mats;  // 8 doubles per fixed 2x2 matrix
    const BTerm* terms;
    const double* params;
    double* grads;
    double* energies;
    char* work;
    int* counter;
};

size_t batch_lds_bytes(int dt, int m);
int batch_resident_blocks(int dt, int m, int threads);
hipError_t launch_batch(const BatchArgs& a, int dt, int threads, int blocks, hipStream_t s);

}  // namespace qsv
