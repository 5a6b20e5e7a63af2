// Device tables of the batched persistent kernel (shared by the host side in
// batch.cpp and the kernel in kernels_batch.hip).
#pragma once

#include "qsv_internal.h"
#include "qsv_tileprog.h"

namespace qsv {

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
    int apt;  // amplitudes per thread in a tile step: 2^m / threads (8 or 16)
    const DPass* passes;
    const DStep* steps;
    const DOp* ops;
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
