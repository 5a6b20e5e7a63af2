// Single-state cache-blocked passes (kernels_tpass.hip).
#pragma once

#include "qsv_internal.h"
#include "qsv_tileprog.h"

namespace qsv {

constexpr int kTpassThreads = 512;

struct TPassArgs {
    DPass pass;
    const DStep* steps;
    const DOp* ops;
    const double* mats;
    const double* params;
    double* partials;  // reverse passes: (slot) x (grid) FP64 sums
    int n;
    int m;             // tile qubits (<= n)
};

size_t tpass_lds_bytes(int dt, int m, bool rev);
int tpass_resident_blocks(int dt, int m, bool rev);
hipError_t launch_tpass(const TPassArgs& a, int dt, bool rev, void* psi, void* lam, int blocks,
                        hipStream_t s);

}  // namespace qsv
