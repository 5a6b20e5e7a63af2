// Single-state cache-blocked passes (kernels_tpass.hip).
#pragma once

#include "qsv_internal.h"
#include "qsv_tileprog.h"

namespace qsv {

struct TPassArgs {
    DPass pass;
    const DStep* steps;  // whole program
    const DOp* ops;      // whole program
    const double* mats;
    const double* params;
    void* lops;          // staged descriptors: 2 * nops_total (forward, then reverse)
    double* partials;    // reverse passes: (slot) x (grid) FP64 sums
    int nops_total;
    int n;
    int m;               // tile qubits (<= n)
};

size_t tpass_lds_bytes(int dt, int m, bool rev);
int tpass_resident_blocks(int dt, int m, bool rev);
// Bytes of the staged descriptors of a program of nops gates.
size_t tpass_lop_bytes(int dt, int nops);
// Stage every gate of the program (a.ops, a.mats, a.params) into a.lops.
hipError_t launch_tstage(const TPassArgs& a, int dt, hipStream_t s);
hipError_t launch_tpass(const TPassArgs& a, int dt, bool rev, void* psi, void* lam, int blocks,
                        hipStream_t s);

}  // namespace qsv
