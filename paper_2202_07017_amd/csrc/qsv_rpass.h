// Register-tile Pauli passes for expectation values (kernels_rpass.hip) and
// their host planner (api.cpp).
#pragma once

#include "qsv_internal.h"

namespace qsv {

constexpr int kRegQubits = 5;                          // register qubits: 32 amplitudes per lane
constexpr int kRegLanes = 6;                           // lane qubits
constexpr int kRegTileQubits = kRegQubits + kRegLanes; // one wave holds a tile of 2^11 amplitudes
constexpr int kMaxRegTerms = 48;

// One Pauli term of a register pass.  Masks are compressed onto the tile
// qubits of the phase that evaluates the term: xr, zr onto the register
// qubits (bit k = register qubit k), zl onto the lane qubits (bit b = lane
// qubit b).  Terms evaluated after the transpose use the transposed roles
// (registers = qubits 0..4; lane bit 0 = lane qubit 5 of the pass, lane bits
// 1..5 = its register qubits).
struct RTerm {
    uint64_t z;      // full z mask: its parity with the tile base gives the tile's sign
    double c;
    uint32_t xr;     // 0 for diagonal terms
    uint32_t zr;
    uint32_t zl;
    int32_t ylo;     // number of Y factors mod 4
};

// One pass: a wave loads a tile -- lanes on the lane qubits (lane bits 0..4
// on qubits 0..4, so every load is a run of >= 32 consecutive amplitudes),
// registers on the register qubits -- and evaluates
//   [0, nd)   diagonal terms,
//   [nd, n1)  terms whose x mask lies on the register qubits,
//   [n1, nt)  terms whose x mask lies on qubits 0..4, after an LDS transpose
//             that swaps the roles of lane bits 0..4 and the register bits.
struct RegPassK {
    uint64_t ntiles;
    uint64_t low[kRegTileQubits];   // insertion masks of the tile qubits, ascending
    uint64_t qstride[kRegQubits];   // 2^q of register qubit k
    int lanepos[kRegLanes];         // qubit of lane bit b (lanepos[b] = b for b < 5)
    int nd;
    int n1;
    int nt;
    int mofs[(1 << kRegQubits) + 1];  // diagonal terms sorted by zr: terms [mofs[m], mofs[m+1]) have zr = m
    RTerm t[kMaxRegTerms];
};

// Adds the pass's part of <psi|H|psi> to partials[b] (b < nslots, one slot
// per block; the imaginary slots partials[nslots + b] get 0: every Hermitian
// pair is summed once, so the imaginary part vanishes identically), or writes
// it when accumulate is 0 (then slots beyond the grid are zeroed too).
hipError_t launch_reg_pass(const RegPassK& a, const void* psi, int dt, double* partials, int nslots,
                           int accumulate, hipStream_t s);

}  // namespace qsv
