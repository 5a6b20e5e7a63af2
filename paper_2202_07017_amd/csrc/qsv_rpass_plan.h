// Register-tile Pauli passes for expectation values: the pass descriptors
// and their host planner (rpass_plan.cpp).  Plain C++ (no HIP): the kernels
// (kernels_rpass.hip) and a CPU checker of the planner both include it.
#pragma once

#include <cstdint>
#include <vector>

#include "qsv.h"

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
//
// Diagonal terms carry their coefficient in c.  A string with an x mask
// contributes, per lane and tile, sign * (c * s0 + c2 * s1), where s0 and s1
// are the lane's two half sums of 2 Re or 2 Im of its pair products (halves
// by the lower x bit, or alternating pairs for a single x bit); c and c2
// hold the factor 2, the sign of i^ylo and the register part of the z sign,
// and several strings with the same x mask, kind and lane/outside z parts
// are merged into one term by adding their (c, c2).
struct RTerm {
    uint64_t z;      // z mask (only its bits outside the tile matter: the tile's sign)
    double c;
    double c2;
    uint32_t xr;     // 0 for diagonal terms
    uint32_t zr;
    uint32_t zl;
    int32_t ylo;     // number of Y factors mod 4 (its parity picks Re or Im)
    uint32_t xl;     // cross-lane strings: lane xor mask of the partner (else 0)
};

// One pass: a wave loads a tile -- lanes on the lane qubits (lane bits 0..4
// on qubits 0..4, so every load is a run of >= 32 consecutive amplitudes),
// registers on the register qubits -- and evaluates
//   [0, nd)     diagonal terms,
//   [nd, ns1)   single-qubit X strings (no Z or Y factors) on a register qubit,
//   [ns1, n1)   other strings whose x mask is one or two register qubits,
//   [n1, ns2)   single-qubit X strings on one of qubits 0..4,
//   [ns2, nc)   other strings whose x mask is one or two of qubits 0..4, and
//   [nc, nt)    strings whose x mask is qubit 4 and one qubit that is a lane
//               qubit of the transposed roles (the pair (4, 5) of a chain):
//               the partner sits in register r ^ 16 of lane ^ xl,
// the last three after an LDS transpose that swaps the roles of lane bits
// 0..4 and the register bits.
struct RegPassK {
    uint64_t ntiles;
    uint64_t low[kRegTileQubits];   // insertion masks of the tile qubits, ascending
    uint64_t qstride[kRegQubits];   // 2^q of register qubit k
    int lanepos[kRegLanes];         // qubit of lane bit b (lanepos[b] = b for b < 5)
    int nd;
    int ns1;
    int n1;
    int ns2;
    int nc;
    int nt;
    int mofs[(1 << kRegQubits) + 1];  // diagonal terms sorted by zr: terms [mofs[m], mofs[m+1]) have zr = m
    RTerm t[kMaxRegTerms];
};

// Register passes for the strings of H they can take (n >= 12; see the
// order of terms in RegPassK).  Every other term index goes to `rest`.
void plan_reg_passes(const qsv_pauli_sum* H, int n, std::vector<RegPassK>& out, std::vector<int>& rest);

}  // namespace qsv
