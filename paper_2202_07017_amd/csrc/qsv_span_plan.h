// Span passes for expectation values: Pauli strings with arbitrary x masks,
// several x masks per state read.  Pass descriptors and their host planner
// (span_plan.cpp).  Plain C++ (no HIP): the kernels (kernels_span.hip) and a
// CPU checker of the planner both include it.
//
// A pass picks up to kSpanDirs x masks d_0..d_4 (the directions) whose parts
// on qubits 6 and above are linearly independent over GF(2), and kSpanDirs
// pivot qubits P (>= 6) on which the directions form an invertible matrix.
// Every index then splits uniquely as
//   i = base ^ L ^ D(r),   D(r) = XOR of d_j over the set bits j of r,
// with base zero on qubits 0..5 and on P (one tile per base), L < 64 (the
// lane) and r < 32 (the register).  A string whose x mask is direction j
// pairs (L, r) with (L, r ^ 2^j): both amplitudes sit in one lane, and every
// load instruction reads 64 amplitudes of one aligned run (lane order
// permuted by the low bits of D(r)).
#pragma once

#include <cstdint>
#include <vector>

#include "qsv.h"

namespace qsv {

constexpr int kSpanDirs = 5;                       // directions: 32 registers per lane
constexpr int kSpanLaneQubits = 6;                 // lanes on qubits 0..5
constexpr int kSpanTileQubits = kSpanDirs + kSpanLaneQubits;
constexpr int kMaxSpanTerms = 32;

// One string of a span pass.  Its value per lane and tile is
//   (-1)^(z . (base ^ L)) c * sum_i (-1)^(bit i of sgn) f_i,
// f_i = Re or Im (by `im`) of conj(psi_b) psi_a over the 16 pairs of its
// direction, a = (L, r_i) with r_i the i-th register index whose bit `dir`
// is clear and b = (L, r_i ^ 2^dir).  c holds the coefficient times 2 and
// the sign of i^ylo (ylo = number of Y factors mod 4); bit i of sgn is the
// register part of the z sign of a, parity(z & D(r_i)).
struct STerm {
    uint64_t z;
    double c;
    uint32_t sgn;
    int32_t dir;
    int32_t im;
};

struct SpanPassK {
    uint64_t ntiles;
    uint64_t low[kSpanTileQubits];  // insertion masks of qubits 0..5 and the pivots, ascending
    uint64_t d[kSpanDirs];          // directions
    int nt;
    int koff[2 * kSpanDirs + 1];    // strings of direction j, Re (g = 2j) or Im (g = 2j + 1): [koff[g], koff[g + 1])
    STerm t[kMaxSpanTerms];
};

// Span passes for the strings of H (n >= 12); strings whose x mask has no
// qubit at 6 or above go to `rest`.
void plan_span_passes(const qsv_pauli_sum* H, int n, std::vector<SpanPassK>& out, std::vector<int>& rest);

}  // namespace qsv
