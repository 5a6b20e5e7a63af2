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
// permuted by the low bits of D(r)).  A string whose x mask lies on qubits
// 0..5 pairs (L, r) with (L ^ x, r) (a lane exchange), and a diagonal string
// needs no partner, so a pass also takes any number of those.
#pragma once

#include <cstdint>
#include <vector>

#include "qsv.h"

namespace qsv {

constexpr int kSpanDirs = 5;                       // directions: 32 registers per lane
constexpr int kSpanLaneQubits = 6;                 // lanes on qubits 0..5
constexpr int kSpanTileQubits = kSpanDirs + kSpanLaneQubits;
constexpr int kMaxSpanTerms = 64;                  // one string per lane
constexpr int kSpanGroups = 2 * kSpanDirs + 2;     // direction strings (Re, Im), lane strings (Re, Im)

// One string of a span pass, of one of three kinds:
//  * direction string (x mask = direction dir): its value per lane and tile
//    is s_t s_L c sum_i (-1)^(bit i of sgn) f_i, f_i = Re or Im (by `im`)
//    of conj(psi_b) psi_a over the 16 pairs of the direction, a = (L, r_i)
//    with r_i the i-th register index whose bit dir is clear, b = (L, r_i ^
//    2^dir); c holds the coefficient times 2 (each pair once) and the sign
//    of i^ylo (ylo = number of Y factors mod 4); bit i of sgn is the
//    register part of the z sign of a, parity(z & D(r_i));
//  * lane string (x mask xl on qubits 0..5): s_t s_L c sum_r (-1)^(bit r of
//    sgn) f_r with a = (L, r), b = (L ^ xl, r), c the coefficient with the
//    sign of i^ylo (every ordered pair once: no factor 2), bit r of sgn =
//    parity(z & D(r));
//  * diagonal string: s_t s_L c N(zr), N(m) = sum_r (-1)^popcount(m & r)
//    |psi_(L,r)|^2, zr bit j = parity(z & d_j).
// s_t = (-1)^(z . base) and s_L = (-1)^(z . L) are the tile and lane parts
// of the sign.
struct STerm {
    uint64_t z;
    double c;
    uint32_t sgn;
    int32_t dir;
    int32_t im;
    uint32_t xl;
    uint32_t zr;
};

struct SpanPassK {
    uint64_t ntiles;
    uint64_t low[kSpanTileQubits];  // insertion masks of qubits 0..5 and the pivots, ascending
    uint64_t d[kSpanDirs];          // directions
    int nt;
    // strings of group g at [koff[g], koff[g + 1]): g = 2 dir + im for the
    // direction strings, 2 kSpanDirs + im for the lane strings; the
    // diagonal strings follow at [koff[kSpanGroups], nt), sorted by zr,
    // those with zr = m at [mofs[m], mofs[m + 1])
    int koff[kSpanGroups + 1];
    int mofs[(1 << kSpanDirs) + 1];
    STerm t[kMaxSpanTerms];
};

// Span passes for the strings of H (n >= 12).  Every string is taken: x
// masks with a qubit at 6 or above become directions (five per pass, the
// parts above qubit 5 independent), the lane and diagonal strings are spread
// over the passes (one more pass if there is none).
void plan_span_passes(const qsv_pauli_sum* H, int n, std::vector<SpanPassK>& out);

}  // namespace qsv
