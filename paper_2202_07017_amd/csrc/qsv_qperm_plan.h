// Host planner of qubit permutation passes (kernels_qperm.hip): a sequence
// of SWAP gates (Sec. 3 gate set) permutes the bits of every amplitude index;
// the composed bit permutation is applied in one in-place pass when it is an
// involution and in two otherwise (every permutation is a product of two
// involutions).  Pure host code, no HIP types, so that a CPU checker can
// build it alone.
#pragma once

#include <cstdint>
#include <utility>
#include <vector>

namespace qsv {

constexpr int kQpMaxQubits = 64;
constexpr int kQpMaxRowBits = 6;

// One pass: output amplitude j takes input amplitude i with bit b of i equal
// to bit q[b] of j, where q is an involution (q[q[b]] == b), so that i and j
// are images of each other.  A tile is the set of indices that agree outside
// the tile bits T: T[k] = k for k < rl (rows of 2^rl consecutive amplitudes)
// and T[rl + k] = hpos[k] (ascending) for k < hb.  T is closed under q and
// holds q(0..rl-1), so a tile maps onto one tile; cmap[k] is the tile-local
// bit of the output that lands on tile-local bit k of the source
// (the position of q[T[k]] in T).
struct QPermPass {
    int n = 0;
    int rl = 0;
    int hb = 0;
    int hpos[kQpMaxRowBits] = {};
    int cmap[2 * kQpMaxRowBits] = {};
    int q[kQpMaxQubits] = {};
    uint64_t ntiles = 0;  // 2^(n - rl - hb)
    // tile order: bit p of the compact tile index is bit wsrc[p] of the
    // workgroup index (p < n - rl - hb), chosen so that consecutive
    // workgroups step through adjacent rows of both a tile and its image
    int wsrc[kQpMaxQubits] = {};
};

// Bit map of a swap sequence applied in order: the result takes its
// amplitude j from input amplitude i with bit b of i = bit Q[b] of j.
std::vector<int> compose_swaps(const std::vector<std::pair<int, int>>& swaps, int n);

// Passes (applied in order) whose product is the bit map Q; none when Q is
// the identity.  Requires n >= 2 rl and 1 <= rl <= kQpMaxRowBits.
void plan_qubit_permutation(const std::vector<int>& Q, int n, int rl, std::vector<QPermPass>& out);

}  // namespace qsv
