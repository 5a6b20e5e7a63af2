// Tiled Pauli-sum passes (kernels_expect.hip) and their host planner.
#pragma once

#include "qsv_internal.h"

namespace qsv {

constexpr int kTileQubits = 12;
constexpr int kMaxTileTerms = 48;

// One Pauli term inside a tile pass.  kind: 0 diagonal, 1 general pair term,
// 2 pure X string (z = 0, no Y).  dpart (diagonal terms): 1 = local mask in
// the low 6 tile bits (or none), 2 = in the high 6, 3 = straddles both.
struct XTerm {
    uint64_t z;
    double c;
    uint32_t zloc;  // z restricted to the tile, compressed to local bits
    uint32_t xloc;  // x compressed to local bits (x lies inside the tile)
    int32_t kind;
    int32_t dpart;
    int32_t ylo;    // number of Y factors mod 4
};

// Terms of a pass, in this order:
//   [0, nx)        diagonal, z inside the tile, local mask in both table halves
//   [nx, nd)       diagonal, z partly outside the tile, local mask not empty
//   [nd, no)       diagonal, z wholly outside the tile (a constant per tile)
//   [no, pstart)   diagonal, z inside the tile, local mask in one table half
//   [pstart, pxend) pure X strings;  [pxend, nt) other pair terms.
// Terms whose sign depends on the tile ([nx, no) and the pair terms) get it
// once per tile; the others are folded into per-block tables.
struct TileExpK {
    uint64_t ntiles;
    InsertSpec ins;  // the kTileQubits tile qubits, ascending (zeros inserted into the tile index)
    int L;           // contiguous low run of tile qubits
    int nt;
    int nx;
    int nd;
    int no;
    int pstart;
    int pxend;
    int ndiag;       // number of diagonal terms (0: no diagonal part in this pass)
    uint64_t choff[64];
    XTerm t[kMaxTileTerms];
};

// hpsi: lam (+)= the pass's part of H psi.  Otherwise the block partials of
// <psi|H_pass|psi> go to partials[b] (real) and partials[nslots + b] (imaginary),
// b < nslots, added to the slots' contents when accumulate is set.
hipError_t launch_tile_pass(const TileExpK& a, const void* psi, void* lam, int dt, bool hpsi,
                            double* partials, int nslots, int accumulate, hipStream_t s);

}  // namespace qsv
