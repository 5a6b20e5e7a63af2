// Tiled Pauli-sum passes (kernels_expect.hip) and their host planner.
#pragma once

#include "qsv_internal.h"

namespace qsv {

constexpr int kTileQubits = 12;
constexpr int kMaxTileTerms = 48;

// One Pauli term inside a tile pass.  kind: 0 diagonal, 1 general pair term,
// 2 pure X string (z = 0, no Y).  dpart (diagonal terms): 1 = local mask in
// the low 6 tile bits, 2 = in the high 6, 3 = straddles both.
struct XTerm {
    uint64_t z;
    double c;
    uint32_t zloc;  // z restricted to the tile, compressed to local bits
    uint32_t xloc;  // x compressed to local bits (x lies inside the tile)
    int32_t kind;
    int32_t dpart;
    int32_t ylo;    // number of Y factors mod 4 (32-bit fields: scalar loads)
};

struct TileExpK {
    uint64_t ntiles;
    InsertSpec ins;  // tile qubits, ascending (zeros inserted into the tile index)
    int L;           // contiguous low run of tile qubits
    int nt;          // terms [0, nstr): straddling diagonal; [nstr, pstart): table diagonal;
    int nstr;        //       [pstart, pxend): pure X strings; [pxend, nt): other pair terms
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
