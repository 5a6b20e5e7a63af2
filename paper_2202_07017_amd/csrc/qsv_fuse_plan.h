// Gate fusion planner (host code): groups the gates of a circuit into blocks
// of at most fuse_k qubits, each applied as one dense launch (Sec. 2, eq. (1)
// for k-qubit blocks).  Pure host code with no HIP types, so that a CPU
// checker can build it alone.
#pragma once

#include <vector>

#include "qsv.h"

namespace qsv {

inline bool is_rotation(int kind)
{
    return kind == QSV_OP_RX || kind == QSV_OP_RY || kind == QSV_OP_RZ;
}

struct Item {
    bool rotation = false;     // standalone unbound rotation
    std::vector<int> ops;      // ops of the block (one op: emitted natively)
    std::vector<int> qs;       // block qubits (ascending)
};

// Greedy DAG-aware fusion: each qubit is owned by at most one open block; a
// gate joins (and merges) the open blocks owning its qubits when the union
// has <= fuse_k qubits, otherwise those blocks are emitted.  Open blocks have
// disjoint qubits, so their relative order is free.
//
// With defer_diagonal (plans ask for it with fuse_k >= 3), a diagonal gate
// that does not fit the blocks owning its qubits leaves them open and waits
// in a pool instead: diagonal gates commute with each other and with gates
// on other qubits, so the pool only has to be applied before the next
// non-diagonal gate (or standalone rotation) on one of its qubits, and after
// the blocks that hold earlier gates on them.  That gate flushes the pool:
// first the blocks owning pooled qubits, then the pooled gates packed (first
// fit) into diagonal blocks of <= fuse_k qubits.  A QFT then keeps its
// Hadamards and the phases among them in blocks of fuse_k qubits, and the
// phases between blocks become a few diagonal blocks each.
//
// Items come out in application order; applying the ops of an item in
// their listed order is equivalent to applying them in circuit order (ops of
// merged blocks act on disjoint qubits).  Each op appears in exactly one item.
std::vector<Item> fuse_ops(const qsv_circuit* C, int fuse_k, bool rotations_standalone,
                           bool defer_diagonal = false);

}  // namespace qsv
