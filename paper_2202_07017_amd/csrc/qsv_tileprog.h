// Tile programs: circuits of single-target gates (<= 2 controls) compiled into
// cache-blocked passes for execution inside LDS tiles.
//
// A pass owns a set B of m qubits (the tile).  Its gates all act on tile
// qubits, so every 2^m-amplitude tile (fixed values of the other qubits) can
// be processed on its own: load it into LDS, run the pass, store it.  Inside
// a pass, consecutive gates whose qubits fit 3 qubits form a step: a thread
// holds the step's 8 amplitudes (per group of the other tile qubits) in
// registers and applies all of the step's gates before the next barrier.
//
// Shared by the host compiler (tileprog.cpp) and the kernels
// (kernels_batch.hip, kernels_tpass.hip).
#pragma once

#include <cstdint>
#include <vector>

namespace qsv {

constexpr int kMaxPassOps = 128;   // gates per pass, batched mode (staged in LDS)
constexpr int kMaxTpassOps = 512;  // gates per pass, single-state passes
constexpr int kMaxStepOps = 8;    // gates per step
constexpr int kStepQubits = 3;

struct DOp {         // a gate of a pass, step-local coordinates
    uint8_t kind;    // 0 fixed matrix, 5 / 6 / 7 = RX / RY / RZ from a parameter
    uint8_t tq;      // target: position inside the step's qubits (0..2)
    uint8_t cm;      // controls: mask over the step's qubits
    uint8_t pad;
    int32_t param;   // rotations: parameter index (instance-local for batches)
    int32_t mat;     // fixed gates: index of the 2x2 matrix (8 doubles)
    int32_t slot;    // rotations: pass-local slot (0..nrot-1); -1 otherwise
};

struct alignas(8) DStep {
    uint8_t nq;      // qubits of the step (always 3)
    uint8_t q[3];    // their tile-local positions, ascending
    int16_t o0, o1;  // gate range [o0, o1) inside the pass
};

struct DPass {
    uint64_t bmask;  // tile qubits
    int step_off, nsteps;
    int op_off, nops;
    int nrot;        // rotation slots in this pass
    int slot_base;   // first global slot of this pass (single-state adjoint)
    int shared;      // 1 if two rotations of this pass share a parameter
    int pad;
};

// Host-side gate before compilation (global qubit indices).
struct HGate {
    int kind;  // 0 fixed (mat), 5 / 6 / 7 rotation (param)
    int t, nc, c0, c1;
    int param;
    int mat;
};

struct TileProgram {
    std::vector<DPass> passes;
    std::vector<DStep> steps;
    std::vector<DOp> ops;
    std::vector<int> slot_param;  // global slot -> parameter (rotations, in pass order)
};

// Compile `gates` (circuit order) on n >= 3 qubits into passes of at most cap
// gates with tiles of m >= 3 qubits (m >= n: passes over the whole state).
// Every step spans exactly three qubits.  Rotations get consecutive global
// slots in forward pass order.
void compile_tile_program(const std::vector<HGate>& gates, int n, int m, int cap, TileProgram& out);

}  // namespace qsv
