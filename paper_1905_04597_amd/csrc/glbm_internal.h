// Internal interface between the C-ABI (glbm_api.cpp) and the per-level
// kernel instantiations (glbm_inst.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "glbm_device.h"

namespace glbm {

using Launch = hipError_t (*)(const KArgs &, int grid, hipStream_t);
using LaunchEnds = hipError_t (*)(const KArgs &, int grid, float, float, hipStream_t);
// Batched step over a tile table for one row set (StepRows).
using LaunchBatch = hipError_t (*)(int rows, const BatchTile *tiles, int ntiles, int block, const KArgs *args,
                                   const int32_t *phase, const int64_t *t0, const int64_t *bstep, int launch,
                                   hipStream_t);

// Resident batched steps: one block per member, `steps` steps in one launch.
using LaunchResident = hipError_t (*)(const int32_t *members, int nmembers, const KArgs *args, const int32_t *phase,
                                      const int64_t *t0, const int64_t *bstep, int steps, hipStream_t);

// Kernels of one (level_x, level_y, storage, bc_x, bc_y) variant.
struct Variant {
    Launch step = nullptr;
    Launch observe = nullptr;
    Launch init = nullptr;
    Launch stats = nullptr;
    LaunchEnds ends = nullptr;
    LaunchBatch batch = nullptr;
    LaunchResident resident = nullptr;
    bool split_rows = false;  // steps run as interior rows + wall rows (16-bit storage with walls)
    bool wall_rates = false;  // the step reads per-column wall factors from a buffer of the solver
};

// Registry of built variants, indexed by axis codes (see Axis), storage, bc_x
// (with the row layout), bc_y; three-dimensional lattices in their own.
Variant *variant_slot(int ax, int ay, int storage, int bcx, int bcy);
Variant *variant3_slot(int ax, int ay, int az, int storage, int bcx, int bcy);
// three dimensions: one per object of glbm_inst3.hip
#define GLBM_OBJECTS3(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)
#define GLBM_DECLARE_REGISTER3(K) void register3_##K();
GLBM_OBJECTS3(GLBM_DECLARE_REGISTER3)

// One registration function per object file of glbm_inst.hip,
// register_E_K_L(): E = 1 for the lattices with G-D1Q(2N+2) axes; K = 0 for
// the one-dimensional lattices (padded rows), 1 for the two-dimensional ones
// (compact rows) with periodic y and for the mixed lattices, 2 for the
// symmetric two-dimensional ones with walls; L = level (0: the mixed
// lattices with a D1Q3 x axis up to level 7; 8..13: the mixed lattice with
// the even axis of that level).
#define GLBM_OBJECTS(X)                                                                                        \
    X(0, 0, 1) X(0, 0, 2) X(0, 0, 3) X(0, 0, 4) X(0, 0, 5) X(0, 0, 6) X(0, 0, 7)                               \
    X(0, 1, 0) X(0, 1, 1) X(0, 1, 2) X(0, 1, 3) X(0, 1, 4) X(0, 1, 5) X(0, 1, 6) X(0, 1, 7)                   \
    X(0, 2, 1) X(0, 2, 2) X(0, 2, 3) X(0, 2, 4) X(0, 2, 5) X(0, 2, 6) X(0, 2, 7)                               \
    X(1, 0, 1) X(1, 0, 2) X(1, 0, 3) X(1, 0, 4) X(1, 0, 5) X(1, 0, 6) X(1, 0, 7)                               \
    X(1, 1, 0) X(1, 1, 1) X(1, 1, 2) X(1, 1, 3) X(1, 1, 4) X(1, 1, 5) X(1, 1, 6) X(1, 1, 7)                   \
    X(1, 2, 1) X(1, 2, 2) X(1, 2, 3) X(1, 2, 4) X(1, 2, 5) X(1, 2, 6) X(1, 2, 7)                               \
    X(1, 1, 8) X(1, 1, 9) X(1, 1, 10) X(1, 1, 11) X(1, 1, 12) X(1, 1, 13)
#define GLBM_DECLARE_REGISTER(E, C, L) void register_##E##_##C##_##L();
GLBM_OBJECTS(GLBM_DECLARE_REGISTER)

}  // namespace glbm
