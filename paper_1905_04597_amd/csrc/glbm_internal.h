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

// Kernels of one (level_x, level_y, storage, bc_x, bc_y) variant.
struct Variant {
    Launch step = nullptr;
    Launch observe = nullptr;
    Launch init = nullptr;
    Launch stats = nullptr;
    LaunchEnds ends = nullptr;
    LaunchBatch batch = nullptr;
    bool split_rows = false;  // steps run as interior rows + wall rows (16-bit storage with walls)
};

// Registry of built variants, indexed by levels (0..kMaxLevel), storage, bc_x, bc_y.
Variant *variant_slot(int lx, int ly, int storage, int bcx, int bcy);

// Defined once per built level in glbm_inst.hip.
void register_level_1();
void register_level_2();
void register_level_3();
void register_level_4();
void register_level_5();
void register_level_6();
void register_level_7();
void register_mixed();
void register_compact_1();
void register_compact_2();
void register_compact_3();
void register_compact_4();
void register_compact_5();
void register_compact_6();
void register_compact_7();
void register_compact_mixed();

}  // namespace glbm
