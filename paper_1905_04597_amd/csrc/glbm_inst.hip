// Kernel instantiations for one hierarchy level, selected at compile time
// with -DGLBM_LEVEL=N (N = 1..7); -DGLBM_LEVEL=0 builds the mixed lattices
// up to level 7, -DGLBM_LEVEL=8..13 the mixed lattice with the even axis of
// that level.
// -DGLBM_EVEN=1 builds the lattices of G-D1Q(2N+2) axes instead of
// G-D1Q(2N+1) ones.  -DGLBM_COMPACT=0 builds the one-dimensional lattices
// (padded rows), -DGLBM_COMPACT=1 the two-dimensional ones (periodic x in
// compact rows), with -DGLBM_WALLS=1 those with walls across y.  Each (axis kind, dimension, level) is its own object file
// so the build runs in parallel.
#include "glbm_internal.h"

namespace glbm {
namespace {

template <int LX, int LY, int ST, int BCX, int BCY>
struct Launchers {
    static hipError_t step(const KArgs &a, int grid, hipStream_t s)
    {
        if constexpr (BCY == BCY_WALL && wall_prepass<LX, LY, ST>()) {
            // the wall factors of every column first (the wall rows read them)
            if (!a.wrate) return hipErrorInvalidValue;
            hipLaunchKernelGGL((wall_rate_kernel<LX, LY, ST, BCX>), dim3((a.nx + kBlock / 2 - 1) / (kBlock / 2)),
                               dim3(kBlock), 0, s, a);
        }
        if constexpr (BCY == BCY_PERIODIC && BCX == BCX_WRAP && split_node<LX, LY, ST>()) {
            // more than 144 velocities: each node split over a wave pair
            const int nodes = a.nx * a.ny;
            hipLaunchKernelGGL((step_kernel_split<LX, LY, ST, BCX, BCY>),
                               dim3((nodes + kSplitNodes - 1) / kSplitNodes), dim3(kBlock), 0, s, a);
        } else if constexpr (BCY == BCY_WALL && BCX == BCX_WRAP && split_node<LX, LY, ST>()) {
            // more than 144 velocities: the interior rows with each node split
            // over a wave pair, then the rows next to the walls
            constexpr int R = Axis<LY>::vmax;
            const int interior = (a.ny - 2 * R) * a.nx, walls = 2 * R * a.nx;
            if (interior > 0)
                hipLaunchKernelGGL((step_kernel_split<LX, LY, ST, BCX, BCY>),
                                   dim3((interior + kSplitNodes - 1) / kSplitNodes), dim3(kBlock), 0, s, a);
            hipLaunchKernelGGL((step_kernel<LX, LY, ST, BCX, BCY, ROWS_WALLS>), dim3((walls + kBlock - 1) / kBlock),
                               dim3(kBlock), 0, s, a);
        } else if constexpr (Elem<ST>::bytes == 2 && BCY == BCY_WALL) {
            // packed interior rows and the rows next to the walls: one launch
            // where both fit the packed kernel's registers, else two
            constexpr int R = Axis<LY>::vmax;  // rows next to each wall that take emission
            const int interior = (a.ny - 2 * R) * a.nx, walls = 2 * R * a.nx;
            const int ib = (interior + kBlock - 1) / kBlock;
            if constexpr (merged_walls<LX, LY, ST>()) {
                if (interior > 0)
                    hipLaunchKernelGGL((step_kernel_rows<LX, LY, ST, BCX, BCY, true>),
                                       dim3(wall_blocks<LY>(a.nx) + ib), dim3(kBlock), 0, s, a);
                else
                    hipLaunchKernelGGL((step_kernel<LX, LY, ST, BCX, BCY, ROWS_WALLS>),
                                       dim3((walls + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
            } else {
                if (interior > 0)
                    hipLaunchKernelGGL((step_kernel_rows<LX, LY, ST, BCX, BCY, false>), dim3(ib), dim3(kBlock), 0,
                                       s, a);
                hipLaunchKernelGGL((step_kernel<LX, LY, ST, BCX, BCY, ROWS_WALLS>),
                                   dim3((walls + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
            }
        } else if constexpr (BCY == BCY_WALL && Axis<LY>::vmax >= 7) {
            // FP32 storage with walls that reach 7 rows or more: the wall rows
            // in the first blocks, the interior rows (branch-free pull) in the
            // others (measured 2-8% faster there than one branchy pull per
            // node; 0.5-3.5% slower for shorter reach, which keeps it)
            constexpr int R = Axis<LY>::vmax;
            const int interior = (a.ny - 2 * R) * a.nx, walls = 2 * R * a.nx;
            if constexpr (fp32_merged_walls<LY>()) {
                if (interior > 0)
                    hipLaunchKernelGGL((step_kernel_rows<LX, LY, ST, BCX, BCY, true>),
                                       dim3(wall_blocks<LY>(a.nx) + (interior + kBlock - 1) / kBlock), dim3(kBlock),
                                       0, s, a);
                else
                    hipLaunchKernelGGL((step_kernel<LX, LY, ST, BCX, BCY, ROWS_WALLS>),
                                       dim3((walls + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
            } else {
                if (interior > 0)
                    hipLaunchKernelGGL((step_kernel_rows<LX, LY, ST, BCX, BCY, false>),
                                       dim3((interior + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
                hipLaunchKernelGGL((step_kernel<LX, LY, ST, BCX, BCY, ROWS_WALLS>), dim3((walls + kBlock - 1) / kBlock),
                                   dim3(kBlock), 0, s, a);
            }
        } else {
            hipLaunchKernelGGL((step_kernel<LX, LY, ST, BCX, BCY, ROWS_ALL>), dim3(grid), dim3(kBlock), 0, s, a);
        }
        return hipGetLastError();
    }
    static hipError_t observe(const KArgs &a, int grid, hipStream_t s)
    {
        hipLaunchKernelGGL((observe_kernel<LX, LY, ST, BCX, BCY>), dim3(grid), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    static hipError_t init(const KArgs &a, int grid, hipStream_t s)
    {
        hipLaunchKernelGGL((init_kernel<LX, LY, ST, BCX, BCY>), dim3(grid), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    static hipError_t stats(const KArgs &a, int grid, hipStream_t s)
    {
        hipLaunchKernelGGL((stats_kernel<LX, LY, ST, BCX, BCY>), dim3(grid), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    static hipError_t ends(const KArgs &a, int grid, float rl, float rr, hipStream_t s)
    {
        hipLaunchKernelGGL((ends_kernel<LX, LY, ST>), dim3(grid), dim3(kBlock), 0, s, a, rl, rr);
        return hipGetLastError();
    }
    static hipError_t batch(int rows, const BatchTile *tiles, int ntiles, int block, const KArgs *args,
                            const int32_t *phase, const int64_t *t0, const int64_t *bstep, int launch, hipStream_t s)
    {
        if (rows == ROWS_INTERIOR)
            hipLaunchKernelGGL((batch_step_kernel<LX, LY, ST, BCX, BCY, ROWS_INTERIOR>), dim3(ntiles), dim3(block), 0,
                               s, tiles, args, phase, t0, bstep, launch);
        else if (rows == ROWS_WALLS)
            hipLaunchKernelGGL((batch_step_kernel<LX, LY, ST, BCX, BCY, ROWS_WALLS>), dim3(ntiles), dim3(block), 0, s,
                               tiles, args, phase, t0, bstep, launch);
        else
            hipLaunchKernelGGL((batch_step_kernel<LX, LY, ST, BCX, BCY, ROWS_ALL>), dim3(ntiles), dim3(block), 0, s,
                               tiles, args, phase, t0, bstep, launch);
        return hipGetLastError();
    }
    static hipError_t resident(const int32_t *members, int nmembers, const KArgs *args, const int32_t *phase,
                               const int64_t *t0, const int64_t *bstep, int steps, hipStream_t s)
    {
        hipLaunchKernelGGL((resident_step_kernel<LX, LY, ST, BCX, BCY>), dim3(nmembers), dim3(kBlock), 0, s, members,
                           args, phase, t0, bstep, steps);
        return hipGetLastError();
    }
    static void add()
    {
        Variant *v = variant_slot(LX, LY, ST, BCX, BCY);
        v->step = &step;
        v->observe = &observe;
        v->init = &init;
        v->stats = &stats;
        v->ends = BCX == BCX_EQ ? &ends : nullptr;
        v->batch = &batch;
        v->resident = &resident;
        v->split_rows = Elem<ST>::bytes == 2 && BCY == BCY_WALL;
        v->wall_rates = BCY == BCY_WALL && wall_prepass<LX, LY, ST>();
    }
};

template <int LX, int LY, int BCX, int BCY>
void add_all_storages()
{
    Launchers<LX, LY, ST_F32, BCX, BCY>::add();
    Launchers<LX, LY, ST_F32S, BCX, BCY>::add();
    Launchers<LX, LY, ST_BF16S, BCX, BCY>::add();
    Launchers<LX, LY, ST_BF16SR, BCX, BCY>::add();
}

}  // namespace

#define GLBM_CAT2(a, b) a##b
#define GLBM_CAT(a, b) GLBM_CAT2(a, b)
#define GLBM_REG3(E, C, L) register_##E##_##C##_##L
#define GLBM_REG(E, C, L) GLBM_REG3(E, C, L)

// The registration function's kind: 0 one-dimensional, 1 two-dimensional
// (periodic y for the symmetric lattices; the mixed lattices), 2 the
// symmetric lattices with walls (-DGLBM_WALLS=1: their own object, so that
// the largest levels build in parallel halves).
#ifndef GLBM_WALLS
#define GLBM_WALLS 0
#endif
#if !GLBM_COMPACT
#define GLBM_KIND 0
#elif GLBM_WALLS && GLBM_LEVEL >= 1 && GLBM_LEVEL <= 7
#define GLBM_KIND 2
#else
#define GLBM_KIND 1
#endif

// Axis codes of this object: the G-D1Q(2N+1) axis of level N, or the
// G-D1Q(2N+2) one (code kEven + N).
#if GLBM_EVEN
#define GLBM_AX(N) (kEven + (N))
#else
#define GLBM_AX(N) (N)
#endif

#if GLBM_LEVEL >= 8
// Levels 8..13: only the mixed channel lattice D1Q3 (streamwise x) x
// G-D1Q(2N+2) (across the walls), one object per level.
#if !GLBM_EVEN || !GLBM_COMPACT
#error "levels above 7 exist only for the even axis of the mixed lattices (-DGLBM_EVEN=1 -DGLBM_COMPACT=1)"
#endif
void GLBM_REG(GLBM_EVEN, GLBM_KIND, GLBM_LEVEL)()
{
    add_all_storages<1, GLBM_AX(GLBM_LEVEL), BCX_WRAP, BCY_WALL>();
}
#elif GLBM_LEVEL >= 1
void GLBM_REG(GLBM_EVEN, GLBM_KIND, GLBM_LEVEL)()
{
    constexpr int N = GLBM_LEVEL, A = GLBM_AX(GLBM_LEVEL);
#if GLBM_COMPACT
    // two dimensions, the same axis twice, periodic x in compact rows:
    // periodic y, or walls across y (-DGLBM_WALLS=1).  Above 144 velocities
    // (N = 7 odd and even) the steps of interior nodes run split over wave
    // pairs; their other one-node launches (wall rows, batched steps,
    // observation) take one wave and may spill to scratch.
#if GLBM_WALLS
    add_all_storages<A, A, BCX_WRAP, BCY_WALL>();
#else
    add_all_storages<A, A, BCX_WRAP, BCY_PERIODIC>();
#endif
#else
    // one dimension: periodic or fixed equilibrium ends (padded rows)
    add_all_storages<A, 0, BCX_PERIODIC, BCY_PERIODIC>();
    add_all_storages<A, 0, BCX_EQ, BCY_PERIODIC>();
#endif
    (void)N;
}
#elif GLBM_COMPACT
// Mixed lattices D1Q3 (streamwise x) x G-D1Q(2N+1) or G-D1Q(2N+2) (across the
// walls), the form the channel flows of sections 5.3-5.4 use; periodic x in
// compact rows.
void GLBM_REG(GLBM_EVEN, GLBM_KIND, 0)()
{
    constexpr int BX = BCX_WRAP;
#if !GLBM_EVEN
    add_all_storages<1, 2, BX, BCY_WALL>();
#else
    add_all_storages<1, GLBM_AX(1), BX, BCY_WALL>();
    add_all_storages<1, GLBM_AX(2), BX, BCY_WALL>();
#endif
    add_all_storages<1, GLBM_AX(3), BX, BCY_WALL>();
    add_all_storages<1, GLBM_AX(4), BX, BCY_WALL>();
    add_all_storages<1, GLBM_AX(5), BX, BCY_WALL>();
    add_all_storages<1, GLBM_AX(6), BX, BCY_WALL>();
    add_all_storages<1, GLBM_AX(7), BX, BCY_WALL>();
}
#else
#error "the mixed lattices are two-dimensional: build them with -DGLBM_COMPACT=1"
#endif

}  // namespace glbm
