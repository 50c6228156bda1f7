// Kernel instantiations for one hierarchy level, selected at compile time
// with -DGLBM_LEVEL=N (N = 1..7); -DGLBM_LEVEL=0 builds the mixed-level
// lattices.  -DGLBM_COMPACT=1 builds the compact-row variants of the 2D
// periodic-x lattices instead (narrow lattices).  Each (level, layout) is its
// own object file so the build runs in parallel.
#include "glbm_internal.h"

namespace glbm {
namespace {

template <int LX, int LY, int ST, int BCX, int BCY>
struct Launchers {
    static hipError_t step(const KArgs &a, int grid, hipStream_t s)
    {
        if constexpr (Elem<ST>::bytes == 2 && BCY == BCY_WALL) {
            // packed interior rows, then the rows next to the walls
            const int interior = (a.ny - 2 * LY) * a.nx, walls = 2 * LY * a.nx;
            if (interior > 0)
                hipLaunchKernelGGL((step_kernel<LX, LY, ST, BCX, BCY, ROWS_INTERIOR>),
                                   dim3((interior + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
            hipLaunchKernelGGL((step_kernel<LX, LY, ST, BCX, BCY, ROWS_WALLS>), dim3((walls + kBlock - 1) / kBlock),
                               dim3(kBlock), 0, s, a);
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
    static void add()
    {
        Variant *v = variant_slot(LX, LY, ST, BCX, BCY);
        v->step = &step;
        v->observe = &observe;
        v->init = &init;
        v->stats = &stats;
        v->ends = BCX == BCX_EQ ? &ends : nullptr;
        v->batch = &batch;
        v->split_rows = Elem<ST>::bytes == 2 && BCY == BCY_WALL;
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

#if GLBM_COMPACT
// Two dimensions with periodic x in compact rows: the same lattices as the
// padded 2D variants below.
#if GLBM_LEVEL >= 1
void GLBM_CAT(register_compact_, GLBM_LEVEL)()
{
    constexpr int N = GLBM_LEVEL;
    add_all_storages<N, N, BCX_WRAP, BCY_PERIODIC>();
    add_all_storages<N, N, BCX_WRAP, BCY_WALL>();
}
#else
void register_compact_mixed()
{
    add_all_storages<1, 2, BCX_WRAP, BCY_WALL>();
    add_all_storages<1, 3, BCX_WRAP, BCY_WALL>();
    add_all_storages<1, 4, BCX_WRAP, BCY_WALL>();
    add_all_storages<1, 5, BCX_WRAP, BCY_WALL>();
    add_all_storages<1, 6, BCX_WRAP, BCY_WALL>();
    add_all_storages<1, 7, BCX_WRAP, BCY_WALL>();
}
#endif
#elif GLBM_LEVEL >= 1
void GLBM_CAT(register_level_, GLBM_LEVEL)()
{
    constexpr int N = GLBM_LEVEL;
    // one dimension: periodic or fixed equilibrium ends
    add_all_storages<N, 0, BCX_PERIODIC, BCY_PERIODIC>();
    add_all_storages<N, 0, BCX_EQ, BCY_PERIODIC>();
    // two dimensions, same level on both axes: periodic or walls across y
    add_all_storages<N, N, BCX_PERIODIC, BCY_PERIODIC>();
    add_all_storages<N, N, BCX_PERIODIC, BCY_WALL>();
}
#else
// Mixed lattices G-D1Q3 (streamwise x) x G-D1Q(2N+1) (across the walls), the
// form the channel flows of sections 5.3-5.4 use.
void register_mixed()
{
    add_all_storages<1, 2, BCX_PERIODIC, BCY_WALL>();
    add_all_storages<1, 3, BCX_PERIODIC, BCY_WALL>();
    add_all_storages<1, 4, BCX_PERIODIC, BCY_WALL>();
    add_all_storages<1, 5, BCX_PERIODIC, BCY_WALL>();
    add_all_storages<1, 6, BCX_PERIODIC, BCY_WALL>();
    add_all_storages<1, 7, BCX_PERIODIC, BCY_WALL>();
}
#endif

}  // namespace glbm
