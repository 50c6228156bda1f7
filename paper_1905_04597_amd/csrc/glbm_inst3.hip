// Kernel instantiations of the three-dimensional lattices (glbm_device3.h),
// periodic x in compact rows.  Built: D3Q27, G-D3Q125, G-D3Q343, and the
// channel lattices D1Q3 x G-D1Q(2N+1) x D1Q3 and D1Q3 x G-D1Q(2N+2) x D1Q3
// (N = 2..7, up to 144 velocities) with y periodic or walls, each in the four
// storages.
#include "glbm_internal.h"
#include "glbm_device3.h"

namespace glbm {
namespace {

template <int LX, int LY, int LZ, int ST, int BCX, int BCY>
struct Launchers3 {
    static hipError_t step(const KArgs &a, int grid, hipStream_t s)
    {
        constexpr int R = Axis<LY>::vmax;
        constexpr int NB = kBlock / split3_waves<LX, LY, LZ, ST>();  // nodes per block
        if constexpr (BCY == BCY_WALL) {
            // the wall factors of every column, then the wall rows in the
            // first blocks of the step and the interior rows in the others
            if (!a.wrate) return hipErrorInvalidValue;
            const int cols = a.nx * a.nz;
            hipLaunchKernelGGL((wall_rate3_kernel<LX, LY, LZ, ST, BCX>), dim3((cols + kBlock / 2 - 1) / (kBlock / 2)),
                               dim3(kBlock), 0, s, a);
            const int interior = a.nz * (a.ny - 2 * R) * a.nx;
            grid = wall_blocks3<LY>(a.nx, a.nz, NB) + (interior + NB - 1) / NB;
        } else {
            grid = (a.nodes + NB - 1) / NB;
        }
        if constexpr (split3<LX, LY, LZ, ST>())
            hipLaunchKernelGGL((step3_split_kernel<LX, LY, LZ, ST, BCX, BCY>), dim3(grid), dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((step3_kernel<LX, LY, LZ, ST, BCX, BCY>), dim3(grid), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    static hipError_t observe(const KArgs &a, int grid, hipStream_t s)
    {
        hipLaunchKernelGGL((observe3_kernel<LX, LY, LZ, ST, BCX, BCY>), dim3(grid), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    static hipError_t init(const KArgs &a, int grid, hipStream_t s)
    {
        hipLaunchKernelGGL((init3_kernel<LX, LY, LZ, ST, BCX, BCY>), dim3(grid), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    static hipError_t stats(const KArgs &a, int grid, hipStream_t s)
    {
        hipLaunchKernelGGL((stats3_kernel<LX, LY, LZ, ST, BCX, BCY>), dim3(grid), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    // batched steps: one row set (every node), tiles of up to kBlock nodes
    static hipError_t batch(int rows, const BatchTile *tiles, int ntiles, int block, const KArgs *args,
                            const int32_t *phase, const int64_t *t0, const int64_t *bstep, int launch, hipStream_t s)
    {
        static_assert(Lat3<LX, LY, LZ, ST>::Q <= 144, "no batched step above 144 velocities");
        if (rows != ROWS_ALL || block > kBlock) return hipErrorInvalidValue;
        hipLaunchKernelGGL((batch_step3_kernel<LX, LY, LZ, ST, BCX, BCY>), dim3(ntiles), dim3(block), 0, s, tiles, args,
                           phase, t0, bstep, launch);
        return hipGetLastError();
    }
    static void add()
    {
        Variant *v = variant3_slot(LX, LY, LZ, ST, BCX, BCY);
        v->step = &step;
        v->observe = &observe;
        v->init = &init;
        v->stats = &stats;
        v->wall_rates = BCY == BCY_WALL;
        // no resident form: three-dimensional members are tiled; no batched
        // form above 144 velocities (the one-lane node code would live in
        // scratch memory)
        if constexpr (Lat3<LX, LY, LZ, ST>::Q <= 144) v->batch = &batch;
    }
};

template <int LX, int LY, int LZ>
void add_lattice3()
{
    constexpr int BCX = BCX_WRAP;
    Launchers3<LX, LY, LZ, ST_F32, BCX, BCY_PERIODIC>::add();
    Launchers3<LX, LY, LZ, ST_F32S, BCX, BCY_PERIODIC>::add();
    Launchers3<LX, LY, LZ, ST_BF16S, BCX, BCY_PERIODIC>::add();
    Launchers3<LX, LY, LZ, ST_BF16SR, BCX, BCY_PERIODIC>::add();
    Launchers3<LX, LY, LZ, ST_F32, BCX, BCY_WALL>::add();
    Launchers3<LX, LY, LZ, ST_F32S, BCX, BCY_WALL>::add();
    Launchers3<LX, LY, LZ, ST_BF16S, BCX, BCY_WALL>::add();
    Launchers3<LX, LY, LZ, ST_BF16SR, BCX, BCY_WALL>::add();
}

}  // namespace

// One object per part (-DGLBM_3D_PART=k), so that the slow three-dimensional
// instantiations build in parallel.
#if GLBM_3D_PART == 0
void register3_0()
{
    add_lattice3<1, 1, 1>();
    add_lattice3<2, 2, 2>();
}
#elif GLBM_3D_PART == 1
void register3_1()
{
    add_lattice3<1, 2, 1>();
    add_lattice3<1, 3, 1>();
    add_lattice3<1, kEven + 2, 1>();
    add_lattice3<1, kEven + 3, 1>();
}
#elif GLBM_3D_PART == 2
void register3_2()
{
    add_lattice3<1, 4, 1>();
    add_lattice3<1, kEven + 4, 1>();
}
#elif GLBM_3D_PART == 3
void register3_3()
{
    add_lattice3<1, 5, 1>();
    add_lattice3<1, kEven + 5, 1>();
}
#elif GLBM_3D_PART == 4
void register3_4() { add_lattice3<1, 6, 1>(); }
#elif GLBM_3D_PART == 5
void register3_5() { add_lattice3<1, kEven + 6, 1>(); }
#elif GLBM_3D_PART == 6
void register3_6() { add_lattice3<1, 7, 1>(); }
#elif GLBM_3D_PART == 7
void register3_7() { add_lattice3<1, kEven + 7, 1>(); }
#elif GLBM_3D_PART == 8
// G-D3Q343: the split step (four waves per node)
void register3_8() { add_lattice3<3, 3, 3>(); }
#else
#error "GLBM_3D_PART must be 0..8"
#endif

}  // namespace glbm
