// Kernel instantiations of the three-dimensional lattices (glbm_device3.h),
// periodic x in compact rows.  Built: D3Q27, G-D3Q125, and the channel lattices D1Q3 x G-D1Q(2N+1) x D1Q3
// (N = 2, 3) and D1Q3 x G-D1Q(2N+2) x D1Q3 (N = 2, 3) with y periodic or
// walls, each in the four storages.
#include "glbm_internal.h"
#include "glbm_device3.h"

namespace glbm {
namespace {

template <int LX, int LY, int LZ, int ST, int BCX, int BCY>
struct Launchers3 {
    static hipError_t step(const KArgs &a, int grid, hipStream_t s)
    {
        if constexpr (BCY == BCY_WALL) {
            // the wall rows in the first blocks, then the interior rows
            constexpr int R = Axis<LY>::vmax;
            const int interior = a.nz * (a.ny - 2 * R) * a.nx;
            grid = wall_blocks3<LY>(a.nx, a.nz) + (interior + kBlock - 1) / kBlock;
        }
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
    static void add()
    {
        Variant *v = variant3_slot(LX, LY, LZ, ST, BCX, BCY);
        v->step = &step;
        v->observe = &observe;
        v->init = &init;
        v->stats = &stats;
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

void register3()
{
    add_lattice3<1, 1, 1>();
    add_lattice3<2, 2, 2>();
    add_lattice3<1, 2, 1>();
    add_lattice3<1, 3, 1>();
    add_lattice3<1, kEven + 2, 1>();
    add_lattice3<1, kEven + 3, 1>();
}

}  // namespace glbm
