// Bandwidth probe: a measurement utility beside the method, giving the HBM
// rates this GPU reaches with plain streaming kernels (the ceiling the step
// kernels' roofline fractions are read against) and a kernel of known byte
// count for calibrating the memory counters.
//
// Three passes over device buffers, 16-byte non-temporal accesses, grid-stride
// loops: copy (read n bytes, write n bytes), read only, write only.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/glbm.h"

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kProbeBlock = 256;

__global__ __launch_bounds__(kProbeBlock) void probe_copy(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                          size_t n)
{
    for (size_t i = (size_t)blockIdx.x * kProbeBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kProbeBlock)
        __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}

// The loads feed a running xor that is stored only if it hits one chosen
// value: the compiler must keep every load, and the store almost never runs.
__global__ __launch_bounds__(kProbeBlock) void probe_read(const u32x4 *__restrict__ src, size_t n,
                                                          uint32_t *__restrict__ sink)
{
    uint32_t acc = 0;
    for (size_t i = (size_t)blockIdx.x * kProbeBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kProbeBlock) {
        const u32x4 v = __builtin_nontemporal_load(&src[i]);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;
}

__global__ __launch_bounds__(kProbeBlock) void probe_write(u32x4 *__restrict__ dst, size_t n, uint32_t value)
{
    const u32x4 v = {value, value, value, value};
    for (size_t i = (size_t)blockIdx.x * kProbeBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kProbeBlock)
        __builtin_nontemporal_store(v, &dst[i]);
}

}  // namespace

extern "C" int glbm_bandwidth_probe(int32_t mode, const void *src, void *dst, size_t bytes, int32_t blocks,
                                    void *stream)
{
    if (bytes == 0 || (bytes & 15) || blocks < 1) return GLBM_ERR_INVALID;
    if ((mode == 0 || mode == 1) && (!src || ((uintptr_t)src & 15))) return GLBM_ERR_INVALID;
    if (!dst || ((uintptr_t)dst & 15)) return GLBM_ERR_INVALID;
    const size_t n = bytes / 16;
    hipStream_t s = (hipStream_t)stream;
    if (mode == 0)
        hipLaunchKernelGGL(probe_copy, dim3(blocks), dim3(kProbeBlock), 0, s, (const u32x4 *)src, (u32x4 *)dst, n);
    else if (mode == 1)
        hipLaunchKernelGGL(probe_read, dim3(blocks), dim3(kProbeBlock), 0, s, (const u32x4 *)src, n, (uint32_t *)dst);
    else if (mode == 2)
        hipLaunchKernelGGL(probe_write, dim3(blocks), dim3(kProbeBlock), 0, s, (u32x4 *)dst, n, 0x3f800000u);
    else
        return GLBM_ERR_INVALID;
    return hipGetLastError() == hipSuccess ? GLBM_OK : GLBM_ERR_HIP;
}
