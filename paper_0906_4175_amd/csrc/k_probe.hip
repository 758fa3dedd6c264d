// Calibration kernel: a plain 16-byte-per-lane streaming copy whose DRAM
// traffic is known exactly (reads `bytes`, writes `bytes`).  Hardware byte
// counters of the filter kernels are scaled by what they read for this copy.
#include <hip/hip_runtime.h>

#include "mf_internal.hpp"

namespace mf {

__global__ void __launch_bounds__(256) k_copy_probe(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                    size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_copy_probe, dim3((unsigned)blocks), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, n16);
    return hipGetLastError();
}

}  // namespace mf
