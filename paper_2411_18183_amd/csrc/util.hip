// Measurement support: a plain streaming copy with a known byte count, used
// to calibrate hardware byte counters (bytes fetched / written per kernel).
#include "asj_internal.h"

namespace {

__global__ __launch_bounds__(256) void copy_kernel(uint4 *__restrict__ dst, const uint4 *__restrict__ src, int64_t n16)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void copy_tail_kernel(uint8_t *__restrict__ dst, const uint8_t *__restrict__ src, int64_t n)
{
    const int64_t i = threadIdx.x;
    if (i < n) dst[i] = src[i];
}

} // namespace

hipError_t asj_launch_copy(void *dst, const void *src, int64_t bytes, hipStream_t st)
{
    const int64_t n16 = bytes / 16;
    if (n16 > 0) {
        int64_t g = (n16 + 255) / 256;
        if (g > 256 * 64) g = 256 * 64;
        hipLaunchKernelGGL(copy_kernel, dim3((unsigned)g), dim3(256), 0, st, (uint4 *)dst, (const uint4 *)src, n16);
    }
    const int64_t tail = bytes - n16 * 16;
    if (tail > 0)
        hipLaunchKernelGGL(copy_tail_kernel, dim3(1), dim3(16), 0, st, (uint8_t *)dst + n16 * 16,
                           (const uint8_t *)src + n16 * 16, tail);
    return hipGetLastError();
}
