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

// Streaming read: every 16-byte word once, XOR-folded to one word per block
// so that the kernel writes (almost) nothing.
__global__ __launch_bounds__(256) void read_kernel(const uint4 *__restrict__ src, int64_t n16,
                                                   uint32_t *__restrict__ out)
{
    uint4 acc = make_uint4(0, 0, 0, 0);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) { // four independent loads in flight per lane
        uint4 v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            acc.x ^= v[u].x;
            acc.y ^= v[u].y;
            acc.z ^= v[u].z;
            acc.w ^= v[u].w;
        }
    }
    for (; i < n16; i += stride) {
        const uint4 v = src[i];
        acc.x ^= v.x;
        acc.y ^= v.y;
        acc.z ^= v.z;
        acc.w ^= v.w;
    }
    const uint32_t x = acc.x ^ acc.y ^ acc.z ^ acc.w;
    if (x) atomicXor(out, x);
}

} // namespace

hipError_t asj_launch_read(const void *src, int64_t bytes, uint32_t *out, int grid, hipStream_t st)
{
    const int64_t n16 = bytes / 16;
    if (n16 <= 0) return hipSuccess;
    hipLaunchKernelGGL(read_kernel, dim3((unsigned)grid), dim3(256), 0, st, (const uint4 *)src, n16, out);
    return hipGetLastError();
}

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
