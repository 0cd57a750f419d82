// Output ordering (ASJ_SORTED): the stored result pairs sorted by (r_id,
// s_id) as signed integers, with an LSD radix sort over 64-bit keys (8-bit
// digits, 8 passes) whose element count is read from device memory, so the
// call needs no host round trip.  A pass whose digit is the same for every
// key is skipped on the device (ids below 2^24 leave two of the eight digits
// constant).
//
// Pass p: per-tile digit histograms -> per-digit exclusive scans over tiles
// -> digit bases -> stable scatter (items keep their order within a digit,
// which is what makes the LSD passes sort).  cur[p] names the buffer pass p
// reads; cur[p + 1] = cur[p] when the pass is skipped, else the other one.
#include "asj_internal.h"

namespace {

constexpr int kBlock = 256;            // threads per block
constexpr int kItems = 16;             // items per thread and tile
constexpr int kTile = kBlock * kItems; // 4096
constexpr int kDigits = 256;
constexpr int kPasses = 8;

__device__ __forceinline__ uint64_t pair_key(asj_pair p)
{
    return ((uint64_t)((uint32_t)p.r_id ^ 0x80000000u) << 32) | (uint64_t)((uint32_t)p.s_id ^ 0x80000000u);
}

__device__ __forceinline__ int64_t stored(const int64_t *count, int64_t cap)
{
    const int64_t c = *count;
    return c < 0 ? 0 : (c < cap ? c : cap);
}

__global__ void to_keys_kernel(const asj_pair *__restrict__ in, const int64_t *__restrict__ count, int64_t cap,
                               uint64_t *__restrict__ k, int32_t *__restrict__ cur)
{
    const int64_t n = stored(count, cap);
    if (blockIdx.x == 0 && threadIdx.x == 0) cur[0] = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        k[i] = pair_key(in[i]);
}

__global__ __launch_bounds__(kBlock) void hist_kernel(const uint64_t *__restrict__ k0, const uint64_t *__restrict__ k1,
                                                      const int32_t *__restrict__ cur, int pass,
                                                      const int64_t *__restrict__ count, int64_t cap,
                                                      uint32_t *__restrict__ tile_hist)
{
    __shared__ uint32_t h[kDigits];
    const int64_t n = stored(count, cap);
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    if (t0 >= n) return;
    const uint64_t *src = cur[pass] ? k1 : k0;
    h[threadIdx.x] = 0;
    __syncthreads();
    for (int r = 0; r < kItems; r++) {
        const int64_t i = t0 + r * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(src[i] >> (8 * pass)) & 255u], 1u);
    }
    __syncthreads();
    tile_hist[(int64_t)blockIdx.x * kDigits + threadIdx.x] = h[threadIdx.x];
}

// Block b: exclusive scan over tiles of digit b's tile counts (in place),
// and digit b's total.
__global__ __launch_bounds__(kBlock) void scan_cols_kernel(uint32_t *__restrict__ tile_hist,
                                                           const int64_t *__restrict__ count, int64_t cap,
                                                           uint32_t *__restrict__ col_tot)
{
    __shared__ uint32_t s[kBlock];
    const int64_t n = stored(count, cap);
    const int64_t ntiles = (n + kTile - 1) / kTile;
    const int b = blockIdx.x;
    uint32_t carry = 0;
    for (int64_t base = 0; base < ntiles; base += kBlock) {
        const int64_t t = base + threadIdx.x;
        const uint32_t v = t < ntiles ? tile_hist[t * kDigits + b] : 0u;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < kBlock; d <<= 1) {
            const uint32_t add = threadIdx.x >= d ? s[threadIdx.x - d] : 0u;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (t < ntiles) tile_hist[t * kDigits + b] = carry + s[threadIdx.x] - v;
        carry += s[kBlock - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) col_tot[b] = carry;
}

// One block: digit bases, and whether the pass can be skipped.
__global__ __launch_bounds__(kBlock) void scan_tot_kernel(const uint32_t *__restrict__ col_tot,
                                                          const int64_t *__restrict__ count, int64_t cap,
                                                          uint32_t *__restrict__ base, int32_t *__restrict__ cur,
                                                          int pass)
{
    __shared__ uint32_t s[kDigits];
    __shared__ int one_digit;
    const int64_t n = stored(count, cap);
    const uint32_t v = col_tot[threadIdx.x];
    if (threadIdx.x == 0) one_digit = 0;
    s[threadIdx.x] = v;
    __syncthreads();
    if ((int64_t)v == n) one_digit = 1; // also true for every digit when n = 0
    for (int d = 1; d < kDigits; d <<= 1) {
        const uint32_t add = threadIdx.x >= d ? s[threadIdx.x - d] : 0u;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    base[threadIdx.x] = s[threadIdx.x] - v;
    if (threadIdx.x == 0) cur[pass + 1] = (one_digit || n == 0) ? cur[pass] : 1 - cur[pass];
}

__global__ __launch_bounds__(kBlock) void scatter_kernel(uint64_t *__restrict__ k0, uint64_t *__restrict__ k1,
                                                         const int32_t *__restrict__ cur, int pass,
                                                         const int64_t *__restrict__ count, int64_t cap,
                                                         const uint32_t *__restrict__ tile_hist,
                                                         const uint32_t *__restrict__ base)
{
    __shared__ uint32_t run[kDigits];                  // items of each digit placed by earlier rounds
    __shared__ uint32_t wcnt[kBlock / ASJ_WAVE][kDigits]; // this round's count per wave and digit
    const int64_t n = stored(count, cap);
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    if (t0 >= n || cur[pass + 1] == cur[pass]) return; // past the end, or the pass is skipped
    const uint64_t *src = cur[pass] ? k1 : k0;
    uint64_t *dst = cur[pass] ? k0 : k1;
    const int lane = threadIdx.x % ASJ_WAVE, wave = threadIdx.x / ASJ_WAVE;
    const uint64_t lanemask_lt = (1ull << lane) - 1ull;
    run[threadIdx.x] = tile_hist[(int64_t)blockIdx.x * kDigits + threadIdx.x] + base[threadIdx.x];
    for (int r = 0; r < kItems; r++) {
        for (int w = 0; w < kBlock / ASJ_WAVE; w++) wcnt[w][threadIdx.x] = 0;
        __syncthreads();
        const int64_t i = t0 + r * kBlock + threadIdx.x;
        const bool valid = i < n;
        const uint64_t key = valid ? src[i] : 0ull;
        const uint32_t d = (uint32_t)(key >> (8 * pass)) & 255u;
        // lanes of this wave with the same digit
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; bit++) {
            const uint64_t ones = __ballot((d >> bit) & 1u);
            same &= ((d >> bit) & 1u) ? ones : ~ones;
        }
        const uint32_t before = (uint32_t)__popcll(same & lanemask_lt);
        if (valid && before == 0) wcnt[wave][d] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + before;
            for (int w = 0; w < wave; w++) pos += wcnt[w][d];
            dst[pos] = key;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kBlock / ASJ_WAVE; w++) add += wcnt[w][threadIdx.x];
        run[threadIdx.x] += add;
        __syncthreads();
    }
}

__global__ void from_keys_kernel(const uint64_t *__restrict__ k0, const uint64_t *__restrict__ k1,
                                 const int32_t *__restrict__ cur, const int64_t *__restrict__ count, int64_t cap,
                                 asj_pair *__restrict__ out)
{
    const int64_t n = stored(count, cap);
    const uint64_t *src = cur[kPasses] ? k1 : k0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = src[i];
        asj_pair p;
        p.r_id = (int32_t)((uint32_t)(k >> 32) ^ 0x80000000u);
        p.s_id = (int32_t)((uint32_t)k ^ 0x80000000u);
        out[i] = p;
    }
}

int grid_for(int64_t n, int block, int cap)
{
    int64_t g = (n + block - 1) / block;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (int)g;
}

} // namespace

size_t asj_sort_scratch_bytes(int64_t cap)
{
    const int64_t tiles = (cap + kTile - 1) / kTile;
    return 2 * sizeof(uint64_t) * (size_t)(cap > 0 ? cap : 1) + sizeof(uint32_t) * kDigits * (size_t)(tiles + 2) +
           sizeof(int32_t) * 16 + 1024;
}

hipError_t asj_launch_sort_pairs(asj_pair *pairs, const int64_t *count, int64_t cap, void *scratch, hipStream_t st)
{
    if (cap <= 0) return hipSuccess;
    const int64_t tiles = (cap + kTile - 1) / kTile;
    uint8_t *p = (uint8_t *)scratch;
    uint64_t *k0 = (uint64_t *)p;
    uint64_t *k1 = k0 + cap;
    uint32_t *tile_hist = (uint32_t *)(k1 + cap);
    uint32_t *col_tot = tile_hist + kDigits * tiles;
    uint32_t *base = col_tot + kDigits;
    int32_t *cur = (int32_t *)(base + kDigits);
    const int g = grid_for(cap, kBlock, 16384);
    hipLaunchKernelGGL(to_keys_kernel, dim3(g), dim3(kBlock), 0, st, pairs, count, cap, k0, cur);
    for (int pass = 0; pass < kPasses; pass++) {
        hipLaunchKernelGGL(hist_kernel, dim3((unsigned)tiles), dim3(kBlock), 0, st, k0, k1, cur, pass, count, cap,
                           tile_hist);
        hipLaunchKernelGGL(scan_cols_kernel, dim3(kDigits), dim3(kBlock), 0, st, tile_hist, count, cap, col_tot);
        hipLaunchKernelGGL(scan_tot_kernel, dim3(1), dim3(kBlock), 0, st, col_tot, count, cap, base, cur, pass);
        hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)tiles), dim3(kBlock), 0, st, k0, k1, cur, pass, count, cap,
                           tile_hist, base);
    }
    hipLaunchKernelGGL(from_keys_kernel, dim3(g), dim3(kBlock), 0, st, k0, k1, cur, count, cap, pairs);
    return hipGetLastError();
}
