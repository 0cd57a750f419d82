// Build(R, H_sign) (Section 3.2, Figure 2): every build row's signature is
// placed in an open-addressing table of 64-bit slots
//     slot = signature << 32 | row        (empty slot = all ones),
// at mix32(signature) modulo the power-of-two capacity, moving to the next
// slot while it is taken (linear probing).  Rows with equal signatures are
// all kept (a multimap): they share a home slot, so every one of them lies
// on the run a probe walks until the first empty slot.
//
// Two passes instead of one CAS per row (64-bit CAS is about three times
// slower than a store here): every row first stores itself into its home
// slot (one of the rows sharing a home survives, whole, as 64-bit stores do
// not tear); after that, a row that does not find itself there claims the
// first empty slot after its home with CAS.  Every slot from a row's home to
// its final slot is then occupied -- the home by the survivor, the rest
// because the row's CAS found them taken and slots never empty again -- so
// lookups find every row on the run from its home.
//
// The baseline simple hash join (Section 2) uses the same layout with the
// plain key hash choosing the home slot and no signature stored (the high
// word is zero), so its probe must compare every occupied slot it visits.
#include "asj_internal.h"

namespace {

__global__ void fill64_kernel(uint64_t *__restrict__ p, int64_t n, uint64_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_i64_kernel(int64_t *__restrict__ p, int64_t n, int64_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// A new table: every slot empty and the status word cleared, in one launch.
__global__ void table_init_kernel(uint64_t *__restrict__ slots, int64_t cap, int32_t *__restrict__ status)
{
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) *status = ASJ_OK;
    for (int64_t i = i0; i < cap; i += (int64_t)gridDim.x * blockDim.x) slots[i] = ASJ_EMPTY_SLOT;
}

// Two 64-bit counters cleared in one launch (b may be NULL).
__global__ void zero2_kernel(int64_t *__restrict__ a, int64_t *__restrict__ b)
{
    if (threadIdx.x == 0) *a = 0;
    if (threadIdx.x == 1 && b) *b = 0;
}

// Counters, status word and a word array cleared in one launch (see
// asj_launch_local_init).
__global__ void local_init_kernel(int64_t *__restrict__ a, int64_t *__restrict__ b, int32_t *__restrict__ status,
                                  uint32_t *__restrict__ words, int64_t nwords)
{
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) {
        *a = 0;
        if (b) *b = 0;
        *status = ASJ_OK;
    }
    if (words)
        for (int64_t i = i0; i < nwords; i += (int64_t)gridDim.x * blockDim.x) words[i] = 0u;
}

__global__ void fill_i32_kernel(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Pass 1 (STORE = 1): row r stores itself into its home slot.  Pass 2
// (STORE = 0): a row that lost its home slot walks on from the next slot,
// taking the first empty one with CAS.
// Offsets that start below zero or decrease would send the kernels outside
// the arena; one violation anywhere marks the status word.
__global__ void validate_kernel(const int64_t *__restrict__ off, int64_t n, int32_t *__restrict__ status)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if ((i == 0 && off[0] < 0) || off[i + 1] < off[i]) atomicExch(status, (int32_t)ASJ_EINVAL);
}

template <int PLAIN, int STORE>
__global__ void insert_kernel(const uint32_t *__restrict__ sig, int64_t m, uint64_t *__restrict__ slots,
                              uint64_t mask, int32_t *__restrict__ status)
{
    if (*status != ASJ_OK) return; // validation failed: the signatures were never written
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t sg = sig[r];
        const uint64_t val = PLAIN ? (uint64_t)(uint32_t)r : (((uint64_t)sg << 32) | (uint32_t)r);
        uint64_t h = asj_mix32(sg) & mask;
        if (STORE) {
            slots[h] = val;
            continue;
        }
        if (slots[h] == val) continue;
        uint64_t tries = 0;
        for (;;) {
            h = (h + 1) & mask;
            if (++tries > mask) { // every slot taken
                atomicExch(status, (int32_t)ASJ_ETABLEFULL);
                break;
            }
            const uint64_t old = atomicCAS((unsigned long long *)&slots[h], (unsigned long long)ASJ_EMPTY_SLOT,
                                           (unsigned long long)val);
            if (old == ASJ_EMPTY_SLOT) break;
        }
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

hipError_t asj_launch_fill64(uint64_t *p, int64_t n, uint64_t v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill64_kernel, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t asj_launch_table_init(uint64_t *slots, int64_t cap, int32_t *status, hipStream_t st)
{
    hipLaunchKernelGGL(table_init_kernel, dim3(grid_for(cap > 0 ? cap : 1, 256, 16384)), dim3(256), 0, st, slots, cap,
                       status);
    return hipGetLastError();
}

hipError_t asj_launch_local_init(int64_t *a, int64_t *b, int32_t *status, uint32_t *words, int64_t nwords,
                                 hipStream_t st)
{
    const int g = grid_for(nwords > 0 ? nwords : 1, 256, 4096);
    hipLaunchKernelGGL(local_init_kernel, dim3(g), dim3(256), 0, st, a, b, status, words, nwords);
    return hipGetLastError();
}

hipError_t asj_launch_zero2(int64_t *a, int64_t *b, hipStream_t st)
{
    hipLaunchKernelGGL(zero2_kernel, dim3(1), dim3(64), 0, st, a, b);
    return hipGetLastError();
}

hipError_t asj_launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i64_kernel, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t asj_launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t asj_launch_validate(const int64_t *off, int64_t n, int32_t *status, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(validate_kernel, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, off, n, status);
    return hipGetLastError();
}

hipError_t asj_launch_insert(const uint32_t *sig, int64_t m, int plain, uint64_t *slots, uint64_t mask,
                             int32_t *status, hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    const dim3 g(grid_for(m, 256, 16384)), b(256);
    if (plain) {
        hipLaunchKernelGGL((insert_kernel<1, 1>), g, b, 0, st, sig, m, slots, mask, status);
        hipLaunchKernelGGL((insert_kernel<1, 0>), g, b, 0, st, sig, m, slots, mask, status);
    } else {
        hipLaunchKernelGGL((insert_kernel<0, 1>), g, b, 0, st, sig, m, slots, mask, status);
        hipLaunchKernelGGL((insert_kernel<0, 0>), g, b, 0, st, sig, m, slots, mask, status);
    }
    return hipGetLastError();
}
