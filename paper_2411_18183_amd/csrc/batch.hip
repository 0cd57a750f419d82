// Many independent joins per launch sequence: every join j gets its own
// segment of one slot array (Build(R_j, H_sign) of Section 3.2, Figure 2),
// sized on the device so that no host round trip is needed; the probe side
// of all joins then runs through the fused probe kernel in one launch.
#include "asj_internal.h"

namespace {

constexpr int kPlanBlock = 1024;

__global__ __launch_bounds__(kPlanBlock) void batch_plan_kernel(const int64_t *__restrict__ r_seg,
                                                                const int64_t *__restrict__ s_seg, int32_t J, float lf,
                                                                asj_join_desc *__restrict__ desc,
                                                                int64_t *__restrict__ rows_done,
                                                                int64_t *__restrict__ out_count,
                                                                int64_t *__restrict__ cand_count,
                                                                uint64_t *__restrict__ done_clock,
                                                                uint64_t *__restrict__ total_slots)
{
    __shared__ uint64_t scan[kPlanBlock];
    __shared__ uint64_t carry;
    const uint64_t start = wall_clock64();
    const int tid = threadIdx.x;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < J; base += kPlanBlock) {
        const int j = base + tid;
        uint64_t cap = 0;
        if (j < J) {
            const int64_t nr = r_seg[j + 1] - r_seg[j];
            cap = 64;
            while ((double)cap * lf < (double)nr) cap <<= 1;
        }
        scan[tid] = cap;
        __syncthreads();
        for (int d = 1; d < kPlanBlock; d <<= 1) { // inclusive scan
            const uint64_t v = tid >= d ? scan[tid - d] : 0;
            __syncthreads();
            scan[tid] += v;
            __syncthreads();
        }
        if (j < J) {
            desc[j].tbase = carry + scan[tid] - cap;
            desc[j].mask = cap - 1;
            rows_done[j] = 0;
            out_count[j] = 0;
            if (cand_count) cand_count[j] = 0;
            if (done_clock) done_clock[j] = (s_seg[j + 1] == s_seg[j]) ? start : 0;
        }
        __syncthreads();
        if (tid == kPlanBlock - 1) carry += scan[kPlanBlock - 1];
        __syncthreads();
    }
    if (tid == 0) {
        *total_slots = carry;
        if (done_clock) done_clock[J] = start;
    }
}

__global__ void fill_slots_kernel(uint64_t *__restrict__ slots, int64_t bound, const uint64_t *__restrict__ total)
{
    const int64_t n = min(bound, (int64_t)*total);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        slots[i] = ASJ_EMPTY_SLOT;
}

__global__ void insert_batch_kernel(const uint32_t *__restrict__ sig, int64_t m, const int64_t *__restrict__ r_seg,
                                    int32_t J, const asj_join_desc *__restrict__ desc, uint64_t *__restrict__ slots,
                                    int32_t *__restrict__ status)
{
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < m; g += (int64_t)gridDim.x * blockDim.x) {
        const int j = asj_find_seg(r_seg, J, g);
        const asj_join_desc d = desc[j];
        const uint32_t sg = sig[g];
        const uint64_t val = ((uint64_t)sg << 32) | (uint32_t)g;
        uint64_t h = asj_mix32(sg) & d.mask;
        uint64_t tries = 0;
        for (;;) {
            const uint64_t old = atomicCAS((unsigned long long *)&slots[d.tbase + h],
                                           (unsigned long long)ASJ_EMPTY_SLOT, (unsigned long long)val);
            if (old == ASJ_EMPTY_SLOT) break;
            h = (h + 1) & d.mask;
            if (++tries > d.mask) {
                atomicExch(status, (int32_t)ASJ_ETABLEFULL);
                break;
            }
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

hipError_t asj_launch_batch_plan(const int64_t *r_seg, const int64_t *s_seg, int32_t njoins, float load_factor,
                                 asj_join_desc *desc, int64_t *rows_done, int64_t *out_count, int64_t *cand_count,
                                 uint64_t *done_clock, uint64_t *total_slots, hipStream_t st)
{
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(kPlanBlock), 0, st, r_seg, s_seg, njoins, load_factor, desc,
                       rows_done, out_count, cand_count, done_clock, total_slots);
    return hipGetLastError();
}

hipError_t asj_launch_fill_slots(uint64_t *slots, int64_t bound, const uint64_t *total_slots, hipStream_t st)
{
    if (bound <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_slots_kernel, dim3(grid_for(bound, 256, 16384)), dim3(256), 0, st, slots, bound,
                       total_slots);
    return hipGetLastError();
}

hipError_t asj_launch_insert_batch(const uint32_t *sig, int64_t m, const int64_t *r_seg, int32_t njoins,
                                   const asj_join_desc *desc, uint64_t *slots, int32_t *status, hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(insert_batch_kernel, dim3(grid_for(m, 256, 16384)), dim3(256), 0, st, sig, m, r_seg, njoins,
                       desc, slots, status);
    return hipGetLastError();
}
