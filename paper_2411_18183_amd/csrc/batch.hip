// Many independent joins per launch sequence: every join j gets its own
// segment of one slot array (Build(R_j, H_sign) of Section 3.2, Figure 2),
// sized on the device so that no host round trip is needed and built by
// regions of up to 4096 slots (table.hip); the probe side of all joins then
// runs through the fused probe kernel in one launch.
// Joins with few build rows (local_rows > 0 and |R_j| <= local_rows) get no
// segment: the blocks that probe them build their table in LDS from the
// build signatures, and their probe windows are numbered apart.
//
// Rows are handled in windows that never span two joins (64 build rows per
// build window, keys_per_window probe rows per probe window), so every
// window knows its join from one map entry instead of a search over the
// segment bounds, and all of a window's bookkeeping goes to one join.
#include "asj_internal.h"

namespace {

constexpr int kPlanBlock = 1024;

// One block: segment capacities, window counts (build, probe and
// LDS-table probe windows), table regions and their prefix sums, counters
// zeroed (with the region counts of a build by regions), batch start clock.  Segment arrays that do not cover the
// relations exactly (first bound 0, last bound the row count, no bound
// decreasing), segments that would not fit slot_cap slots, or (local_only)
// a join too large for an LDS table, set *status to ASJ_EINVAL so that no
// later kernel of the batch touches the slots or reads a key.
template <int Q> // scanned quantities: 5, or 4 without table regions (no device table is built)
__global__ __launch_bounds__(kPlanBlock) void batch_plan_kernel(const int64_t *__restrict__ r_seg,
                                                                const int64_t *__restrict__ s_seg, int32_t J,
                                                                int64_t n_r, int64_t n_s, int64_t slot_cap, float lf,
                                                                int kpw, int64_t local_rows, int local_only,
                                                                asj_join_desc *__restrict__ desc,
                                                                int64_t *__restrict__ rows_done,
                                                                int64_t *__restrict__ out_count,
                                                                int64_t *__restrict__ cand_count,
                                                                uint64_t *__restrict__ done_clock,
                                                                uint64_t *__restrict__ tot, int32_t *__restrict__ status,
                                                                uint32_t *__restrict__ rcnt, int64_t rcnt_cap,
                                                                uint64_t *__restrict__ novf)
{
    constexpr int kWaves = kPlanBlock / ASJ_WAVE;
    __shared__ uint64_t wtot[Q][kWaves]; // per-wave totals of the current pass
    __shared__ uint64_t carry[Q];
    __shared__ int bad;
    const uint64_t start = wall_clock64();
    const int tid = threadIdx.x;
    const int lane = tid % ASJ_WAVE, wave = tid / ASJ_WAVE;
    if (tid < Q) carry[tid] = 0;
    if (tid == 0) bad = (r_seg[0] != 0 || s_seg[0] != 0 || r_seg[J] != n_r || s_seg[J] != n_s);
    __syncthreads();
    for (int base = 0; base < J; base += kPlanBlock) {
        const int j = base + tid;
        uint64_t v[5] = {0, 0, 0, 0, 0};
        if (j < J) {
            if (r_seg[j + 1] < r_seg[j] || s_seg[j + 1] < s_seg[j]) bad = 1;
            const int64_t nr = max((int64_t)0, r_seg[j + 1] - r_seg[j]);
            const int64_t ns = max((int64_t)0, s_seg[j + 1] - s_seg[j]);
            const uint64_t nw = (uint64_t)((ns + kpw - 1) / kpw);
            if (nr <= local_rows) { // no segment, no build windows: an LDS table
                v[3] = nw;
            } else {
                if (local_only) bad = 1; // the caller promised LDS tables only; nothing builds device tables
                uint64_t cap = 64;
                while ((double)cap * lf < (double)nr) cap <<= 1;
                v[0] = cap;
                v[1] = (uint64_t)((nr + ASJ_WAVE - 1) / ASJ_WAVE);
                v[2] = nw;
                if (Q > 4) v[4] = cap >> asj_seg_region_bits(cap);
            }
        }
        // inclusive scans: within each wave by shuffles, then over the
        // waves' totals
        uint64_t inc[Q];
#pragma unroll
        for (int q = 0; q < Q; q++) {
            uint64_t x = v[q];
#pragma unroll
            for (int d = 1; d < ASJ_WAVE; d <<= 1) {
                const uint64_t y = __shfl_up(x, d, ASJ_WAVE);
                if (lane >= d) x += y;
            }
            inc[q] = x;
            if (lane == ASJ_WAVE - 1) wtot[q][wave] = x;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; q++)
            for (int w = 0; w < wave; w++) inc[q] += wtot[q][w];
        if (j < J) {
            desc[j].tbase = carry[0] + inc[0] - v[0];
            desc[j].mask = v[0] - 1; // ~0 for an LDS table
            desc[j].wbase_r = (int64_t)(carry[1] + inc[1] - v[1]);
            desc[j].wbase = (int64_t)(carry[2] + inc[2] - v[2]);
            desc[j].wbase_l = (int64_t)(carry[3] + inc[3] - v[3]);
            desc[j].rbase = Q > 4 ? (int64_t)(carry[Q > 4 ? 4 : 0] + inc[Q > 4 ? 4 : 0] - v[4]) : 0;
            rows_done[j] = 0;
            out_count[j] = 0;
            if (cand_count) cand_count[j] = 0;
            if (done_clock) done_clock[j] = (s_seg[j + 1] <= s_seg[j]) ? start : 0;
        }
        __syncthreads(); // every thread has read carry and the wave totals
        if (tid < Q) {
            uint64_t t = 0;
            for (int w = 0; w < kWaves; w++) t += wtot[tid][w];
            carry[tid] += t;
        }
        __syncthreads();
    }
    if constexpr (Q > 4) {
        // (carry is final: its last update was followed by a barrier)
        if (rcnt && carry[4] > (uint64_t)rcnt_cap) bad = 1; // (only with more slots than slot_cap as well)
        __syncthreads();
    }
    if (tid < Q) tot[tid] = bad ? 0 : carry[tid];
    if (Q == 4 && tid == 4) tot[4] = 0; // no table regions
    if (Q > 4 && rcnt && !bad) { // region counts and the overflow count of a build by regions
        for (uint64_t i = tid; i < carry[Q > 4 ? 4 : 0]; i += kPlanBlock) rcnt[i] = 0u;
        if (tid == 0) *novf = 0;
    }
    if (tid == 0) {
        if (done_clock) done_clock[J] = start;
        *status = (bad || carry[0] > (uint64_t)slot_cap) ? (int32_t)ASJ_EINVAL : (int32_t)ASJ_OK;
    }
}

// The preparation (asj_batch_prep_run) when the build side has no key to
// sign (otherwise the signature kernel does it).
__global__ void batch_prep_kernel(asj_batch_prep p)
{
    asj_batch_prep_run(p, blockIdx.x, gridDim.x, threadIdx.x, blockDim.x);
}

int grid_for(int64_t n, int block, int cap)
{
    int64_t g = (n + block - 1) / block;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (int)g;
}

} // namespace

hipError_t asj_launch_batch_plan(const int64_t *r_seg, const int64_t *s_seg, int32_t njoins, int64_t n_r, int64_t n_s,
                                 int64_t slot_cap, float load_factor, int keys_per_window, int64_t local_rows,
                                 int local_only, asj_join_desc *desc, int64_t *rows_done, int64_t *out_count, int64_t *cand_count,
                                 uint64_t *done_clock, uint64_t *tot, int32_t *status, uint32_t *rcnt,
                                 int64_t rcnt_cap, uint64_t *novf, hipStream_t st)
{
    if (keys_per_window < 1 || keys_per_window > ASJ_WAVE) return hipErrorInvalidValue;
    if (rcnt && !novf) return hipErrorInvalidValue;
    if (local_only) // every join gets an LDS table: no table regions to number
        hipLaunchKernelGGL(batch_plan_kernel<4>, dim3(1), dim3(kPlanBlock), 0, st, r_seg, s_seg, njoins, n_r, n_s,
                           slot_cap, load_factor, keys_per_window, local_rows, local_only, desc, rows_done, out_count,
                           cand_count, done_clock, tot, status, (uint32_t *)nullptr, (int64_t)0, (uint64_t *)nullptr);
    else
        hipLaunchKernelGGL(batch_plan_kernel<5>, dim3(1), dim3(kPlanBlock), 0, st, r_seg, s_seg, njoins, n_r, n_s,
                           slot_cap, load_factor, keys_per_window, local_rows, local_only, desc, rows_done, out_count,
                           cand_count, done_clock, tot, status, rcnt, rcnt_cap, novf);
    return hipGetLastError();
}

hipError_t asj_launch_batch_prep(const asj_batch_prep *p, hipStream_t st)
{
    if (p->kpw < 1) return hipErrorInvalidValue;
    const int g = grid_for(p->njoins * 256LL, 256, 2048); // a block per join, bounded
    hipLaunchKernelGGL(batch_prep_kernel, dim3(g), dim3(256), 0, st, *p);
    return hipGetLastError();
}

