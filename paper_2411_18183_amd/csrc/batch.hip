// Many independent joins per launch sequence: every join j gets its own
// segment of one slot array (Build(R_j, H_sign) of Section 3.2, Figure 2),
// sized on the device so that no host round trip is needed; the probe side
// of all joins then runs through the fused probe kernel in one launch.
// Joins with few build rows (local_rows > 0 and |R_j| <= local_rows) get no
// segment: the blocks that probe them build their table in LDS from the
// build signatures, and their probe windows are numbered apart.
//
// Rows are handled in windows that never span two joins (64 build rows per
// insert window, keys_per_window probe rows per probe window), so every
// window knows its join from one map entry instead of a search over the
// segment bounds, and all of a window's bookkeeping goes to one join.
#include "asj_internal.h"

namespace {

constexpr int kPlanBlock = 1024;

// One block: segment capacities, window counts (build, probe and
// LDS-table probe windows) and their prefix sums, counters zeroed, batch
// start clock.  Segment arrays that do not cover the
// relations exactly (first bound 0, last bound the row count, no bound
// decreasing), segments that would not fit slot_cap slots, or (local_only)
// a join too large for an LDS table, set *status to ASJ_EINVAL so that no
// later kernel of the batch touches the slots or reads a key.
__global__ __launch_bounds__(kPlanBlock) void batch_plan_kernel(const int64_t *__restrict__ r_seg,
                                                                const int64_t *__restrict__ s_seg, int32_t J,
                                                                int64_t n_r, int64_t n_s, int64_t slot_cap, float lf,
                                                                int kpw, int64_t local_rows, int local_only,
                                                                asj_join_desc *__restrict__ desc,
                                                                int64_t *__restrict__ rows_done,
                                                                int64_t *__restrict__ out_count,
                                                                int64_t *__restrict__ cand_count,
                                                                uint64_t *__restrict__ done_clock,
                                                                uint64_t *__restrict__ tot, int32_t *__restrict__ status)
{
    constexpr int Q = 4; // scanned quantities
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
        uint64_t v[Q] = {0, 0, 0, 0};
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
    if (tid < Q) tot[tid] = bad ? 0 : carry[tid];
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

// Lane l of build window w inserts row r_seg[j] + 64 (w - wbase_r) + l of
// join j = win_r[w] into the join's segment, in the two passes of the
// single-join build (table.hip): STORE = 1 stores every row into its home
// slot, STORE = 0 moves the rows that lost their home slot to the first
// empty slot after it with CAS.
template <int STORE>
__global__ void insert_batch_kernel(const uint32_t *__restrict__ sig, int64_t m, const int64_t *__restrict__ r_seg,
                                    const asj_join_desc *__restrict__ desc, const int32_t *__restrict__ win_r,
                                    const uint64_t *__restrict__ tot, int64_t win_cap, uint64_t *__restrict__ slots,
                                    int32_t *__restrict__ status)
{
    if (*status != ASJ_OK) return; // same value for every thread
    const int64_t nw = min(win_cap, (int64_t)tot[1]);
    const int lane = threadIdx.x % ASJ_WAVE;
    const int wpb = blockDim.x / ASJ_WAVE;
    // a window of 64 build rows is one wave's work, so its join, segment
    // and table descriptor are wave-uniform values
    for (int64_t w = (int64_t)blockIdx.x * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x / ASJ_WAVE); w < nw;
         w += (int64_t)gridDim.x * wpb) {
        const int j = __builtin_amdgcn_readfirstlane(win_r[w]);
        const int64_t lo = r_seg[j], hi = min(r_seg[j + 1], m);
        const uint64_t tbase = desc[j].tbase, mask = desc[j].mask;
        const int64_t g = lo + (w - desc[j].wbase_r) * ASJ_WAVE + lane;
        if (g < lo || g >= hi) continue;
        const uint32_t sg = sig[g];
        const uint64_t val = ((uint64_t)sg << 32) | (uint32_t)g;
        uint64_t h = asj_mix32(sg) & mask;
        if (STORE) {
            slots[tbase + h] = val;
            continue;
        }
        if (slots[tbase + h] == val) continue;
        uint64_t tries = 0;
        for (;;) {
            h = (h + 1) & mask;
            if (++tries > mask) {
                atomicExch(status, (int32_t)ASJ_ETABLEFULL);
                break;
            }
            const uint64_t old = atomicCAS((unsigned long long *)&slots[tbase + h],
                                           (unsigned long long)ASJ_EMPTY_SLOT, (unsigned long long)val);
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

hipError_t asj_launch_batch_plan(const int64_t *r_seg, const int64_t *s_seg, int32_t njoins, int64_t n_r, int64_t n_s,
                                 int64_t slot_cap, float load_factor, int keys_per_window, int64_t local_rows,
                                 int local_only, asj_join_desc *desc, int64_t *rows_done, int64_t *out_count, int64_t *cand_count,
                                 uint64_t *done_clock, uint64_t *tot, int32_t *status, hipStream_t st)
{
    if (keys_per_window < 1 || keys_per_window > ASJ_WAVE) return hipErrorInvalidValue;
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(kPlanBlock), 0, st, r_seg, s_seg, njoins, n_r, n_s, slot_cap,
                       load_factor, keys_per_window, local_rows, local_only, desc, rows_done, out_count, cand_count,
                       done_clock, tot, status);
    return hipGetLastError();
}

hipError_t asj_launch_batch_prep(const asj_batch_prep *p, hipStream_t st)
{
    if (p->kpw < 1) return hipErrorInvalidValue;
    // a bounded grid: the fill loop strides, and a batch whose joins all
    // have LDS tables fills nothing
    const int64_t work = p->slot_cap > p->njoins * 256LL ? p->slot_cap : p->njoins * 256LL;
    const int g = grid_for(work, 256, 2048);
    hipLaunchKernelGGL(batch_prep_kernel, dim3(g), dim3(256), 0, st, *p);
    return hipGetLastError();
}

hipError_t asj_launch_insert_batch(const uint32_t *sig, int64_t m, const int64_t *r_seg, const asj_join_desc *desc,
                                   const int32_t *win_r, const uint64_t *tot, int64_t win_r_cap, uint64_t *slots,
                                   int32_t *status, hipStream_t st)
{
    if (m <= 0 || win_r_cap <= 0) return hipSuccess;
    // bounded grid (the window loop strides): a batch whose joins all have
    // LDS tables inserts nothing
    const dim3 g(grid_for(win_r_cap * ASJ_WAVE, 256, 2048)), b(256);
    hipLaunchKernelGGL(insert_batch_kernel<1>, g, b, 0, st, sig, m, r_seg, desc, win_r, tot, win_r_cap, slots, status);
    hipLaunchKernelGGL(insert_batch_kernel<0>, g, b, 0, st, sig, m, r_seg, desc, win_r, tot, win_r_cap, slots, status);
    return hipGetLastError();
}
