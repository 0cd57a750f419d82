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
//
// A single table of 327680 rows or more and at most 2^25 slots is built by
// regions instead (same layout, same probing).  Each row's (signature, row)
// word is first scattered into the slots of the region of its home slot
// (regions of 4096 slots; of 512 to 2048 in tables under 2^22 slots, so that
// there are 1024), which hold that region's rows until it is built; one
// block then reads a region's rows, places them in LDS with LDS CAS and
// writes the region out whole, empty slots included, so the table needs no
// fill.  The few rows whose run leaves their region, or that find its slots
// all claimed by the partition, are placed afterwards in device memory with
// CAS from their home slot.  Every table line is then written in order and
// whole, instead of taking one random store and one random read per row.
// Batches (segments sized on the device), smaller tables and the host-memory
// join keep the two passes.
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
__global__ void table_init_kernel(uint64_t *__restrict__ slots, int64_t cap, int32_t *__restrict__ status,
                                  int64_t *__restrict__ z0, int64_t *__restrict__ z1)
{
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) {
        *status = ASJ_OK;
        if (z0) *z0 = 0;
        if (z1) *z1 = 0;
    }
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
__global__ void local_init_kernel(int64_t *__restrict__ a, int64_t *__restrict__ b, int64_t *__restrict__ c,
                                  int32_t *__restrict__ status, uint32_t *__restrict__ words, int64_t nwords)
{
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) {
        *a = 0;
        if (b) *b = 0;
        if (c) *c = 0;
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

constexpr int kRegionBits = 12;   // slots per region, at most: 4096 (32 KB of LDS)
constexpr int kRegionMinBits = 8; // slots per region, at least (tables of 256 slots and more)
// Build rows from which the region build is used: below, its three short
// launches cost more than the two-pass insert's random accesses (measured
// crossover near 300000 rows at load factors 0.25 and 0.5).
constexpr int64_t kRegionMinRows = 327680;
constexpr int kRegionMax = 8192;  // regions per table (the LDS histogram of the partition)
constexpr int kPartBlock = 1024;  // threads of the partition kernel
constexpr int kPartRows = 4096;   // rows per partition block
constexpr int kRegionBlock = 256; // threads of the region-build kernel
constexpr int kRegionPer = (1 << kRegionBits) / kRegionBlock; // rows per thread, at most

__device__ __forceinline__ uint32_t region_of(uint32_t sg, uint64_t mask, int rbits)
{
    return (uint32_t)((asj_mix32(sg) & mask) >> rbits);
}

// Every row's word (signature << 32 | row) into the slots of its home region,
// which serve as that region's bucket until the region is built: a block
// counts its rows per region in LDS, reserves each region's share with one
// atomic, and ranks its rows within the shares in LDS.  A region's rows
// beyond its slot count go straight to the overflow list.
__global__ __launch_bounds__(kPartBlock) void region_scatter_kernel(const uint32_t *__restrict__ sig, int64_t m,
                                                                    uint64_t mask, int rbits, int nreg,
                                                                    uint32_t *__restrict__ cnt,
                                                                    uint64_t *__restrict__ slots,
                                                                    uint64_t *__restrict__ ovf,
                                                                    uint32_t *__restrict__ novf,
                                                                    const int32_t *__restrict__ status)
{
    if (*status != ASJ_OK) return;
    constexpr int kPer = kPartRows / kPartBlock;
    __shared__ uint32_t h[kRegionMax];
    const int64_t r0 = (int64_t)blockIdx.x * kPartRows + threadIdx.x;
    uint32_t sg[kPer], q[kPer];
#pragma unroll
    for (int k = 0; k < kPer; k++) {
        const int64_t r = r0 + k * kPartBlock;
        sg[k] = r < m ? sig[r] : 0u;
    }
    for (int i = threadIdx.x; i < nreg; i += kPartBlock) h[i] = 0u;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; k++) {
        q[k] = region_of(sg[k], mask, rbits);
        if (r0 + k * kPartBlock < m) atomicAdd(&h[q[k]], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nreg; i += kPartBlock)
        if (h[i]) h[i] = atomicAdd(&cnt[i], h[i]); // this block's first position in region i
    __syncthreads();
    const uint32_t Z = 1u << rbits;
#pragma unroll
    for (int k = 0; k < kPer; k++) {
        const int64_t r = r0 + k * kPartBlock;
        if (r >= m) break;
        const uint32_t pos = atomicAdd(&h[q[k]], 1u);
        const uint64_t e = ((uint64_t)sg[k] << 32) | (uint32_t)r;
        if (pos < Z) slots[((uint64_t)q[k] << rbits) + pos] = e;
        else ovf[atomicAdd(novf, 1u)] = e;
    }
}

// The build rows of a batch into the slots of their home region, each
// region of a join's segment holding 2^asj_seg_region_bits slots.  A block
// takes 64 consecutive build windows (64 rows of one join each, so 4096 rows
// of one or more joins, whose regions are numbered consecutively): it counts
// its rows per region in LDS, reserves each region's share with one device
// atomic, and ranks its rows within the shares in LDS.  Regions more than
// kRegionMax past the block's first one (windows of several joins with very
// large segments) take one device atomic per row instead.
constexpr int kScatterWins = kPartRows / ASJ_WAVE; // build windows per block

__global__ __launch_bounds__(kPartBlock) void region_scatter_batch_kernel(
    const uint32_t *__restrict__ sig, int64_t m, const int64_t *__restrict__ r_seg,
    const asj_join_desc *__restrict__ desc, const int32_t *__restrict__ win_r, const uint64_t *__restrict__ tot,
    int64_t win_cap, uint32_t *__restrict__ rcnt, uint64_t *__restrict__ slots, uint64_t *__restrict__ ovf,
    uint32_t *__restrict__ novf, const int32_t *__restrict__ status)
{
    if (*status != ASJ_OK) return; // same value for every thread
    constexpr int kPer = kScatterWins / (kPartBlock / ASJ_WAVE); // windows per wave
    __shared__ uint32_t h[kRegionMax];
    const int64_t nw = min(win_cap, (int64_t)tot[1]);
    const int64_t w0 = (int64_t)blockIdx.x * kScatterWins;
    if (w0 >= nw) return; // block-uniform
    const int64_t rlo = desc[win_r[w0]].rbase;
    const int lane = threadIdx.x % ASJ_WAVE, wave = threadIdx.x / ASJ_WAVE;
    int64_t reg[kPer];   // the row's region, or -1
    uint64_t e[kPer];    // its word (signature << 32 | row)
    uint64_t sbase[kPer]; // first slot of its region
    uint32_t Zk[kPer];
#pragma unroll
    for (int k = 0; k < kPer; k++) {
        reg[k] = -1;
        const int64_t w = w0 + wave * kPer + k;
        if (w >= nw) continue;
        const int j = __builtin_amdgcn_readfirstlane(win_r[w]);
        const int64_t lo = r_seg[j], hi = min(r_seg[j + 1], m);
        const asj_join_desc d = desc[j];
        const int64_t g = lo + (w - d.wbase_r) * ASJ_WAVE + lane;
        if (g < lo || g >= hi) continue;
        const uint32_t sg = sig[g];
        const int rb = asj_seg_region_bits(d.mask + 1);
        const uint64_t q = (asj_mix32(sg) & d.mask) >> rb;
        reg[k] = d.rbase + (int64_t)q;
        e[k] = ((uint64_t)sg << 32) | (uint32_t)g;
        sbase[k] = d.tbase + (q << rb);
        Zk[k] = 1u << rb;
    }
    for (int i = threadIdx.x; i < kRegionMax; i += kPartBlock) h[i] = 0u;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; k++)
        if (reg[k] >= 0 && reg[k] - rlo < kRegionMax) atomicAdd(&h[reg[k] - rlo], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < kRegionMax; i += kPartBlock)
        if (h[i]) h[i] = atomicAdd(&rcnt[rlo + i], h[i]); // this block's first position in region rlo + i
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; k++) {
        if (reg[k] < 0) continue;
        const uint32_t pos = reg[k] - rlo < kRegionMax ? atomicAdd(&h[reg[k] - rlo], 1u) : atomicAdd(&rcnt[reg[k]], 1u);
        if (pos < Zk[k]) slots[sbase[k] + pos] = e[k];
        else ovf[atomicAdd(novf, 1u)] = e[k];
    }
}

// Region r's rows (the first min(cnt[r], its slot count) words of its
// slots) placed by linear probing in LDS with CAS, then the region written
// out whole, empty slots included; a row that finds every slot from its home
// to the region's end taken goes to the overflow list.  A single table: the
// regions of 2^rbits slots of slots[0 .. nreg << rbits); a batch (BATCH):
// region r of the join rmap[r], the regions of each segment numbered from
// the join's rbase.
template <int BATCH>
__global__ __launch_bounds__(kRegionBlock) void region_build_kernel(const uint32_t *__restrict__ cnt, int64_t nreg,
                                                                    int rbits, uint64_t mask, int plain,
                                                                    const uint64_t *__restrict__ tot,
                                                                    const int32_t *__restrict__ rmap,
                                                                    const asj_join_desc *__restrict__ desc,
                                                                    uint64_t *__restrict__ slots,
                                                                    uint64_t *__restrict__ ovf,
                                                                    uint32_t *__restrict__ novf,
                                                                    const int32_t *__restrict__ status)
{
    // A single table whose validation failed still gets every region
    // written (empty), so that it is defined whatever its status; a batch
    // whose plan or validation failed is left alone (its probe does nothing).
    const bool ok = *status == ASJ_OK;
    if (BATCH) {
        if (!ok) return;
        nreg = min(nreg, (int64_t)tot[4]);
    }
    __shared__ unsigned long long tab[1 << kRegionBits];
    for (int64_t r = blockIdx.x; r < nreg; r += gridDim.x) { // block-uniform
        uint64_t tb = 0, q = (uint64_t)r;
        if (BATCH) {
            const asj_join_desc d = desc[rmap[r]];
            tb = d.tbase;
            mask = d.mask;
            rbits = asj_seg_region_bits(d.mask + 1);
            q = (uint64_t)(r - d.rbase);
        }
        const uint32_t Z = 1u << rbits;
        const uint64_t home0 = q << rbits; // the region's first slot within its table
        const uint64_t base = tb + home0;
        const uint32_t c = ok ? min(cnt[r], Z) : 0u;
        uint64_t e[kRegionPer];
#pragma unroll
        for (int k = 0; k < kRegionPer; k++) {
            const uint32_t i = threadIdx.x + k * kRegionBlock;
            e[k] = i < c ? slots[base + i] : 0ull;
        }
        for (uint32_t i = threadIdx.x; i < Z; i += kRegionBlock) tab[i] = ASJ_EMPTY_SLOT;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kRegionPer; k++) {
            if (threadIdx.x + k * kRegionBlock >= c) break;
            const uint32_t sg = (uint32_t)(e[k] >> 32);
            const unsigned long long val = plain ? (unsigned long long)(uint32_t)e[k] : (unsigned long long)e[k];
            uint32_t h = (uint32_t)((asj_mix32(sg) & mask) - home0);
            while (h < Z && atomicCAS(&tab[h], (unsigned long long)ASJ_EMPTY_SLOT, val) != ASJ_EMPTY_SLOT) h++;
            if (h == Z) ovf[atomicAdd(novf, 1u)] = e[k];
        }
        __syncthreads(); // every row read and placed
        for (uint32_t i = threadIdx.x; i < Z; i += kRegionBlock) slots[base + i] = tab[i];
        __syncthreads(); // the next region reuses tab
    }
}

// The overflow rows, once every region is written: linear probing with CAS
// in device memory from the home slot, wrapping at the table's (segment's)
// end.  A row moved here by the partition (its region had more rows than
// slots) never saw its region, which may still hold empty slots after its
// home.  A batch finds each row's join from the build segments.
template <int BATCH>
__global__ void region_overflow_kernel(const uint64_t *__restrict__ ovf, const uint32_t *__restrict__ novf,
                                       uint64_t mask, int plain, const int64_t *__restrict__ r_seg, int32_t njoins,
                                       const asj_join_desc *__restrict__ desc, uint64_t *__restrict__ slots,
                                       int32_t *__restrict__ status)
{
    if (*status != ASJ_OK) return; // a failed plan or validation leaves the overflow count unset
    const uint32_t n = *novf;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint64_t e = ovf[i];
        const uint32_t sg = (uint32_t)(e >> 32);
        const unsigned long long val = plain ? (unsigned long long)(uint32_t)e : (unsigned long long)e;
        uint64_t tb = 0;
        if (BATCH) { // the last join whose rows start at or before row g: the one holding g
            const int64_t g = (int64_t)(uint32_t)e;
            int lo = 0, hi = njoins - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) / 2;
                if (r_seg[mid] <= g) lo = mid;
                else hi = mid - 1;
            }
            tb = desc[lo].tbase;
            mask = desc[lo].mask;
        }
        const uint64_t home = asj_mix32(sg) & mask;
        bool placed = false;
        for (uint64_t t = 0; t <= mask && !placed; t++) // every slot of the table once
            placed = atomicCAS((unsigned long long *)&slots[tb + ((home + t) & mask)],
                               (unsigned long long)ASJ_EMPTY_SLOT, val) == ASJ_EMPTY_SLOT;
        if (!placed) atomicExch(status, (int32_t)ASJ_ETABLEFULL);
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

hipError_t asj_launch_table_init(uint64_t *slots, int64_t cap, int32_t *status, hipStream_t st, int64_t *z0,
                                 int64_t *z1)
{
    hipLaunchKernelGGL(table_init_kernel, dim3(grid_for(cap > 0 ? cap : 1, 256, 16384)), dim3(256), 0, st, slots, cap,
                       status, z0, z1);
    return hipGetLastError();
}

hipError_t asj_launch_local_init(int64_t *a, int64_t *b, int32_t *status, uint32_t *words, int64_t nwords,
                                 hipStream_t st, int64_t *c)
{
    const int g = grid_for(nwords > 0 ? nwords : 1, 256, 4096);
    hipLaunchKernelGGL(local_init_kernel, dim3(g), dim3(256), 0, st, a, b, c, status, words, nwords);
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

namespace {
struct region_layout {
    int rbits, nreg;
    uint32_t *novf, *cnt;
    uint64_t *ovf;
    int64_t bytes;
};

// The scratch of a region build: overflow count | region counts (nreg
// words) | overflow list (m words).
bool region_plan(int64_t m, int64_t cap, uint8_t *p, region_layout *L)
{
    if (cap < 64 || (cap & (cap - 1)) || m < kRegionMinRows || m >= ((int64_t)1 << 31)) return false;
    // regions of 4096 slots, smaller for tables under 2^22 slots (at least
    // 1024 regions then, each of at least 256 slots or the whole table)
    const int lg = __builtin_ctzll((unsigned long long)cap);
    L->rbits = std::max(std::min(lg - 10, kRegionBits), std::min(lg, kRegionMinBits));
    const int64_t nreg = cap >> L->rbits;
    if (nreg > kRegionMax) return false;
    L->nreg = (int)nreg;
    const int64_t o_ovf = 256 + ((4 * nreg + 255) & ~(int64_t)255);
    L->bytes = o_ovf + 8 * (m > 0 ? m : 1);
    L->novf = (uint32_t *)p;
    L->cnt = (uint32_t *)(p + 256);
    L->ovf = (uint64_t *)(p + o_ovf);
    return true;
}

int region_grid(int nreg) { return std::min(nreg, 2048); }
} // namespace

int64_t asj_region_scratch_bytes(int64_t m, int64_t cap)
{
    region_layout L;
    return region_plan(m, cap, nullptr, &L) ? L.bytes : -1;
}

hipError_t asj_launch_region_init(void *scratch, int64_t m, int64_t cap, int32_t *status, hipStream_t st,
                                  int64_t *z0, int64_t *z1)
{
    region_layout L;
    if (!scratch || !region_plan(m, cap, (uint8_t *)scratch, &L)) return hipErrorInvalidValue;
    return asj_launch_local_init((int64_t *)L.novf, z0, status, L.cnt, L.nreg, st, z1);
}

hipError_t asj_launch_region_build(const uint32_t *sig, int64_t m, int plain, uint64_t *slots, int64_t cap,
                                   int32_t *status, void *scratch, hipStream_t st)
{
    region_layout L;
    if (!scratch || !region_plan(m, cap, (uint8_t *)scratch, &L)) return hipErrorInvalidValue;
    const uint64_t mask = (uint64_t)cap - 1;
    const int pb = (int)((m + kPartRows - 1) / kPartRows);
    if (pb > 0)
        hipLaunchKernelGGL(region_scatter_kernel, dim3(pb), dim3(kPartBlock), 0, st, sig, m, mask, L.rbits, L.nreg,
                           L.cnt, slots, L.ovf, L.novf, (const int32_t *)status);
    hipLaunchKernelGGL(region_build_kernel<0>, dim3(region_grid(L.nreg)), dim3(kRegionBlock), 0, st,
                       (const uint32_t *)L.cnt, (int64_t)L.nreg, L.rbits, mask, plain, (const uint64_t *)nullptr,
                       (const int32_t *)nullptr, (const asj_join_desc *)nullptr, slots, L.ovf, L.novf,
                       (const int32_t *)status);
    if (pb > 0)
        hipLaunchKernelGGL(region_overflow_kernel<0>, dim3(64), dim3(256), 0, st, (const uint64_t *)L.ovf,
                           (const uint32_t *)L.novf, mask, plain, (const int64_t *)nullptr, 0,
                           (const asj_join_desc *)nullptr, slots, status);
    return hipGetLastError();
}

hipError_t asj_launch_region_build_batch(const uint32_t *sig, int64_t m, const int64_t *r_seg, int32_t njoins,
                                         const asj_join_desc *desc, const int32_t *win_r, const uint64_t *tot,
                                         int64_t win_r_cap, const int32_t *rmap, int64_t rmap_cap, uint32_t *rcnt,
                                         uint64_t *ovf, uint64_t *novf, uint64_t *slots, int32_t *status,
                                         hipStream_t st)
{
    if (njoins < 1 || rmap_cap < 1 || !rmap || !rcnt || !ovf || !novf) return hipErrorInvalidValue;
    uint32_t *nov = (uint32_t *)novf;
    if (m > 0 && win_r_cap > 0) // a block per 64 build windows that may exist (the rest exit at once)
        hipLaunchKernelGGL(region_scatter_batch_kernel, dim3((unsigned)((win_r_cap + kScatterWins - 1) / kScatterWins)),
                           dim3(kPartBlock), 0, st, sig, m, r_seg, desc, win_r, tot, win_r_cap, rcnt, slots, ovf, nov,
                           (const int32_t *)status);
    // every region, rows or not: the segments get no other fill
    hipLaunchKernelGGL(region_build_kernel<1>, dim3((unsigned)std::min<int64_t>(rmap_cap, 2048)), dim3(kRegionBlock),
                       0, st, (const uint32_t *)rcnt, rmap_cap, 0, (uint64_t)0, 0, tot, rmap, desc, slots, ovf, nov,
                       (const int32_t *)status);
    if (m > 0)
        hipLaunchKernelGGL(region_overflow_kernel<1>, dim3(64), dim3(256), 0, st, (const uint64_t *)ovf,
                           (const uint32_t *)nov, (uint64_t)0, 0, r_seg, njoins, desc, slots, status);
    return hipGetLastError();
}
