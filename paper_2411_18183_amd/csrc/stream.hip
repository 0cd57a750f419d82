// Joins of relations held in host memory (asj_join_host).
//
// One partition: the simple hash join of Section 2 / Figure 2 with the build
// side copied to the device whole and the probe side streamed through it in
// pieces, two pieces in flight on two streams.
//
// More partitions: the Grace hash join of Section 2.  A partitioning pass
// streams each relation through the device in chunks; a chunk is signed
// (Section 3.1) and its keys are moved, with their ids and signatures, into
// groups by the top bits of mix32(signature), so that equal keys -- and keys
// of equal signature -- always share a partition.  The grouped chunk goes back
// to pinned host memory.  Then each build partition R_p is copied in and
// inserted from its stored signatures, and the pieces of S_p are probed
// against it with the stored signatures, so no key is signed twice.  The
// table slot uses the low bits of the same mix32 value, which the partition
// bits leave uniformly distributed.
//
// Device memory is taken only through a budget: every buffer is counted, and
// the partition count is raised until the largest build partition and its
// table fit half of it.
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <vector>

#include "asj_internal.h"

namespace {

constexpr int kMaxLogP = 10;                // at most 1024 partitions
constexpr int64_t kMaxChunkKeys = 1 << 22;  // keys per partitioning chunk (packed key counts use 24 bits)
constexpr int kByteBits = 40;               // per-partition counters: keys << 40 | bytes
constexpr unsigned long long kByteMask = (1ull << kByteBits) - 1;
constexpr int kGridCap = 256 * 16;
constexpr int64_t kMaxPieceBytes = 128ll << 20; // probe piece input (keys + 16 bytes per key)
constexpr int64_t kPerKeyBytes = 24;        // device bytes per key beside its key bytes (offset, id, signature, move)

size_t al(size_t x) { return ((x ? x : 1) + 255) & ~(size_t)255; }

int grid_for(int64_t n, int block)
{
    int64_t g = (n + block - 1) / block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, kGridCap));
}

__device__ inline uint32_t part_of(uint32_t sig, int logp)
{
    return logp ? asj_mix32(sig) >> (32 - logp) : 0u;
}

__global__ void rebase_kernel(int64_t *__restrict__ off, int64_t n, int64_t add)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        off[i] += add;
}

__global__ void iota_kernel(int32_t *__restrict__ ids, int64_t n, int64_t base)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        ids[i] = (int32_t)(base + i);
}

// Keys and bytes of every partition in a chunk (block histograms in LDS,
// one global add per block and partition).
__global__ __launch_bounds__(256) void part_hist_kernel(const uint32_t *__restrict__ sig,
                                                        const int64_t *__restrict__ off, int64_t n, int logp,
                                                        unsigned long long *__restrict__ cnt)
{
    __shared__ unsigned long long h[1 << kMaxLogP];
    const int P = 1 << logp;
    for (int i = threadIdx.x; i < P; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long len = (unsigned long long)(off[k + 1] - off[k]);
        atomicAdd(&h[part_of(sig[k], logp)], (1ull << kByteBits) + len);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < P; i += blockDim.x)
        if (h[i]) atomicAdd(&cnt[i], h[i]);
}

// Exclusive prefix over the partitions: partition p of the grouped chunk
// starts at key info[4p] and byte info[4p + 2] and holds info[4p + 1] keys
// and info[4p + 3] bytes; cursor[p] = first key << 40 | first byte; the
// grouped offsets end at out_off[n] = all bytes.
__global__ __launch_bounds__(1024) void part_scan_kernel(const unsigned long long *__restrict__ cnt, int logp,
                                                         unsigned long long *__restrict__ cursor,
                                                         int64_t *__restrict__ info, int64_t *__restrict__ out_off,
                                                         int64_t n)
{
    __shared__ unsigned long long c[1 << kMaxLogP], base[1 << kMaxLogP];
    const int P = 1 << logp;
    for (int i = threadIdx.x; i < P; i += blockDim.x) c[i] = cnt[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long run = 0; // keys << 40 | bytes, summed field by field
        for (int p = 0; p < P; p++) {
            base[p] = run;
            run += c[p];
        }
        out_off[n] = (int64_t)(run & kByteMask);
    }
    __syncthreads();
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
        cursor[p] = base[p];
        info[4 * p + 0] = (int64_t)(base[p] >> kByteBits);
        info[4 * p + 1] = (int64_t)(c[p] >> kByteBits);
        info[4 * p + 2] = (int64_t)(base[p] & kByteMask);
        info[4 * p + 3] = (int64_t)(c[p] & kByteMask);
    }
}

// Places every key of the chunk in its partition: a key's position (key
// index and byte offset in the grouped chunk) is its block's reservation in
// the partition plus its rank inside the block, both taken with packed adds
// so that key order and byte order agree.  Writes the grouped offsets, ids
// and signatures, and for the move kernel the key's new byte offset.
__global__ __launch_bounds__(256) void part_scatter_kernel(const uint32_t *__restrict__ sig,
                                                           const int64_t *__restrict__ off,
                                                           const int32_t *__restrict__ ids, int64_t n, int logp,
                                                           unsigned long long *__restrict__ cursor,
                                                           uint32_t *__restrict__ out_sig,
                                                           int32_t *__restrict__ out_ids,
                                                           int64_t *__restrict__ out_off, int64_t *__restrict__ dpos)
{
    __shared__ unsigned long long h[1 << kMaxLogP];
    const int P = 1 << logp;
    for (int i = threadIdx.x; i < P; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t sg = 0, p = 0;
    unsigned long long local = 0;
    if (k < n) {
        sg = sig[k];
        p = part_of(sg, logp);
        local = atomicAdd(&h[p], (1ull << kByteBits) + (unsigned long long)(off[k + 1] - off[k]));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < P; i += blockDim.x)
        if (h[i]) h[i] = atomicAdd(&cursor[i], h[i]);
    __syncthreads();
    if (k < n) {
        const unsigned long long pos = h[p] + local;
        const int64_t kd = (int64_t)(pos >> kByteBits), bd = (int64_t)(pos & kByteMask);
        out_sig[kd] = sg;
        out_ids[kd] = ids[k];
        out_off[kd] = bd;
        dpos[k] = bd;
    }
}

// Moves the key bytes to their grouped positions: one wave per key, one
// byte per lane and step (consecutive lanes, consecutive bytes).
__global__ __launch_bounds__(256) void part_move_kernel(const uint8_t *__restrict__ src,
                                                        const int64_t *__restrict__ off,
                                                        const int64_t *__restrict__ dpos, int64_t n,
                                                        uint8_t *__restrict__ dst)
{
    const int lane = threadIdx.x % ASJ_WAVE;
    const int64_t wpb = blockDim.x / ASJ_WAVE;
    for (int64_t k = (int64_t)blockIdx.x * wpb + threadIdx.x / ASJ_WAVE; k < n; k += (int64_t)gridDim.x * wpb) {
        const int64_t a = off[k], len = off[k + 1] - a, d = dpos[k];
        for (int64_t i = lane; i < len; i += ASJ_WAVE) dst[d + i] = src[a + i];
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// Rows of a relation in host memory: key k is bytes[off[k] - off_sub ..
// off[k + 1] - off_sub); its id is ids[k], or id_base + k without ids; sig
// holds its signature when it has been signed already.
struct HostRel {
    const uint8_t *bytes = nullptr;
    const int64_t *off = nullptr;
    int64_t off_sub = 0;
    const int32_t *ids = nullptr;
    int64_t id_base = 0;
    const uint32_t *sig = nullptr;
    int64_t n = 0;
};

// Device buffers for up to cap_keys keys and cap_bytes key bytes.
struct DevRel {
    uint8_t *bytes = nullptr;
    int64_t *off = nullptr;
    int32_t *ids = nullptr;
    uint32_t *sig = nullptr;
    int64_t cap_keys = 0, cap_bytes = 0;
};

size_t devrel_bytes(int64_t keys, int64_t bytes)
{
    return al((size_t)bytes + 16) + al(8 * (size_t)(keys + 1)) + 2 * al(4 * (size_t)keys);
}

struct Range {
    const HostRel *h;
    int64_t a, b;
};

// A grouped chunk in pinned host memory, with its partition table.
struct HostChunk {
    uint8_t *bytes = nullptr;
    int64_t *off = nullptr;
    int32_t *ids = nullptr;
    uint32_t *sig = nullptr;
    int64_t n = 0, nbytes = 0;
    int64_t *info = nullptr; // pinned, 4 per partition: first key, keys, first byte, bytes
    HostRel rel() const
    {
        HostRel h;
        h.bytes = bytes;
        h.off = off;
        h.ids = ids;
        h.sig = sig;
        h.n = n;
        return h;
    }
};

// The partitioned chunks of one relation, in one pinned host region: the
// library's cached region (kept for later calls, see asj_join_host_release)
// when no other call holds the cache, else a private one freed at the end.
struct HostStore {
    std::vector<HostChunk> chunks;
    uint8_t *arena = nullptr;
    size_t size = 0;
    int cache = -1; // index of the cached region in use, or -1 for a private one
};

std::mutex g_pin_mu; // held by the call that uses the cached regions
struct Pinned {
    uint8_t *p = nullptr;
    size_t size = 0;
};
Pinned g_pin[2];

struct Ctx {
    hipStream_t st = nullptr;
    int64_t budget = 0, used = 0;
    asj_host_stats stats = {};
    const uint16_t *tab = nullptr;
    asj_resolved ro = {};
    int mode = ASJ_MODE_SIG16, nsym = 2;
    bool cache = false; // this call holds g_pin_mu
    HostStore store_r, store_s;
};

int from_hip(hipError_t e)
{
    if (e == hipSuccess) return ASJ_OK;
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? ASJ_ENOMEM : ASJ_EHIP;
}

// Device allocation counted against the budget.
int dalloc(Ctx &c, void **p, size_t bytes)
{
    *p = nullptr;
    bytes = al(bytes);
    if (c.used + (int64_t)bytes > c.budget) return ASJ_ENOMEM;
    const int rc = from_hip(hipMalloc(p, bytes));
    if (rc != ASJ_OK) return rc;
    c.used += (int64_t)bytes;
    c.stats.device_peak = std::max(c.stats.device_peak, c.used);
    return ASJ_OK;
}

void dfree(Ctx &c, void *p, size_t bytes)
{
    if (!p) return;
    (void)hipFree(p);
    c.used -= (int64_t)al(bytes);
}

int alloc_rel(Ctx &c, DevRel &d, int64_t keys, int64_t bytes)
{
    d.cap_keys = keys;
    d.cap_bytes = bytes;
    int rc = dalloc(c, (void **)&d.bytes, (size_t)bytes + 16);
    if (rc == ASJ_OK) rc = dalloc(c, (void **)&d.off, 8 * (size_t)(keys + 1));
    if (rc == ASJ_OK) rc = dalloc(c, (void **)&d.ids, 4 * (size_t)keys);
    if (rc == ASJ_OK) rc = dalloc(c, (void **)&d.sig, 4 * (size_t)keys);
    return rc;
}

void free_rel(Ctx &c, DevRel &d)
{
    dfree(c, d.bytes, (size_t)d.cap_bytes + 16);
    dfree(c, d.off, 8 * (size_t)(d.cap_keys + 1));
    dfree(c, d.ids, 4 * (size_t)d.cap_keys);
    dfree(c, d.sig, 4 * (size_t)d.cap_keys);
    d = DevRel();
}

void free_store(HostStore &s)
{
    if (s.arena && s.cache < 0) (void)hipHostFree(s.arena);
    s = HostStore();
}

// A pinned region of at least `size` bytes for store s (which = 0 for the
// build relation, 1 for the probe relation).
int store_arena(Ctx &c, HostStore &s, int which, size_t size)
{
    if (s.arena && s.size >= size) return ASJ_OK;
    free_store(s);
    if (c.cache) {
        Pinned &g = g_pin[which];
        if (g.size < size) {
            if (g.p) (void)hipHostFree(g.p);
            g = Pinned();
            if (hipHostMalloc((void **)&g.p, size, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                return ASJ_ENOMEM;
            }
            g.size = size;
        }
        s.arena = g.p;
        s.size = g.size;
        s.cache = which;
        return ASJ_OK;
    }
    if (hipHostMalloc((void **)&s.arena, size, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        s.arena = nullptr;
        return ASJ_ENOMEM;
    }
    s.size = size;
    return ASJ_OK;
}

size_t chunk_host_bytes(int64_t keys, int64_t bytes, int P)
{
    return al((size_t)bytes + 16) + al(8 * (size_t)(keys + 1)) + 2 * al(4 * (size_t)keys + 4) + al(32 * (size_t)P);
}

int64_t rows_bytes(const HostRel &h, int64_t a, int64_t b) { return h.off[b] - h.off[a]; }

// Cuts rows [a, b) of h into ranges of at most max_keys keys whose key bytes
// plus per_key bytes per key stay within max_cost.  ASJ_ENOMEM when one key
// alone exceeds it.
int split_rows(const HostRel *h, int64_t a, int64_t b, int64_t max_keys, int64_t per_key, int64_t max_cost,
               std::vector<Range> &out)
{
    while (a < b) {
        // largest e in (a, min(b, a + max_keys)] with cost(a, e) <= max_cost; cost grows with e
        int64_t lo = a, hi = std::min(b, a + max_keys);
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo + 1) / 2;
            if (rows_bytes(*h, a, mid) + per_key * (mid - a) <= max_cost) lo = mid;
            else hi = mid - 1;
        }
        if (lo == a) return ASJ_ENOMEM;
        out.push_back(Range{h, a, lo});
        a = lo;
    }
    return ASJ_OK;
}

// Copies rows [a, b) of h into d at key kb and byte bb (offsets rebased to
// d's bytes; ids materialized; signatures when h has them).  Copies that
// follow one another on a stream concatenate: the closing offset of one
// range is the opening offset of the next.
int load_rows(Ctx &c, const HostRel &h, int64_t a, int64_t b, DevRel &d, int64_t kb, int64_t bb, hipStream_t st)
{
    const int64_t o0 = h.off[a], nb = h.off[b] - o0, nk = b - a;
    hipError_t e = hipSuccess;
    if (nb > 0) e = hipMemcpyAsync(d.bytes + bb, h.bytes + (o0 - h.off_sub), (size_t)nb, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d.off + kb, h.off + a, 8 * (size_t)(nk + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(rebase_kernel, dim3(grid_for(nk + 1, 256)), dim3(256), 0, st, d.off + kb, nk + 1, bb - o0);
        e = hipGetLastError();
    }
    c.stats.bytes_h2d += nb + 8 * (nk + 1);
    if (e == hipSuccess && nk > 0) {
        if (h.ids) {
            e = hipMemcpyAsync(d.ids + kb, h.ids + a, 4 * (size_t)nk, hipMemcpyHostToDevice, st);
            c.stats.bytes_h2d += 4 * nk;
        } else {
            hipLaunchKernelGGL(iota_kernel, dim3(grid_for(nk, 256)), dim3(256), 0, st, d.ids + kb, nk, h.id_base + a);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess && nk > 0 && h.sig) {
        e = hipMemcpyAsync(d.sig + kb, h.sig + a, 4 * (size_t)nk, hipMemcpyHostToDevice, st);
        c.stats.bytes_h2d += 4 * nk;
    }
    return from_hip(e);
}

hipError_t sign_rel(Ctx &c, const DevRel &d, int64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    asj_keys k = {d.bytes, d.off, d.ids, n};
    return asj_launch_sign(c.mode, c.nsym, &k, d.sig, c.tab, kGridCap, st);
}

// ---- partitioning pass ----
// Two lanes (stream + buffers) take alternate chunks, so that one chunk's
// grouped output goes back to the host while the next chunk comes in.  A
// chunk's host-to-device copies start once the previous chunk's have ended
// (in_done), so the two directions of the host link overlap instead of two
// chunks sharing one direction.
struct Lane {
    DevRel in, grp;
    int64_t *dpos = nullptr, *info = nullptr;
    unsigned long long *cnt = nullptr, *cursor = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    hipEvent_t in_done = nullptr; // the chunk's input is on the device
    bool busy = false;
};

int open_lane(Ctx &c, Lane &l, int64_t mk, int64_t mb, int P, hipEvent_t after)
{
    int rc = alloc_rel(c, l.in, mk, mb);
    if (rc == ASJ_OK) rc = alloc_rel(c, l.grp, mk, mb);
    if (rc == ASJ_OK) rc = dalloc(c, (void **)&l.dpos, 8 * (size_t)mk);
    if (rc == ASJ_OK) rc = dalloc(c, (void **)&l.cnt, 8 * (size_t)P);
    if (rc == ASJ_OK) rc = dalloc(c, (void **)&l.cursor, 8 * (size_t)P);
    if (rc == ASJ_OK) rc = dalloc(c, (void **)&l.info, 32 * (size_t)P);
    if (rc != ASJ_OK) return rc;
    hipError_t e = hipStreamCreateWithFlags(&l.st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&l.ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&l.in_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamWaitEvent(l.st, after, 0);
    return from_hip(e);
}

void close_lane(Ctx &c, Lane &l, int64_t mk, int P)
{
    if (l.st) (void)hipStreamSynchronize(l.st);
    free_rel(c, l.in);
    free_rel(c, l.grp);
    dfree(c, l.dpos, 8 * (size_t)mk);
    dfree(c, l.cnt, 8 * (size_t)P);
    dfree(c, l.cursor, 8 * (size_t)P);
    dfree(c, l.info, 32 * (size_t)P);
    if (l.ev) (void)hipEventDestroy(l.ev);
    if (l.in_done) (void)hipEventDestroy(l.in_done);
    if (l.st) (void)hipStreamDestroy(l.st);
    l = Lane();
}

// Signs and groups rows [a, b) of h on lane l and copies the grouped chunk
// into hc's pinned region; completion is l.ev.  The input copies wait for
// prev_in (the previous chunk's input copies, may be NULL).
int partition_chunk(Ctx &c, Lane &l, const HostRel &h, int64_t a, int64_t b, int logp, HostChunk &hc,
                    hipEvent_t prev_in)
{
    const int P = 1 << logp;
    const int64_t nk = b - a, nb = rows_bytes(h, a, b);
    if (prev_in) {
        const int rw = from_hip(hipStreamWaitEvent(l.st, prev_in, 0));
        if (rw != ASJ_OK) return rw;
    }
    int rc = load_rows(c, h, a, b, l.in, 0, 0, l.st);
    if (rc != ASJ_OK) return rc;
    hipError_t e = hipEventRecord(l.in_done, l.st);
    if (e == hipSuccess) e = sign_rel(c, l.in, nk, l.st);
    if (e == hipSuccess) e = asj_launch_fill_i64((int64_t *)l.cnt, P, 0, l.st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(part_hist_kernel, dim3(grid_for(nk, 256)), dim3(256), 0, l.st, l.in.sig, l.in.off, nk, logp,
                           l.cnt);
        hipLaunchKernelGGL(part_scan_kernel, dim3(1), dim3(1024), 0, l.st, l.cnt, logp, l.cursor, l.info, l.grp.off,
                           nk);
        hipLaunchKernelGGL(part_scatter_kernel, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, l.st, l.in.sig,
                           l.in.off, l.in.ids, nk, logp, l.cursor, l.grp.sig, l.grp.ids, l.grp.off, l.dpos);
        hipLaunchKernelGGL(part_move_kernel, dim3(grid_for(nk, 4)), dim3(256), 0, l.st, l.in.bytes, l.in.off, l.dpos,
                           nk, l.grp.bytes);
        e = hipGetLastError();
    }
    if (e == hipSuccess && nb > 0) e = hipMemcpyAsync(hc.bytes, l.grp.bytes, (size_t)nb, hipMemcpyDeviceToHost, l.st);
    if (e == hipSuccess) e = hipMemcpyAsync(hc.off, l.grp.off, 8 * (size_t)(nk + 1), hipMemcpyDeviceToHost, l.st);
    if (e == hipSuccess) e = hipMemcpyAsync(hc.ids, l.grp.ids, 4 * (size_t)nk, hipMemcpyDeviceToHost, l.st);
    if (e == hipSuccess) e = hipMemcpyAsync(hc.sig, l.grp.sig, 4 * (size_t)nk, hipMemcpyDeviceToHost, l.st);
    if (e == hipSuccess) e = hipMemcpyAsync(hc.info, l.info, 32 * (size_t)P, hipMemcpyDeviceToHost, l.st);
    if (e == hipSuccess) e = hipEventRecord(l.ev, l.st);
    c.stats.bytes_d2h += nb + 16 * nk + 8 + 32 * P;
    c.stats.chunks++;
    l.busy = true;
    return from_hip(e);
}

int lane_wait(Lane &l)
{
    if (!l.busy) return ASJ_OK;
    l.busy = false;
    return from_hip(hipEventSynchronize(l.ev));
}

int partition_rel(Ctx &c, const HostRel &h, int logp, HostStore &store, int which)
{
    const int P = 1 << logp;
    std::vector<Range> ranges;
    // two lanes, each with an input and a grouped copy of its chunk, share
    // three quarters of the budget
    const int64_t cost = std::max<int64_t>(c.budget * 3 / 16 - 4096, 1);
    int rc = split_rows(&h, 0, h.n, kMaxChunkKeys, kPerKeyBytes, cost, ranges);
    if (rc != ASJ_OK) return rc;
    int64_t mk = 1, mb = 1;
    size_t host = 0;
    for (const Range &r : ranges) {
        mk = std::max(mk, r.b - r.a);
        mb = std::max(mb, rows_bytes(h, r.a, r.b));
        host += chunk_host_bytes(r.b - r.a, rows_bytes(h, r.a, r.b), P);
    }
    store.chunks.clear();
    rc = store_arena(c, store, which, host);
    if (rc != ASJ_OK) return rc;
    // carve every chunk's pinned region up front
    size_t carve = 0;
    for (const Range &r : ranges) {
        HostChunk hc;
        hc.n = r.b - r.a;
        hc.nbytes = rows_bytes(h, r.a, r.b);
        hc.bytes = store.arena + carve;
        hc.off = (int64_t *)(hc.bytes + al((size_t)hc.nbytes + 16));
        hc.ids = (int32_t *)((uint8_t *)hc.off + al(8 * (size_t)(hc.n + 1)));
        hc.sig = (uint32_t *)((uint8_t *)hc.ids + al(4 * (size_t)hc.n + 4));
        hc.info = (int64_t *)((uint8_t *)hc.sig + al(4 * (size_t)hc.n + 4));
        carve += chunk_host_bytes(hc.n, hc.nbytes, P);
        store.chunks.push_back(hc);
    }
    hipEvent_t start = nullptr;
    hipError_t e = hipEventCreateWithFlags(&start, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(start, c.st); // after the caller's earlier work on its stream
    rc = from_hip(e);
    Lane lanes[2];
    for (int i = 0; rc == ASJ_OK && i < 2 && i < (int)ranges.size(); i++) rc = open_lane(c, lanes[i], mk, mb, P, start);
    for (size_t i = 0; rc == ASJ_OK && i < ranges.size(); i++) {
        Lane &l = lanes[i & 1];
        rc = lane_wait(l);
        if (rc == ASJ_OK)
            rc = partition_chunk(c, l, h, ranges[i].a, ranges[i].b, logp, store.chunks[i],
                                 i > 0 ? lanes[(i - 1) & 1].in_done : nullptr);
    }
    for (int i = 0; i < 2; i++) {
        const int r2 = lane_wait(lanes[i]);
        if (rc == ASJ_OK) rc = r2;
        close_lane(c, lanes[i], mk, P);
    }
    if (start) (void)hipEventDestroy(start);
    return rc;
}

// ---- build and probe ----
struct Table {
    DevRel rel;
    int64_t n = 0;
    uint64_t *slots = nullptr;
    int64_t cap = 0, slot_cap = 0;
    int32_t *status = nullptr;
};

int64_t table_slots(int64_t n, float lf)
{
    int64_t cap = 64;
    while ((double)cap * lf < (double)n) cap <<= 1;
    return cap;
}

size_t table_bytes(int64_t keys, int64_t bytes, float lf)
{
    return devrel_bytes(keys, bytes) + al(8 * (size_t)table_slots(keys, lf)) + al(4);
}

// Loads the ranges (one build partition, or the whole build relation) into
// t.rel back to back and builds the table: signatures from the ranges when
// they carry them, else signed here (Section 3.2, Figure 2, build phase).
int build_table(Ctx &c, Table &t, const std::vector<Range> &parts)
{
    int64_t kb = 0, bb = 0;
    bool signed_ = true;
    for (const Range &r : parts) {
        const int rc = load_rows(c, *r.h, r.a, r.b, t.rel, kb, bb, c.st);
        if (rc != ASJ_OK) return rc;
        signed_ = signed_ && r.h->sig;
        kb += r.b - r.a;
        bb += rows_bytes(*r.h, r.a, r.b);
    }
    if (parts.empty()) {
        hipError_t e = asj_launch_fill_i64(t.rel.off, 1, 0, c.st);
        if (e != hipSuccess) return from_hip(e);
    }
    t.n = kb;
    t.cap = table_slots(kb, c.ro.lf);
    hipError_t e = asj_launch_fill64(t.slots, t.cap, ASJ_EMPTY_SLOT, c.st);
    if (e == hipSuccess) e = asj_launch_fill_i32(t.status, 1, 0, c.st);
    if (e == hipSuccess && !signed_) e = sign_rel(c, t.rel, kb, c.st);
    if (e == hipSuccess && kb > 0)
        e = asj_launch_insert(t.rel.sig, kb, c.ro.plain, t.slots, (uint64_t)t.cap - 1, t.status, c.st);
    return from_hip(e);
}

struct Slot {
    DevRel rel;
    asj_pair *out = nullptr;
    int64_t out_cap = 0;
    int64_t *dcount = nullptr; // device
    int64_t *hcount = nullptr; // pinned host
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    Range r = {nullptr, 0, 0};
};

struct Output {
    asj_pair *out;
    int64_t cap;
    int64_t total;
};

// Probes rows r of a host relation, staged in slot s, against t.
int enqueue_probe(Ctx &c, const Table &t, Slot &s, const Range &r)
{
    const int64_t nk = r.b - r.a;
    int rc = load_rows(c, *r.h, r.a, r.b, s.rel, 0, 0, s.st);
    if (rc != ASJ_OK) return rc;
    hipError_t e = asj_launch_fill_i64(s.dcount, 1, 0, s.st);
    const bool presigned = r.h->sig != nullptr;
    if (e == hipSuccess && !presigned && c.ro.split) e = sign_rel(c, s.rel, nk, s.st);
    if (e == hipSuccess) {
        asj_probe_args a = {};
        a.rdata = t.rel.bytes;
        a.roff = t.rel.off;
        a.rids = t.rel.ids;
        a.rn = t.n;
        a.keys_per_window = c.ro.kpw;
        a.sdata = s.rel.bytes;
        a.soff = s.rel.off;
        a.sids = s.rel.ids;
        a.n = nk;
        a.ssig = (presigned || c.ro.split) ? s.rel.sig : nullptr;
        a.slots = t.slots;
        a.mask = (uint64_t)t.cap - 1;
        a.out = s.out;
        a.cap = s.out_cap;
        a.out_count = s.dcount;
        a.table_status = t.status;
        a.grid_rounds = c.ro.grid_rounds;
        a.plain = c.ro.plain;
        a.verify = c.ro.verify;
        a.kind = c.ro.kind;
        if (nk > 0) e = asj_launch_probe(&a, c.mode, c.nsym, c.tab, kGridCap, s.st);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(s.hcount, s.dcount, 8, hipMemcpyDeviceToHost, s.st);
    if (e == hipSuccess) e = hipEventRecord(s.ev, s.st);
    c.stats.pieces++;
    s.r = r;
    s.busy = true;
    return from_hip(e);
}

int copy_out(Ctx &c, Slot &s, int64_t cnt, Output &o)
{
    const int64_t room = std::max<int64_t>(0, o.cap - o.total), ncopy = std::min(cnt, room);
    hipError_t e = hipSuccess;
    if (ncopy > 0) {
        e = hipMemcpyAsync(o.out + o.total, s.out, 8 * (size_t)ncopy, hipMemcpyDeviceToHost, s.st);
        if (e == hipSuccess) e = hipStreamSynchronize(s.st);
        c.stats.bytes_d2h += 8 * ncopy;
    }
    o.total += cnt;
    return from_hip(e);
}

// Waits for slot s and collects its pairs; a range whose pairs overflow the
// slot's output buffer is probed again in halves.
int finish(Ctx &c, const Table &t, Slot &s, Output &o)
{
    if (!s.busy) return ASJ_OK;
    s.busy = false;
    hipError_t e = hipEventSynchronize(s.ev);
    if (e != hipSuccess) return from_hip(e);
    const int64_t cnt = *s.hcount;
    if (cnt < 0) return ASJ_EINVAL;
    if (cnt <= s.out_cap) return copy_out(c, s, cnt, o);
    const Range r = s.r;
    if (r.b - r.a == 1) return ASJ_ENOMEM; // one probe row has more pairs than the buffer holds
    const int64_t mid = r.a + (r.b - r.a) / 2;
    for (const Range &half : {Range{r.h, r.a, mid}, Range{r.h, mid, r.b}}) {
        int rc = enqueue_probe(c, t, s, half);
        if (rc == ASJ_OK) rc = finish(c, t, s, o);
        if (rc != ASJ_OK) return rc;
    }
    return ASJ_OK;
}

int table_status(const Table &t, hipStream_t st)
{
    int32_t v = 0;
    hipError_t e = hipMemcpyAsync(&v, t.status, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return from_hip(e);
    return v;
}

// Probes the ranges against t through the two slots.
int stream_probe(Ctx &c, const Table &t, Slot *slots, const std::vector<Range> &ranges, Output &o)
{
    hipEvent_t built = nullptr;
    hipError_t e = hipEventCreateWithFlags(&built, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(built, c.st);
    for (int i = 0; e == hipSuccess && i < 2; i++) e = hipStreamWaitEvent(slots[i].st, built, 0);
    int rc = from_hip(e);
    for (size_t i = 0; rc == ASJ_OK && i < ranges.size(); i++) {
        Slot &s = slots[i & 1];
        rc = finish(c, t, s, o);
        if (rc == ASJ_OK) rc = enqueue_probe(c, t, s, ranges[i]);
    }
    for (int i = 0; i < 2; i++) {
        const int r2 = finish(c, t, slots[i], o);
        if (rc == ASJ_OK) rc = r2;
    }
    if (built) (void)hipEventDestroy(built);
    if (rc == ASJ_OK) {
        const int ts = table_status(t, c.st);
        if (ts != ASJ_OK) rc = ts;
    }
    return rc;
}

// Device bytes of one slot for probe ranges of up to keys / bytes, with an
// output buffer of out_cap pairs.
size_t slot_bytes(int64_t keys, int64_t bytes, int64_t out_cap)
{
    return devrel_bytes(keys, bytes) + al(8 * (size_t)out_cap) + 2 * al(8);
}

int open_slots(Ctx &c, Slot *slots, int64_t keys, int64_t bytes, int64_t out_cap)
{
    for (int i = 0; i < 2; i++) {
        Slot &s = slots[i];
        s.out_cap = out_cap;
        int rc = alloc_rel(c, s.rel, keys, bytes);
        if (rc == ASJ_OK) rc = dalloc(c, (void **)&s.out, 8 * (size_t)out_cap);
        if (rc == ASJ_OK) rc = dalloc(c, (void **)&s.dcount, 8);
        if (rc != ASJ_OK) return rc;
        hipError_t e = hipHostMalloc((void **)&s.hcount, 8, hipHostMallocDefault);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
        if (e != hipSuccess) return from_hip(e);
    }
    return ASJ_OK;
}

void close_slots(Ctx &c, Slot *slots)
{
    for (int i = 0; i < 2; i++) {
        Slot &s = slots[i];
        if (s.st) (void)hipStreamSynchronize(s.st);
        free_rel(c, s.rel);
        dfree(c, s.out, 8 * (size_t)s.out_cap);
        dfree(c, s.dcount, 8);
        if (s.hcount) (void)hipHostFree(s.hcount);
        if (s.ev) (void)hipEventDestroy(s.ev);
        if (s.st) (void)hipStreamDestroy(s.st);
        s = Slot();
    }
}

// Splits the device memory left beside the table into two slots (input
// three quarters, output pairs one quarter) and cuts the probe ranges to fit.
int plan_slots(Ctx &c, int64_t left, const std::vector<Range> &in, std::vector<Range> &out, int64_t *keys,
               int64_t *bytes, int64_t *out_cap)
{
    const int64_t per_slot = left / 2 - 4096;
    // pieces of at most kMaxPieceBytes keep the two slots alternating (one
    // piece's copy in while the other is probed) and their buffers small
    const int64_t input = std::min<int64_t>(per_slot / 4 * 3, kMaxPieceBytes);
    *out_cap = std::max<int64_t>(1, (per_slot - input) / 8 - 64);
    if (input <= 1024) return ASJ_ENOMEM;
    for (const Range &r : in) {
        const int rc = split_rows(r.h, r.a, r.b, INT32_MAX, 16, input - 1024, out);
        if (rc != ASJ_OK) return rc;
    }
    *keys = 1;
    *bytes = 1;
    for (const Range &r : out) {
        *keys = std::max(*keys, r.b - r.a);
        *bytes = std::max(*bytes, rows_bytes(*r.h, r.a, r.b));
    }
    (void)c;
    return ASJ_OK;
}

int host_rel_ok(const asj_keys *k)
{
    if (!k || k->n < 0 || k->n >= (int64_t)INT32_MAX) return ASJ_EINVAL;
    if (k->n == 0) return ASJ_OK;
    if (!k->offsets || k->offsets[0] < 0) return ASJ_EINVAL;
    for (int64_t i = 0; i < k->n; i++)
        if (k->offsets[i + 1] < k->offsets[i]) return ASJ_EINVAL;
    if (k->offsets[k->n] > k->offsets[0] && !k->data) return ASJ_EINVAL;
    return ASJ_OK;
}

HostRel whole(const asj_keys *k)
{
    static const int64_t zero = 0;
    HostRel h;
    h.bytes = k->data;
    h.off = k->n > 0 ? k->offsets : &zero;
    h.ids = k->ids;
    h.n = k->n;
    return h;
}

int join_host(Ctx &c, const asj_keys *r, const asj_keys *s, int forced_p, Output &o)
{
    using clk = std::chrono::steady_clock;
    const HostRel hr = whole(r), hs = whole(s);
    const int64_t rbytes = rows_bytes(hr, 0, hr.n);
    const size_t need1 = table_bytes(hr.n, rbytes, c.ro.lf);
    int logp = 0;
    if (forced_p > 0) {
        while ((1 << logp) < forced_p) logp++;
    } else {
        while ((int64_t)need1 * 5 / 4 / (1 << logp) > c.budget / 2 && logp < kMaxLogP) logp++;
        if (logp == 0 && (int64_t)need1 > c.budget / 2) logp = 1;
    }
    std::vector<std::vector<Range>> rparts, sparts;
    auto t0 = clk::now();
    if (logp == 0) {
        rparts.push_back({Range{&hr, 0, hr.n}});
        sparts.push_back({Range{&hs, 0, hs.n}});
    } else {
        for (;;) { // partition R; more partitions while the largest does not fit half the budget
            int rc = partition_rel(c, hr, logp, c.store_r, 0);
            if (rc != ASJ_OK) return rc;
            size_t worst = 0;
            for (int p = 0; p < (1 << logp); p++) {
                int64_t k = 0, b = 0;
                for (const HostChunk &h : c.store_r.chunks) {
                    k += h.info[4 * p + 1];
                    b += h.info[4 * p + 3];
                }
                worst = std::max(worst, table_bytes(k, b, c.ro.lf));
            }
            if ((int64_t)worst <= c.budget / 2) break;
            if (logp >= kMaxLogP || forced_p > 0) return ASJ_ENOMEM;
            logp++;
        }
        int rc = partition_rel(c, hs, logp, c.store_s, 1);
        if (rc != ASJ_OK) return rc;
    }
    auto t1 = clk::now();
    const int P = 1 << logp;
    c.stats.partitions = P;
    // host views of the grouped chunks (their addresses must stay put)
    std::vector<HostRel> vr, vs;
    for (const HostChunk &h : c.store_r.chunks) vr.push_back(h.rel());
    for (const HostChunk &h : c.store_s.chunks) vs.push_back(h.rel());
    if (logp > 0) {
        rparts.assign(P, {});
        sparts.assign(P, {});
        for (int p = 0; p < P; p++) {
            for (size_t i = 0; i < vr.size(); i++) {
                const int64_t a = c.store_r.chunks[i].info[4 * p], n = c.store_r.chunks[i].info[4 * p + 1];
                if (n > 0) rparts[p].push_back(Range{&vr[i], a, a + n});
            }
            for (size_t i = 0; i < vs.size(); i++) {
                const int64_t a = c.store_s.chunks[i].info[4 * p], n = c.store_s.chunks[i].info[4 * p + 1];
                if (n > 0) sparts[p].push_back(Range{&vs[i], a, a + n});
            }
        }
    }
    // the largest build partition sizes the table buffers
    int64_t mk = 0, mb = 0;
    for (const auto &rp : rparts) {
        int64_t k = 0, b = 0;
        for (const Range &x : rp) {
            k += x.b - x.a;
            b += rows_bytes(*x.h, x.a, x.b);
        }
        mk = std::max(mk, k);
        mb = std::max(mb, b);
    }
    Table t;
    t.slot_cap = table_slots(mk, c.ro.lf);
    int rc = alloc_rel(c, t.rel, mk, mb);
    if (rc == ASJ_OK) rc = dalloc(c, (void **)&t.slots, 8 * (size_t)t.slot_cap);
    if (rc == ASJ_OK) rc = dalloc(c, (void **)&t.status, 4);
    Slot slots[2];
    std::vector<std::vector<Range>> pieces(sparts.size());
    int64_t sk = 0, sb = 0, out_cap = 0;
    if (rc == ASJ_OK) {
        std::vector<Range> all;
        for (const auto &sp : sparts) all.insert(all.end(), sp.begin(), sp.end());
        std::vector<Range> cut;
        rc = plan_slots(c, c.budget - c.used, all, cut, &sk, &sb, &out_cap);
        // regroup the cut ranges by partition (cutting keeps their order)
        size_t j = 0;
        for (size_t p = 0; rc == ASJ_OK && p < sparts.size(); p++)
            for (const Range &x : sparts[p])
                while (j < cut.size() && cut[j].h == x.h && cut[j].a >= x.a && cut[j].b <= x.b)
                    pieces[p].push_back(cut[j++]);
    }
    if (rc == ASJ_OK) {
        // output buffers: four pairs per probe row of the largest piece (at
        // least 64k), within what the budget still holds beside the input;
        // a piece that produces more is probed again in halves
        out_cap = std::min(out_cap, std::max<int64_t>(4 * sk, 1 << 16));
        while (out_cap > 1 && c.used + 2 * (int64_t)slot_bytes(sk, sb, out_cap) > c.budget) out_cap /= 2;
        rc = open_slots(c, slots, sk, sb, out_cap);
    }
    const bool keep_empty_build = c.ro.kind == ASJ_KIND_ANTI || c.ro.kind == ASJ_KIND_LEFT;
    for (size_t p = 0; rc == ASJ_OK && p < rparts.size(); p++) {
        if (pieces[p].empty()) continue;                        // no probe rows: no output
        if (rparts[p].empty() && !keep_empty_build) continue;   // no build rows: only anti / left rows
        rc = build_table(c, t, rparts[p]);
        if (rc == ASJ_OK) rc = stream_probe(c, t, slots, pieces[p], o);
    }
    close_slots(c, slots);
    free_rel(c, t.rel);
    dfree(c, t.slots, 8 * (size_t)t.slot_cap);
    dfree(c, t.status, 4);
    auto t2 = clk::now();
    c.stats.ms_partition = std::chrono::duration<double, std::milli>(t1 - t0).count();
    c.stats.ms_join = std::chrono::duration<double, std::milli>(t2 - t1).count();
    return rc;
}

} // namespace

extern "C" int asj_join_host(const asj_keys *r, const asj_keys *s, const asj_opts *opts, const asj_host_opts *hopts,
                             asj_pair *out, int64_t out_cap, int64_t *out_count, asj_host_stats *stats,
                             hipStream_t stream)
{
    if (!out_count || out_cap < 0 || (out_cap > 0 && !out)) return ASJ_EINVAL;
    int rc = host_rel_ok(r);
    if (rc == ASJ_OK) rc = host_rel_ok(s);
    if (rc != ASJ_OK) return rc;
    asj_host_opts ho = {};
    if (hopts) ho = *hopts;
    if (ho.hbm_budget < 0 || ho.partitions < 0 || ho.partitions > (1 << kMaxLogP) ||
        (ho.partitions & (ho.partitions - 1)))
        return ASJ_EINVAL;
    if (opts && (opts->flags & ASJ_SORTED)) return ASJ_EUNSUPPORTED;
    Ctx c;
    rc = asj_resolve_opts(opts, r->n, &c.ro);
    if (rc != ASJ_OK) return rc;
    int dev = 0;
    c.tab = asj_device_tables(&dev);
    if (!c.tab) return ASJ_EHIP;
    c.mode = c.ro.plain ? ASJ_MODE_PLAIN : (c.ro.sig.f == 16 ? ASJ_MODE_SIG16 : ASJ_MODE_SIG8);
    c.nsym = c.ro.plain ? 1 : c.ro.sig.nsym;
    c.st = stream;
    if (ho.hbm_budget > 0) {
        c.budget = ho.hbm_budget;
    } else {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return ASJ_EHIP;
        c.budget = (int64_t)(fr / 5 * 4);
    }
    Output o = {out, out_cap, 0};
    std::unique_lock<std::mutex> pin(g_pin_mu, std::try_to_lock);
    c.cache = pin.owns_lock();
    rc = join_host(c, r, s, ho.partitions, o);
    free_store(c.store_r);
    free_store(c.store_s);
    if (rc != ASJ_OK) return rc;
    *out_count = o.total;
    if (stats) *stats = c.stats;
    return ASJ_OK;
}

extern "C" int asj_join_host_release(void)
{
    std::lock_guard<std::mutex> lk(g_pin_mu);
    for (Pinned &g : g_pin) {
        if (g.p) (void)hipHostFree(g.p);
        g = Pinned();
    }
    return ASJ_OK;
}
