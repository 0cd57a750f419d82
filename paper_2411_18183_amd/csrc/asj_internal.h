// Internal declarations shared by the HIP translation units of libasjoin.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "asjoin.h"

#define ASJ_WAVE 64
#define ASJ_CHUNK 64          // key bytes handled by one lane per pass
#define ASJ_EMPTY_SLOT (~0ull)
#define ASJ_DEFAULT_KEYS_PER_WINDOW 64

// ---------------------------------------------------------------------------
// GF(2^16) constant-multiply tables.
//
// Multiplying a 16-bit field element v by a fixed constant c is linear over
// GF(2), so it is the XOR of two byte-indexed lookups:
//     v * c = T_c[v & 255] ^ T_c[256 + (v >> 8)],
// with T_c[b] = b * c and T_c[256 + b] = (b x^8) * c.  Each table pair is
// 512 uint16 = 1 KB.  The library builds the pairs it needs once per device
// (field polynomial x^16 + x^12 + x^3 + x + 1, alpha = x).
//
// Index map (ASJ_NTAB16 pairs), components j = 1, 2:
//   0                     c = x^16 (folds bits 16..31 of an unreduced word)
//   1 + 17(j-1) + v       c = alpha^(32 j v),   v = 0..7  (chunk index digit 0)
//   1 + 17(j-1) + 8 + v   c = alpha^(256 j v),  v = 0..7  (chunk index digit 1)
//   1 + 17(j-1) + 16      c = alpha^(2048 j)             (64-chunk block)
// ---------------------------------------------------------------------------
#define ASJ_TAB_WORDS 512
#define ASJ_NTAB16 35
#define ASJ_TAB_RED 0
__host__ __device__ inline int asj_tab_d0(int j, int v) { return 1 + 17 * (j - 1) + v; }
__host__ __device__ inline int asj_tab_d1(int j, int v) { return 1 + 17 * (j - 1) + 8 + v; }
__host__ __device__ inline int asj_tab_blk(int j) { return 1 + 17 * (j - 1) + 16; }

// GF(2^8) (polynomial x^8 + x^4 + x^3 + x^2 + 1, alpha = x) tables, stored
// after the GF(2^16) pairs as uint16 words (low byte used):
//   [0, 510)       exp8[e] = alpha^(e mod 255)
//   [512, 768)     log8[v]  (log8[0] unused)
//   [768 + 256(k-1) + b]   b * x^(8k) mod g8, k = 1, 2, 3 (fold bytes 1..3)
#define ASJ_NTAB8 4
#define ASJ_TAB8_BASE (ASJ_NTAB16 * ASJ_TAB_WORDS)
#define ASJ_TAB8_EXP 0
#define ASJ_TAB8_LOG 512
#define ASJ_TAB8_RED 768

// GF(2^16) pairs read from device memory only (never copied to LDS), after
// the GF(2^8) tables: c = alpha^(2048 j d 8^k) for components j = 1, 2,
// octal digit k = 0..6 of a chunk's 64-chunk block index and digit value
// d = 1..7 -- the position factor of chunks 192 and beyond (keys longer
// than 12 KB), one pair per non-zero digit.
#define ASJ_NTAB_HI 98
#define ASJ_TAB_HI_BASE ((ASJ_NTAB16 + ASJ_NTAB8) * ASJ_TAB_WORDS)
__host__ __device__ inline int asj_tab_hi(int j, int k, int d) { return (7 * (j - 1) + k) * 7 + (d - 1); }
#define ASJ_TAB_TOTAL_WORDS ((ASJ_NTAB16 + ASJ_NTAB8 + ASJ_NTAB_HI) * ASJ_TAB_WORDS)

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------
typedef uint32_t asj_u32x4 __attribute__((ext_vector_type(4), aligned(4)));

__device__ inline void asj_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Bijective 32-bit mixer (finalizer of MurmurHash3) used to place a
// signature in the table; any bijection gives the same join output.
__host__ __device__ inline uint32_t asj_mix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

__device__ inline uint32_t asj_cmul16(uint32_t v, const uint16_t *t)
{
    return (uint32_t)t[v & 255u] ^ (uint32_t)t[256u + (v >> 8)];
}

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ inline int asj_wave_incl_scan(int v)
{
    const int lane = threadIdx.x & (ASJ_WAVE - 1);
#pragma unroll
    for (int d = 1; d < ASJ_WAVE; d <<= 1) {
        int o = __shfl_up(v, d, ASJ_WAVE);
        if (lane >= d) v += o;
    }
    return v;
}

// Chunk loaders.  A key of len bytes is read as floor(len / 64) full 64-byte
// chunks and, when len is not a multiple of 64, one tail chunk of len % 64
// bytes.  The loaders return 16 little-endian words holding key-relative bytes
// (word t = key bytes k0+4t .. k0+4t+3, where `a` is the arena address of
// key byte k0).  Only 4-byte-aligned words that hold at least one byte of
// the key are read, so a load never leaves the pages of the arena.

// Full chunk: the 64 bytes at a are all key bytes.  Words are read at
// a & ~3 and realigned; the 17th word (needed when a is not 4-aligned)
// still starts before the key's end.  Fetching (issuing the loads) and
// realigning are separate steps so that a caller can have the loads of the
// next chunk in flight while it folds the current one.
struct asj_raw_chunk {
    uint32_t d[17];
    uint32_t sh;
};

__device__ __forceinline__ void asj_fetch_full(const uint8_t *__restrict__ data, int64_t a, asj_raw_chunk &r)
{
    r.sh = (uint32_t)(a & 3);
    const uint32_t *p = (const uint32_t *)(data + (a - r.sh));
    const asj_u32x4 *q = (const asj_u32x4 *)p;
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const asj_u32x4 v = q[t];
        r.d[4 * t + 0] = v.x;
        r.d[4 * t + 1] = v.y;
        r.d[4 * t + 2] = v.z;
        r.d[4 * t + 3] = v.w;
    }
    r.d[16] = 0u;
    if (r.sh) r.d[16] = p[16];
}

__device__ __forceinline__ void asj_align_full(const asj_raw_chunk &r, uint32_t kd[16])
{
#pragma unroll
    for (int t = 0; t < 16; t++) kd[t] = __builtin_amdgcn_alignbyte(r.d[t + 1], r.d[t], r.sh);
}

__device__ __forceinline__ void asj_load_full(const uint8_t *__restrict__ data, int64_t a, uint32_t kd[16])
{
    asj_raw_chunk r;
    asj_fetch_full(data, a, r);
    asj_align_full(r, kd);
}

// The first min(len, 16) bytes of the key at a, zero past them; reads only
// 4-byte words that hold at least one of those bytes (none for len = 0).
__device__ __forceinline__ void asj_load_head16(const uint8_t *__restrict__ data, int64_t a, int len, uint32_t k[4])
{
    const uint32_t sh = (uint32_t)(a & 3);
    const uint32_t *p = (const uint32_t *)(data + (a - sh));
    const int n = len < 16 ? len : 16;
    const int avail = n + (int)sh; // bytes from p through the last wanted byte
    uint32_t w[5];
#pragma unroll
    for (int t = 0; t < 5; t++) w[t] = (n > 0 && 4 * t < avail) ? p[t] : 0u;
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const uint32_t v = __builtin_amdgcn_alignbyte(w[t + 1], w[t], sh);
        const int keep = n - 4 * t;
        k[t] = keep >= 4 ? v : keep <= 0 ? 0u : (v & ((1u << (8 * keep)) - 1u));
    }
}

// Tail chunk: rem (1..63) key bytes at a; bytes at or past rem read as zero.
__device__ __forceinline__ void asj_load_tail(const uint8_t *__restrict__ data, int64_t a, int rem, uint32_t kd[16])
{
    const uint32_t sh = (uint32_t)(a & 3);
    const uint32_t *p = (const uint32_t *)(data + (a - sh));
    const int avail = rem + (int)sh; // bytes from p through the key's end
    uint32_t d[17];
#pragma unroll
    for (int t = 0; t < 17; t++) d[t] = (4 * t < avail) ? p[t] : 0u;
#pragma unroll
    for (int t = 0; t < 16; t++) {
        const uint32_t w = __builtin_amdgcn_alignbyte(d[t + 1], d[t], sh);
        const int nb = rem - 4 * t; // key bytes in this word
        const uint32_t m = nb >= 4 ? 0xFFFFFFFFu : (nb <= 0 ? 0u : ((1u << (8 * nb)) - 1u));
        kd[t] = w & m;
    }
}

// Tail chunk read as a full chunk when the 68 bytes from the 4-byte-aligned
// address below a all lie before `end` (the end of the relation's keys, whose
// bytes run back to back, so the words past this key hold the next keys'
// bytes): 4 wide loads instead of up to 17 guarded ones; bytes at or past
// rem are masked to zero.  Near the end of the keys, the guarded loader.
__device__ __forceinline__ void asj_load_tail_fast(const uint8_t *__restrict__ data, int64_t a, int rem, int64_t end,
                                                   uint32_t kd[16])
{
    if ((a & ~(int64_t)3) + 68 <= end) {
        asj_load_full(data, a, kd);
#pragma unroll
        for (int t = 0; t < 16; t++) {
            const int nb = rem - 4 * t;
            kd[t] &= nb >= 4 ? 0xFFFFFFFFu : (nb <= 0 ? 0u : ((1u << (8 * nb)) - 1u));
        }
    } else {
        asj_load_tail(data, a, rem, kd);
    }
}

// Inclusive prefix maximum across the 64 lanes of a wave (values >= -1):
// shifts within each row of 16 lanes, then the last lane of a row into the
// rows after it (DPP row_shr and row_bcast).
__device__ __forceinline__ int asj_wave_incl_max(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x111, 0xf, 0xf, false)); // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x112, 0xf, 0xf, false)); // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x114, 0xf, 0xf, false)); // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x118, 0xf, 0xf, false)); // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x142, 0xa, 0xf, false)); // row_bcast:15 into rows 1, 3
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x143, 0xc, 0xf, false)); // row_bcast:31 into rows 2, 3
    return v;
}

// Owner of chunk position base + lane in a pass over keys laid out back to
// back: the last key (lane index) with chunks that starts at or before it.
// ex_me / n_me: this lane's key's first chunk and chunk count; own: the
// wave's 64-entry LDS scratch; carry: the owner of the previous pass's last
// position (-1 before the first pass), updated.
__device__ __forceinline__ int asj_pass_owner(int ex_me, int n_me, int base, int32_t *own, int &carry)
{
    const int lane = threadIdx.x & (ASJ_WAVE - 1);
    own[lane] = -1;
    asj_wave_sync();
    if (n_me > 0 && ex_me >= base && ex_me < base + ASJ_WAVE) own[ex_me - base] = lane;
    asj_wave_sync();
    const int o = asj_wave_incl_max(max(own[lane], carry));
    carry = __builtin_amdgcn_readlane(o, ASJ_WAVE - 1);
    asj_wave_sync();
    return min(max(o, 0), ASJ_WAVE - 1);
}

// Largest i in [0, 64) with ex[i] <= x, for a non-decreasing ex[] in LDS
// whose first entry is 0.
__device__ __forceinline__ int asj_find_owner(const int32_t *ex, int x)
{
    int lo = 0, hi = ASJ_WAVE - 1;
#pragma unroll
    for (int it = 0; it < 6; it++) {
        const int mid = (lo + hi + 1) >> 1;
        if (ex[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The build-side table (asj_table in the public header).
struct asj_table {
    asj_keys r;          // borrowed build relation
    void *block;         // one device allocation: slots, status, build signatures, region-build scratch
    uint64_t *slots;     // capacity slots
    int64_t capacity;    // power of two
    int32_t *status;     // device word: 0 or ASJ_ETABLEFULL
    int plain;           // baseline table (no signature stored)
    int fp;              // fingerprint control: the baseline's key hash stored and compared as a signature
    int verify;          // probe compares key bytes of candidates
    asj_sig_params sig;  // signature parameters of the build
    uint32_t *sig_hi;    // four GF(2^16) components: the build rows' high words (the slots hold the low words)
    int keys_per_window; // probe keys per wave window used by probes of this table
    int grid_rounds;     // probe grid in units of the blocks the device holds at once
    int split;           // probes sign the probe keys in a separate kernel first
    int sorted;          // probes sort their output pairs by (r_id, s_id)
    int validate;        // probes check the probe relation's offsets first
    int kind;            // ASJ_KIND_*
    hipStream_t stream;  // build stream (orders free)
    int device;
};

// Options recorded by the autotuner for a size class (build rows rounded
// up to a power of two, signature parameters, plain/verify flags, single
// join or batch) on the current device.
struct asj_tuned {
    float load_factor;
    int keys_per_window;
    int split;
    int grid_rounds;
};
bool asj_tuned_lookup(int batch, int64_t n_build, const asj_opts &o, asj_tuned *t);
void asj_tuned_store(int batch, int64_t n_build, const asj_opts &o, const asj_tuned &t);

// Join options resolved as asj_build resolves them (signature parameters,
// plain / verify, join kind, and load factor, keys per window and schedule
// from the caller, else the autotuner's record, else the defaults) for a
// build side of n_build rows.
struct asj_resolved {
    asj_sig_params sig;
    int plain, verify, kind, split, kpw, grid_rounds;
    float lf;
};
int asj_resolve_opts(const asj_opts *opts, int64_t n_build, asj_resolved *r);

// GF constant tables of the current device (initialising the library on
// first use); nullptr on failure.
const uint16_t *asj_device_tables(int *dev);

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files; all asynchronous on `st`)
// ---------------------------------------------------------------------------
enum asj_sign_mode {
    ASJ_MODE_SIG16 = 0, // GF(2^16) signature, nsym components (1 or 2)
    ASJ_MODE_SIG8 = 1,  // GF(2^8) signature, nsym components (2 or 4)
    ASJ_MODE_PLAIN = 2, // plain multiplicative full-key hash (baseline)
};

hipError_t asj_launch_tables(uint16_t *tab, hipStream_t st);
// status (may be NULL): device word; when it is non-zero the kernel reads no key.
// out[k * stride] = signature (plain hash) of key k; with four GF(2^16)
// components that is the low word (components 1, 2) and out_hi[k * stride]
// receives the high word (components 3, 4).
// prep (may be NULL): the batch's window and region maps, written by the
// kernel's blocks before they sign (one launch fewer per batch).
// kpw: keys per signing window (1 .. 64), or 0 for asj_auto_kpw's choice
// from the keys' mean length, made by the kernel.
struct asj_batch_prep;
hipError_t asj_launch_sign(int mode, int nsym, const asj_keys *k, uint32_t *out, const uint16_t *tab,
                           int grid_cap, hipStream_t st, const int32_t *status = nullptr,
                           uint32_t *out_hi = nullptr, int stride = 1, const asj_batch_prep *prep = nullptr,
                           int kpw = ASJ_WAVE);
// Sets *status = ASJ_EINVAL unless off[0] >= 0 and off[] never decreases.
hipError_t asj_launch_validate(const int64_t *off, int64_t n, int32_t *status, hipStream_t st);
hipError_t asj_launch_fill64(uint64_t *p, int64_t n, uint64_t v, hipStream_t st);
hipError_t asj_launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t st);
hipError_t asj_launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);
// slots[0 .. cap) = empty and *status = ASJ_OK in one launch (and *z0, *z1 =
// 0 where not NULL: the counters of the probe that follows).
hipError_t asj_launch_table_init(uint64_t *slots, int64_t cap, int32_t *status, hipStream_t st,
                                 int64_t *z0 = nullptr, int64_t *z1 = nullptr);
// *a = 0 and, when b is not NULL, *b = 0 in one launch.
hipError_t asj_launch_zero2(int64_t *a, int64_t *b, hipStream_t st);
hipError_t asj_launch_insert(const uint32_t *sig, int64_t m, int plain, uint64_t *slots, uint64_t mask,
                             int32_t *status, hipStream_t st);
// The same table built by regions of its slots (rows scattered into the
// slots of their home region, each region then built in LDS and written
// whole, the runs that leave a region finished with CAS).
// asj_region_scratch_bytes gives the device scratch it needs, or -1 when the
// table has more than 8192 regions (2^25 slots), m < 327680 or m >= 2^31:
// then the two-pass insert builds it.
// asj_launch_region_init replaces asj_launch_table_init (no slot is written
// there: the build writes every slot) and sets *status = ASJ_OK;
// asj_launch_region_build then fills slots[0 .. cap) from the signatures.
int64_t asj_region_scratch_bytes(int64_t m, int64_t cap);
hipError_t asj_launch_region_init(void *scratch, int64_t m, int64_t cap, int32_t *status, hipStream_t st,
                                  int64_t *z0 = nullptr, int64_t *z1 = nullptr);
hipError_t asj_launch_region_build(const uint32_t *sig, int64_t m, int plain, uint64_t *slots, int64_t cap,
                                   int32_t *status, void *scratch, hipStream_t st);

// Per-join plan of a batch (written on the device by the plan kernel, or by
// the host for the server).  Rows are cut into windows per join, so that no
// window spans two joins: join j's build rows form windows wbase_r ..
// (64 rows each, for the inserts) and its probe rows windows wbase ..
// (keys_per_window rows each, for the probe kernel).
// Join kinds (the flags ASJ_SEMI, ASJ_ANTI, ASJ_LEFT_OUTER).
enum { ASJ_KIND_INNER = 0, ASJ_KIND_SEMI = 1, ASJ_KIND_ANTI = 2, ASJ_KIND_LEFT = 3, ASJ_KIND_RIGHT = 4, ASJ_KIND_FULL = 5 };
// The kinds that list the build rows without a match (their probes mark
// matched build rows, and a kernel appends the others afterwards).
inline bool asj_kind_marks_build(int kind) { return kind == ASJ_KIND_RIGHT || kind == ASJ_KIND_FULL; }

// One probe window of a batch: its join, its first probe row and how many
// rows it holds (1 .. keys_per_window).
struct asj_win {
    int32_t join;
    int32_t rows;
    int64_t first;
};

struct asj_join_desc {
    uint64_t tbase;  // first slot of the join's segment
    uint64_t mask;   // segment capacity - 1 (a power of two minus one); ~0 for a join with an LDS table
    int64_t wbase;   // first probe window of the join (device-memory table)
    int64_t wbase_r; // first build window of the join (device-memory table)
    int64_t wbase_l; // first probe window of the join (LDS table)
    int64_t rbase;   // first table region of the join's segment (batch tables built by regions)
};

// Slots per table region of a batch segment of `cap` slots (a power of two,
// at least 64), as a power of two: the whole segment up to 4096 slots.
__host__ __device__ inline int asj_seg_region_bits(uint64_t cap)
{
    const int b = 63 - __builtin_clzll((unsigned long long)cap);
    return b < 12 ? b : 12;
}

// Batches: a join with at most this many build rows is probed against a
// table that each probing block builds in LDS from the build signatures
// (bucketed by mix32, entries sorted by bucket), instead of a segment of the
// device-memory slot array.
#define ASJ_LOCAL_ROWS 10240

// Blocks of `kernel` that the device holds at once (blocks per compute unit
// from the occupancy calculator x compute units); 0 when the runtime cannot
// say.
inline int64_t asj_resident_blocks(const void *kernel, int block)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, block, 0) != hipSuccess || cus <= 0 || per <= 0) {
        (void)hipGetLastError();
        return 0;
    }
    return (int64_t)cus * per;
}

// Keys per signing window when the caller leaves the choice to the keys
// (kpw = 0): the power of two nearest (on a log scale) to 32768 / mean key
// length, i.e. windows of about eight passes of 64 chunks of 64 bytes,
// within asj_kpw_min(n) .. 64.  Measured on the signature kernel alone, this
// choice came within 11% of the best window size (and within 4% on
// average) over seven sets from 32k keys of 4 KB to 1M keys of 16 bytes to
// 1M DNA keys of 5.5 KB; windows of 64 throughout were up to 47% slower
// (few long keys leave most compute units idle, and long windows balance
// poorly).  bytes / n is the mean key length; 46341 = 32768 * sqrt(2).
// Sets of at most 10240 keys may go down to one key per window (a few
// keys of a megabyte each still spread over many waves); larger sets stop
// at four, which keeps the grid that must cover the smallest windows small.
__host__ __device__ inline int asj_kpw_min(int64_t n) { return n <= ASJ_LOCAL_ROWS ? 1 : 4; }
__host__ __device__ inline int asj_auto_kpw(int64_t n, int64_t bytes)
{
    const int lo = asj_kpw_min(n);
    int kpw = ASJ_WAVE;
    while (kpw > lo && 46341 * n < (int64_t)kpw * bytes) kpw >>= 1;
    return kpw;
}

// A batch's preparation after its plan: the window and region maps (block b
// writes those of joins b, b + nblocks, ...): build window -> join, for every
// probe window its join, first row and row count, LDS-table probe window ->
// join, and table region -> join.  Every write stays inside the capacities
// whatever the segment arrays hold.  (No slot is written: the segments are
// built by regions, which write every slot.)
struct asj_batch_prep {
    const uint64_t *tot; // planned totals: slots, build windows, probe windows, LDS-table windows, regions
    const asj_join_desc *desc;
    const int64_t *s_seg;
    int32_t njoins;
    int32_t kpw;
    int32_t *win_r;
    int64_t win_r_cap;
    asj_win *win_s;
    int64_t win_s_cap;
    int32_t *win_l;
    int64_t win_l_cap;
    uint32_t *rmatch;     // right and full outer joins: the matched-row bytes, zeroed here
    int64_t rmatch_words; // in 4-byte words
    int32_t *rmap;        // table region -> join
    int64_t rmap_cap;
};

__device__ inline void asj_batch_prep_run(const asj_batch_prep &p, int64_t block, int64_t nblocks, int tid,
                                          int nthreads)
{
    if (p.rmatch)
        for (int64_t i = block * nthreads + tid; i < p.rmatch_words; i += nblocks * nthreads) p.rmatch[i] = 0u;
    const int64_t nr = p.win_r_cap < (int64_t)p.tot[1] ? p.win_r_cap : (int64_t)p.tot[1];
    const int64_t ns = p.win_s_cap < (int64_t)p.tot[2] ? p.win_s_cap : (int64_t)p.tot[2];
    const int64_t nl = p.win_l_cap < (int64_t)p.tot[3] ? p.win_l_cap : (int64_t)p.tot[3];
    const int64_t nq = p.rmap_cap < (int64_t)p.tot[4] ? p.rmap_cap : (int64_t)p.tot[4];
    for (int64_t j = block; j < p.njoins; j += nblocks) {
        const asj_join_desc d = p.desc[j];
        const int64_t r1 = j + 1 < p.njoins ? p.desc[j + 1].wbase_r : nr;
        const int64_t s1 = j + 1 < p.njoins ? p.desc[j + 1].wbase : ns;
        const int64_t l1 = j + 1 < p.njoins ? p.desc[j + 1].wbase_l : nl;
        const int64_t q1 = j + 1 < p.njoins ? p.desc[j + 1].rbase : nq;
        const int64_t first = p.s_seg[j], end = p.s_seg[j + 1];
        for (int64_t w = d.wbase_r + tid; w < (r1 < nr ? r1 : nr); w += nthreads) p.win_r[w] = (int32_t)j;
        for (int64_t q = d.rbase + tid; q < (q1 < nq ? q1 : nq); q += nthreads) p.rmap[q] = (int32_t)j;
        for (int64_t w = d.wbase_l + tid; w < (l1 < nl ? l1 : nl); w += nthreads) p.win_l[w] = (int32_t)j;
        for (int64_t w = d.wbase + tid; w < (s1 < ns ? s1 : ns); w += nthreads) {
            asj_win e;
            e.join = (int32_t)j;
            e.first = first + (w - d.wbase) * p.kpw;
            const int64_t left = end - e.first;
            e.rows = (int32_t)(left < p.kpw ? left : p.kpw);
            p.win_s[w] = e;
        }
    }
}

struct asj_probe_args {
    const uint8_t *rdata;
    const int64_t *roff;
    const int32_t *rids;
    int64_t rn; // build rows (roff[rn] is the end of the build arena)
    const uint8_t *sdata;
    const int64_t *soff;
    const int32_t *sids;
    int64_t n;
    const uint32_t *ssig; // signatures (plain hashes) of the probe keys, or NULL to sign them in the kernel
    const uint32_t *rsig_hi; // four GF(2^16) components: high words (components 3, 4) of the build rows
    const uint64_t *slots;
    uint64_t mask;
    asj_pair *out;
    int64_t cap;
    int64_t *out_count;
    int64_t *cand_count;
    const int32_t *table_status; // device; non-zero means the build failed
    const int32_t *probe_status; // device or NULL; non-zero means the probe relation failed validation
    int plain;
    int verify;
    int keys_per_window; // probe keys per wave window (1..64)
    int grid_rounds;     // > 0: grid = grid_rounds x the kernel's resident blocks (capped by grid_cap)
    int kind;            // ASJ_KIND_*: inner, semi, anti, left, right or full outer join
    uint8_t *rmatch;     // right and full outer joins: one byte per build row, zeroed; set for matched rows
    // batch of joins (njoins > 0): probe row k belongs to join j with
    // s_seg[j] <= k < s_seg[j+1]; its table is slots[desc[j].tbase ..] with
    // mask desc[j].mask, its output out[out_seg[j] .. out_seg[j+1]) and its
    // counters out_count[j], cand_count[j].  Window w (w < min(*nwin,
    // nwin_cap)) is wins[w]: rows first .. first + rows of join wins[w].join.
    int32_t njoins;
    const int64_t *s_seg;
    const asj_join_desc *desc;
    const asj_win *wins;
    const uint64_t *nwin;
    int64_t nwin_cap;
    const int64_t *out_seg;
    int64_t *rows_done;   // int64[njoins], zeroed: probe rows finished per join (kept when done_clock is set)
    uint64_t *done_clock; // uint64[njoins] or NULL
    // joins with LDS tables: their probe windows are numbered apart, window w
    // (w < min(*nwin_l, nwin_l_cap)) belongs to join win_l[w], whose build
    // rows r_seg[j] .. r_seg[j+1] have signatures rsig[..]
    const int32_t *win_l;
    const uint64_t *nwin_l;
    int64_t nwin_l_cap;
    const int64_t *r_seg;
    const uint32_t *rsig;
};
// Signs the probe keys and probes/verifies/compacts in one kernel.
hipError_t asj_launch_probe(const asj_probe_args *a, int mode, int nsym, const uint16_t *tab, int grid_cap,
                            hipStream_t st);
// A single join whose a->rn <= ASJ_LOCAL_ROWS build rows have signatures
// a->rsig: every probing block builds the LDS table itself (no device-memory
// table); a->table_status must point to a cleared status word.
hipError_t asj_launch_probe_local_single(const asj_probe_args *a, int mode, int nsym, const uint16_t *tab,
                                         hipStream_t st);
// Clears the counters (b and c may be NULL), sets *status = ASJ_OK and clears
// words[0 .. nwords) (may be NULL), in one launch.
hipError_t asj_launch_local_init(int64_t *a, int64_t *b, int32_t *status, uint32_t *words, int64_t nwords,
                                 hipStream_t st, int64_t *c = nullptr);
// Right and full outer joins: (r_id, -1) for every build row r < m with
// rmatch[r] == 0, appended to the output like the probe kernel's pairs.
// Batch (njoins > 0): row r belongs to join j with r_seg[j] <= r <
// r_seg[j+1] and goes to out[out_seg[j] ..] with out_count[j].  Nothing
// happens when a status word is set (the probe then reported -1).
hipError_t asj_launch_unmatched_build(const uint8_t *rmatch, const int32_t *rids, int64_t m, asj_pair *out, int64_t cap,
                                      int64_t *out_count, const int32_t *status1, const int32_t *status2,
                                      int32_t njoins, const int64_t *r_seg, const int64_t *out_seg, hipStream_t st);
// Batches with LDS tables: the probe windows of every join, those with
// device-memory tables (a->wins ..) and those with LDS tables (a->win_l ..),
// in one launch of grid_rounds x the kernel's resident blocks.
hipError_t asj_launch_probe_local(const asj_probe_args *a, int mode, int nsym, const uint16_t *tab, hipStream_t st);
hipError_t asj_launch_copy(void *dst, const void *src, int64_t bytes, hipStream_t st);
// Sorts pairs[0 .. min(*count, cap)) by (r_id, s_id); scratch holds
// asj_sort_scratch_bytes(cap) device bytes.
size_t asj_sort_scratch_bytes(int64_t cap);
hipError_t asj_launch_sort_pairs(asj_pair *pairs, const int64_t *count, int64_t cap, void *scratch, hipStream_t st);
hipError_t asj_launch_read(const void *src, int64_t bytes, uint32_t *out, int grid, hipStream_t st);

// Batch: per-join segment plan (capacities, prefix offsets, counters, start
// clock), the preparation (window and region maps), the build by regions.
// tot[0] = slots of all segments, tot[1] = build windows, tot[2] = probe
// windows, tot[3] = LDS-table probe windows, tot[4] = table regions (of
// asj_seg_region_bits slots each); win_r / win_s map windows to joins.  With
// rcnt, the plan also clears rcnt[0 .. tot[4]) (at most rcnt_cap words) and
// *novf, the region counts and overflow count of a build by regions.
hipError_t asj_launch_batch_plan(const int64_t *r_seg, const int64_t *s_seg, int32_t njoins, int64_t n_r, int64_t n_s,
                                 int64_t slot_cap, float load_factor, int keys_per_window, int64_t local_rows,
                                 int local_only, asj_join_desc *desc, int64_t *rows_done, int64_t *out_count, int64_t *cand_count,
                                 uint64_t *done_clock, uint64_t *tot, int32_t *status, uint32_t *rcnt, int64_t rcnt_cap,
                                 uint64_t *novf, hipStream_t st);
hipError_t asj_launch_batch_prep(const asj_batch_prep *p, hipStream_t st);
// The batch's segments built by regions, as a single table of 327680 rows or
// more is (every slot written, so no fill): the build rows' words scattered
// into their home regions (a block per 64 build windows), every region
// (rmap: region -> join, written by the preparation) built in LDS and
// written whole, then the rows that left their region.  rcnt and *novf must
// be zero (the plan clears them); ovf holds m words.
hipError_t asj_launch_region_build_batch(const uint32_t *sig, int64_t m, const int64_t *r_seg, int32_t njoins,
                                         const asj_join_desc *desc, const int32_t *win_r, const uint64_t *tot,
                                         int64_t win_r_cap, const int32_t *rmap, int64_t rmap_cap, uint32_t *rcnt,
                                         uint64_t *ovf, uint64_t *novf, uint64_t *slots, int32_t *status,
                                         hipStream_t st);
