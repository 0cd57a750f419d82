// Host side of the libasjoin C interface: argument checks, stream-ordered
// allocation, kernel launches and error mapping.  Every step of the join
// runs in the library's own kernels (sign.hip, table.hip, probe.hip).
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "asj_internal.h"

namespace {

constexpr int kMaxDevices = 64;
constexpr int kSignGridCap = 256 * 16;  // blocks; the sign kernel loops over windows
constexpr int kProbeGridCap = 256 * 16;

struct DeviceState {
    uint16_t *tab = nullptr;    // GF constant tables: this device's copy of gf_tab
    uint8_t *scratch = nullptr; // asj_join_noalloc's scratch: this device's copy of `scratch`
    bool ready = false;
};

// Both arrays live in the code object, so every device that loads the
// library holds a copy of each until the process ends and the library never
// allocates them.  Host code reaches them only through the per-device
// addresses that hipGetSymbolAddress returns at initialisation (the names
// themselves are host-side stand-ins, not device addresses).
static __device__ __align__(256) uint16_t gf_tab[ASJ_TAB_TOTAL_WORDS];
// Scratch of asj_join_noalloc: status word, build signatures, probe status
// word and right-outer marks of one join with at most
// ASJ_NOALLOC_MAX_BUILD_ROWS build rows (layout: noalloc_layout).
static __device__ __align__(256) uint8_t scratch[ASJ_NOALLOC_SCRATCH_BYTES];
static_assert(ASJ_NOALLOC_MAX_BUILD_ROWS == ASJ_LOCAL_ROWS, "asj_join_noalloc takes the LDS-table path only");
// status word, signatures, probe status word, right-outer marks (local_layout) at the row limit
static_assert(256 + ((4 * ASJ_NOALLOC_MAX_BUILD_ROWS + 255) / 256 * 256) + 256 +
                      ((ASJ_NOALLOC_MAX_BUILD_ROWS + 255) / 256 * 256) <=
                  ASJ_NOALLOC_SCRATCH_BYTES,
              "scratch too small for the largest build side");

std::mutex g_mu;
DeviceState g_dev[kMaxDevices];

// ---- per-thread kernel timing (measurement support) ----
// While timing is on, every kernel phase launched by this thread is
// bracketed by two events on its stream; records accumulate until
// asj_timing_read() collects them.
constexpr int kMaxTimed = 4096;
struct Timing {
    bool on = false;
    int count = 0;
    hipEvent_t ev[2 * kMaxTimed] = {};
    const char *names[kMaxTimed] = {};
};
thread_local Timing g_tim;

struct TimingScope { // kept for call-site symmetry; records are never reset here
    TimingScope() {}
};

void tim_begin(const char *name, hipStream_t st)
{
    if (!g_tim.on || g_tim.count >= kMaxTimed) return;
    int i = g_tim.count;
    // timing-only events: no system-scope fence (no cache writeback and
    // invalidation between the kernels they bracket)
    for (int e = 0; e < 2; e++)
        if (!g_tim.ev[2 * i + e]) (void)hipEventCreateWithFlags(&g_tim.ev[2 * i + e], hipEventDisableSystemFence);
    g_tim.names[i] = name;
    (void)hipEventRecord(g_tim.ev[2 * i], st);
}

void tim_end(hipStream_t st)
{
    if (!g_tim.on || g_tim.count >= kMaxTimed) return;
    (void)hipEventRecord(g_tim.ev[2 * g_tim.count + 1], st);
    g_tim.count++;
}

int hip_fail(hipError_t e)
{
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return ASJ_ENOMEM;
    return ASJ_EHIP;
}

#define TIMED(name, stmt)                      \
    do {                                       \
        tim_begin(name, st);                   \
        hipError_t e_ = (stmt);                \
        tim_end(st);                           \
        if (e_ != hipSuccess) return hip_fail(e_); \
    } while (0)

int ensure_init(int *dev_out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return ASJ_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return ASJ_EHIP;
    *dev_out = dev;
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceState &d = g_dev[dev];
    if (d.ready) return ASJ_OK;
    // this device's copies of the two arrays (the device is current here)
    uint16_t *tab = nullptr;
    uint8_t *scr = nullptr;
    if (hipGetSymbolAddress((void **)&tab, HIP_SYMBOL(gf_tab)) != hipSuccess || !tab) return ASJ_EHIP;
    if (hipGetSymbolAddress((void **)&scr, HIP_SYMBOL(scratch)) != hipSuccess || !scr) return ASJ_EHIP;
    if (asj_launch_tables(tab, 0) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return ASJ_EHIP;
    // keep freed stream-ordered blocks cached in the default pool
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    d.tab = tab;
    d.scratch = scr;
    d.ready = true;
    return ASJ_OK;
}

bool keys_ok(const asj_keys *k)
{
    if (!k || k->n < 0 || k->n >= (int64_t)INT32_MAX) return false;
    if (k->n > 0 && !k->offsets) return false;
    return true;
}

int resolve_sig(asj_sig_params p, asj_sig_params *out)
{
    if (p.f == 0 && p.nsym == 0) p = asj_sig_params{16, 2};
    if (p.f == 16 && (p.nsym == 1 || p.nsym == 2 || p.nsym == 4)) {
        *out = p;
        return ASJ_OK;
    }
    if (p.f == 8 && (p.nsym == 2 || p.nsym == 4)) {
        *out = p;
        return ASJ_OK;
    }
    if (p.f != 8 && p.f != 16) return ASJ_EINVAL;
    if (p.nsym < 1 || p.f * p.nsym > 64) return ASJ_EINVAL;
    return ASJ_EUNSUPPORTED;
}

// Join kind from the flags; -1 when more than one is set.
int join_kind(uint32_t flags)
{
    const bool semi = flags & ASJ_SEMI, anti = flags & ASJ_ANTI;
    const bool left = flags & ASJ_LEFT_OUTER, right = flags & ASJ_RIGHT_OUTER;
    if ((int)semi + (int)anti + (int)(left || right) > 1) return -1;
    if (semi) return ASJ_KIND_SEMI;
    if (anti) return ASJ_KIND_ANTI;
    if (left && right) return ASJ_KIND_FULL;
    if (left) return ASJ_KIND_LEFT;
    if (right) return ASJ_KIND_RIGHT;
    return ASJ_KIND_INNER;
}

// Table load factor, probe keys per window and probe schedule (1 = split:
// sign kernel, then a probe kernel with the stored signatures; 0 = fused)
// for options that may leave them to the library: a value the caller set
// wins, then the autotuner's record for this size class, then the defaults
// (0.5, 64, fused -- fused was faster on every measured workload).
// ASJ_EINVAL for contradictory schedule flags or a load factor >= 1.
int resolve_auto(int batch, int64_t n_build, const asj_opts &o, float *lf, int *kpw, int *split, int *rounds)
{
    const bool fused = (o.flags & ASJ_PROBE_FUSED) != 0, sp = (o.flags & ASJ_PROBE_SPLIT) != 0;
    if (fused && sp) return ASJ_EINVAL;
    asj_tuned t = {};
    const bool tuned = asj_tuned_lookup(batch, n_build, o, &t);
    *lf = o.load_factor > 0.0f ? o.load_factor : (tuned ? t.load_factor : 0.5f);
    if (!(*lf > 0.0f && *lf < 1.0f)) return ASJ_EINVAL;
    *kpw = (o.keys_per_window >= 1 && o.keys_per_window <= ASJ_WAVE)
               ? o.keys_per_window
               : (tuned ? t.keys_per_window : ASJ_DEFAULT_KEYS_PER_WINDOW);
    *split = fused ? 0 : sp ? 1 : (tuned ? t.split : 0);
    *rounds = (o.grid_rounds >= 1 && o.grid_rounds <= 8) ? o.grid_rounds : (tuned ? t.grid_rounds : 2);
    if (o.grid_rounds > 8) return ASJ_EINVAL;
    return ASJ_OK;
}

// out_hi / stride: see asj_launch_sign (four GF(2^16) components only).
// kpw: the join's keys per window, also used for signing (see sign.hip).
hipError_t launch_sign_for(const asj_keys *k, asj_sig_params sig, int plain, uint32_t *out, const uint16_t *tab,
                           hipStream_t st, const int32_t *status = nullptr, uint32_t *out_hi = nullptr,
                           int stride = 1, const asj_batch_prep *prep = nullptr, int kpw = ASJ_WAVE)
{
    if (plain)
        return asj_launch_sign(ASJ_MODE_PLAIN, 1, k, out, tab, kSignGridCap, st, status, nullptr, 1, prep, kpw);
    return asj_launch_sign(sig.f == 16 ? ASJ_MODE_SIG16 : ASJ_MODE_SIG8, sig.nsym, k, out, tab, kSignGridCap, st,
                           status, out_hi, stride, prep, kpw);
}

bool sig64(asj_sig_params s) { return s.f == 16 && s.nsym == 4; }

template <typename T>
hipError_t alloc_async(T **p, size_t count, hipStream_t st)
{
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMallocAsync((void **)p, sizeof(T) * count, st);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// zc0, zc1 (may be NULL): counters of a probe that follows on the stream,
// cleared by the build's first launch (asj_join: one launch fewer).
int build_impl(const asj_keys *r, const asj_opts *opts, asj_table **table_out, hipStream_t st,
               int64_t *zc0 = nullptr, int64_t *zc1 = nullptr)
{
    if (!table_out || !keys_ok(r)) return ASJ_EINVAL;
    *table_out = nullptr;
    asj_opts o = {};
    if (opts) o = *opts;
    const int plain = (o.flags & ASJ_PLAIN) != 0;
    const int verify = (o.flags & ASJ_NO_VERIFY) == 0;
    const int fp = (o.flags & ASJ_FINGERPRINT) != 0;
    if (plain && !verify) return ASJ_EINVAL; // the plain table has no signature to trust
    if (fp && (plain || !verify)) return ASJ_EINVAL;
    if (join_kind(o.flags) < 0) return ASJ_EINVAL;
    asj_sig_params sig = {16, 2};
    if (!plain) {
        int rc = resolve_sig(o.sig, &sig);
        if (rc != ASJ_OK) return rc;
    }
    float lf;
    int kpw, split, rounds;
    if (resolve_auto(0, r->n, o, &lf, &kpw, &split, &rounds) != ASJ_OK) return ASJ_EINVAL;
    const bool wide = !plain && !fp && sig64(sig);
    if (wide) { // 64-bit signatures: the fused probe schedule only
        if (o.flags & ASJ_PROBE_SPLIT) return ASJ_EUNSUPPORTED;
        split = 0;
    }
    int dev = 0;
    int rc = ensure_init(&dev);
    if (rc != ASJ_OK) return rc;

    int64_t cap = 64;
    while ((double)cap * lf < (double)r->n) cap <<= 1;

    asj_table *t = (asj_table *)calloc(1, sizeof(asj_table));
    if (!t) return ASJ_ENOMEM;
    t->r = *r;
    t->capacity = cap;
    t->plain = plain;
    t->fp = fp;
    t->verify = verify;
    t->sig = sig;
    t->keys_per_window = kpw;
    t->grid_rounds = rounds;
    t->split = split;
    t->sorted = (o.flags & ASJ_SORTED) != 0;
    t->validate = (o.flags & ASJ_VALIDATE) != 0;
    t->kind = join_kind(o.flags);
    t->stream = st;
    t->device = dev;
    // one stream-ordered allocation: slots | status | signatures (low, high
    // words) | region-build scratch
    const size_t o_status = align256(8 * (size_t)cap);
    const size_t o_sig = align256(o_status + 4);
    const size_t o_hi = align256(o_sig + 4 * (size_t)(r->n > 0 ? r->n : 1));
    const size_t o_reg = wide ? align256(o_hi + 4 * (size_t)(r->n > 0 ? r->n : 1)) : o_hi;
    // the table built by regions when it fits their limits (their scratch
    // after the signatures), else by the two-pass insert
    const int64_t region_bytes = asj_region_scratch_bytes(r->n, cap);
    const size_t bytes = region_bytes > 0 ? o_reg + (size_t)region_bytes : o_reg;
    hipError_t e = hipMallocAsync(&t->block, bytes, st);
    if (e != hipSuccess) {
        free(t);
        return hip_fail(e);
    }
    uint8_t *blk = (uint8_t *)t->block;
    t->slots = (uint64_t *)blk;
    t->status = (int32_t *)(blk + o_status);
    uint32_t *sig_r = (uint32_t *)(blk + o_sig);
    t->sig_hi = wide ? (uint32_t *)(blk + o_hi) : nullptr;
    void *region = region_bytes > 0 ? (void *)(blk + o_reg) : nullptr;
    int out_rc = ASJ_OK;
    do {
        hipError_t le;
        tim_begin("table_init", st);
        le = region ? asj_launch_region_init(region, r->n, cap, t->status, st, zc0, zc1)
                    : asj_launch_table_init(t->slots, cap, t->status, st, zc0, zc1);
        if (le == hipSuccess && t->validate) le = asj_launch_validate(r->offsets, r->n, t->status, st);
        tim_end(st);
        if (le != hipSuccess) { out_rc = hip_fail(le); break; }
        tim_begin(plain ? "hash_build" : fp ? "fp_build" : "sign_build", st);
        le = launch_sign_for(r, sig, plain || fp, sig_r, g_dev[dev].tab, st, t->status, t->sig_hi, 1, nullptr,
                             0 /* windows sized by the kernel */);
        tim_end(st);
        if (le != hipSuccess) { out_rc = hip_fail(le); break; }
        tim_begin("insert", st);
        le = region ? asj_launch_region_build(sig_r, r->n, plain, t->slots, cap, t->status, region, st)
                    : asj_launch_insert(sig_r, r->n, plain, t->slots, (uint64_t)cap - 1, t->status, st);
        tim_end(st);
        if (le != hipSuccess) { out_rc = hip_fail(le); break; }
    } while (0);
    if (out_rc != ASJ_OK) {
        (void)hipFreeAsync(t->block, st);
        free(t);
        return out_rc;
    }
    *table_out = t;
    return ASJ_OK;
}

int probe_unsorted(const asj_table *t, const asj_keys *s, asj_pair *out, int64_t out_cap, int64_t *out_count,
                   int64_t *cand_count, hipStream_t st, bool zeroed);

// zeroed: the counters were cleared earlier on the stream (by the build).
int probe_impl(const asj_table *t, const asj_keys *s, asj_pair *out, int64_t out_cap, int64_t *out_count,
               int64_t *cand_count, hipStream_t st, bool zeroed = false)
{
    int rc = probe_unsorted(t, s, out, out_cap, out_count, cand_count, st, zeroed);
    if (rc != ASJ_OK || !t->sorted || out_cap == 0) return rc;
    void *sort_tmp = nullptr;
    hipError_t e = hipMallocAsync(&sort_tmp, asj_sort_scratch_bytes(out_cap), st);
    if (e != hipSuccess) return hip_fail(e);
    tim_begin("sort", st);
    e = asj_launch_sort_pairs(out, out_count, out_cap, sort_tmp, st);
    tim_end(st);
    (void)hipFreeAsync(sort_tmp, st);
    return e == hipSuccess ? ASJ_OK : hip_fail(e);
}

int probe_unsorted(const asj_table *t, const asj_keys *s, asj_pair *out, int64_t out_cap, int64_t *out_count,
                   int64_t *cand_count, hipStream_t st, bool zeroed)
{
    if (!t || !keys_ok(s) || !out_count || out_cap < 0 || (out_cap > 0 && !out)) return ASJ_EINVAL;
    int dev = 0;
    int rc = ensure_init(&dev);
    if (rc != ASJ_OK) return rc;
    hipError_t e = zeroed ? hipSuccess : asj_launch_zero2(out_count, cand_count, st);
    if (e != hipSuccess) return hip_fail(e);
    asj_probe_args a = {};
    a.rdata = t->r.data;
    a.roff = t->r.offsets;
    a.rids = t->r.ids;
    a.rn = t->r.n;
    a.keys_per_window = t->keys_per_window;
    a.sdata = s->data;
    a.soff = s->offsets;
    a.sids = s->ids;
    a.n = s->n;
    a.slots = t->slots;
    a.mask = (uint64_t)t->capacity - 1;
    a.rsig_hi = t->sig_hi;
    a.out = out;
    a.cap = out_cap;
    a.out_count = out_count;
    a.cand_count = cand_count;
    a.table_status = t->status;
    a.grid_rounds = t->grid_rounds;
    a.plain = t->plain;
    a.verify = t->verify;
    a.kind = t->kind;
    const int mode = (t->plain || t->fp) ? ASJ_MODE_PLAIN : (t->sig.f == 16 ? ASJ_MODE_SIG16 : ASJ_MODE_SIG8);
    const int nsym = (t->plain || t->fp) ? 1 : t->sig.nsym;
    int32_t *pstatus = nullptr; // validation result of the probe relation
    if (t->validate && s->n > 0) {
        e = alloc_async(&pstatus, 1, st);
        if (e == hipSuccess) e = asj_launch_fill_i32(pstatus, 1, 0, st);
        if (e == hipSuccess) e = asj_launch_validate(s->offsets, s->n, pstatus, st);
        if (e != hipSuccess) {
            if (pstatus) (void)hipFreeAsync(pstatus, st);
            return hip_fail(e);
        }
        a.probe_status = pstatus;
    }
    // right and full outer joins: a byte per build row, set by the probe
    // for the matched rows; the others are appended after the probe
    uint8_t *rmatch = nullptr;
    if (asj_kind_marks_build(t->kind) && t->r.n > 0) {
        const int64_t words = (t->r.n + 3) / 4;
        e = alloc_async(&rmatch, (size_t)words * 4, st);
        if (e == hipSuccess) e = asj_launch_fill_i32((int32_t *)rmatch, words, 0, st);
        if (e != hipSuccess) {
            if (rmatch) (void)hipFreeAsync(rmatch, st);
            if (pstatus) (void)hipFreeAsync(pstatus, st);
            return hip_fail(e);
        }
        a.rmatch = rmatch;
    }
    uint32_t *ssig = nullptr;
    if (!t->split || s->n == 0) {
        tim_begin(t->plain ? "hash_probe_verify" : t->fp ? "fp_probe_verify" : "sign_probe_verify", st);
        e = asj_launch_probe(&a, mode, nsym, g_dev[dev].tab, kProbeGridCap, st);
        tim_end(st);
    } else {
        e = alloc_async(&ssig, (size_t)s->n, st);
        if (e == hipSuccess) {
            tim_begin(t->plain ? "hash_S" : t->fp ? "fp_S" : "sign_S", st);
            e = launch_sign_for(s, t->sig, t->plain || t->fp, ssig, g_dev[dev].tab, st, pstatus, nullptr, 1, nullptr,
                                t->keys_per_window);
            tim_end(st);
        }
        if (e == hipSuccess) {
            a.ssig = ssig;
            tim_begin(t->plain ? "hash_probe_verify" : "probe_verify", st);
            e = asj_launch_probe(&a, mode, nsym, g_dev[dev].tab, kProbeGridCap, st);
            tim_end(st);
        }
        if (ssig) (void)hipFreeAsync(ssig, st);
    }
    if (e == hipSuccess && rmatch) {
        tim_begin("unmatched_build", st);
        e = asj_launch_unmatched_build(rmatch, t->r.ids, t->r.n, out, out_cap, out_count, t->status, pstatus, 0,
                                       nullptr, nullptr, st);
        tim_end(st);
    }
    if (rmatch) (void)hipFreeAsync(rmatch, st);
    if (pstatus) (void)hipFreeAsync(pstatus, st);
    return e == hipSuccess ? ASJ_OK : hip_fail(e);
}

int table_free_impl(asj_table *t)
{
    if (!t) return ASJ_OK;
    const hipError_t e = hipFreeAsync(t->block, t->stream);
    free(t);
    return e == hipSuccess ? ASJ_OK : ASJ_EHIP;
}

// ---- batch workspace layout (each part 256-byte aligned) ----
struct BatchLayout {
    size_t desc, rows_done, tot, status, win_r, win_s, win_l, rmatch, sig, ssig, slots, rcnt, rmap, novf, ovf, bytes;
    int64_t slot_bound, win_r_cap, win_s_cap, region_cap;
};

// local_only: every join has an LDS table, so no device table is built and
// the layout holds no region-build scratch.
bool batch_layout(int32_t J, int64_t n_build, int64_t n_probe, int kpw, float lf, BatchLayout *L,
                  bool local_only = false)
{
    if (J < 1 || n_build < 0 || n_probe < 0 || kpw < 1 || !(lf > 0.0f && lf < 1.0f)) return false;
    // every segment has capacity 64 or less than 2 |R_j| / lf
    L->slot_bound = 64 * (int64_t)J + (int64_t)(2.0 * (double)n_build / lf) + 1;
    // sum over joins of ceil(rows_j / w) <= rows / w + J
    L->win_r_cap = n_build / ASJ_WAVE + J + 1;
    L->win_s_cap = n_probe / kpw + J + 1;
    // table regions of 64 slots or more each
    L->region_cap = local_only ? 0 : L->slot_bound / 64 + 1;
    size_t off = 0;
    L->desc = off;
    off = align256(off + sizeof(asj_join_desc) * (size_t)J);
    L->rows_done = off;
    off = align256(off + sizeof(int64_t) * (size_t)J);
    L->tot = off;
    off = align256(off + 5 * sizeof(uint64_t));
    L->status = off;
    off = align256(off + sizeof(int32_t));
    L->win_r = off;
    off = align256(off + sizeof(int32_t) * (size_t)L->win_r_cap);
    L->win_s = off;
    off = align256(off + sizeof(asj_win) * (size_t)L->win_s_cap);
    L->win_l = off; // LDS-table probe windows: at most as many as probe windows
    off = align256(off + sizeof(int32_t) * (size_t)L->win_s_cap);
    L->rmatch = off; // right and full outer joins: a byte per build row
    off = align256(off + 4 * (size_t)((n_build + 3) / 4));
    L->sig = off;
    off = align256(off + sizeof(uint32_t) * (size_t)(n_build > 0 ? n_build : 1));
    L->ssig = off;
    off = align256(off + sizeof(uint32_t) * (size_t)(n_probe > 0 ? n_probe : 1));
    L->slots = off;
    off = align256(off + sizeof(uint64_t) * (size_t)L->slot_bound);
    // build by regions: region counts, region -> join, overflow count and list
    L->rcnt = off;
    off = align256(off + sizeof(uint32_t) * (size_t)L->region_cap);
    L->rmap = off;
    off = align256(off + sizeof(int32_t) * (size_t)L->region_cap);
    L->novf = off;
    off = align256(off + sizeof(uint64_t));
    L->ovf = off;
    if (!local_only) off = align256(off + sizeof(uint64_t) * (size_t)(n_build > 0 ? n_build : 1));
    L->bytes = off;
    return true;
}

int batch_opts(const asj_opts *opts, int64_t n_build, int *plain, int *verify, asj_sig_params *sig, float *lf,
               int *kpw, int *split, int *validate = nullptr, int *kind = nullptr, int *rounds_out = nullptr,
               int *local_out = nullptr, int *local_only_out = nullptr)
{
    int rounds_local = 2;
    int *rounds = rounds_out ? rounds_out : &rounds_local;
    asj_opts o = {};
    if (opts) o = *opts;
    *plain = (o.flags & ASJ_PLAIN) != 0;
    *verify = (o.flags & ASJ_NO_VERIFY) == 0;
    if (*plain && !*verify) return ASJ_EINVAL;
    if (o.flags & (ASJ_SORTED | ASJ_FINGERPRINT)) return ASJ_EUNSUPPORTED;
    if (validate) *validate = (o.flags & ASJ_VALIDATE) != 0;
    if (local_out) *local_out = (o.flags & ASJ_GLOBAL_TABLES) == 0;
    const int local_only = (o.flags & ASJ_LOCAL_ONLY) != 0;
    if (local_only && (o.flags & (ASJ_GLOBAL_TABLES | ASJ_PROBE_SPLIT))) return ASJ_EINVAL;
    if (local_only_out) *local_only_out = local_only;
    const int k = join_kind(o.flags);
    if (k < 0) return ASJ_EINVAL;
    if (kind) *kind = k;
    *sig = asj_sig_params{16, 2};
    if (!*plain) {
        int rc = resolve_sig(o.sig, sig);
        if (rc != ASJ_OK) return rc;
        if (sig64(*sig)) return ASJ_EUNSUPPORTED; // 64-bit signatures: single joins only
    }
    const int rc = resolve_auto(1, n_build, o, lf, kpw, split, rounds);
    if (local_only) *split = 0; // LDS tables need the fused schedule (an explicit split was refused above)
    return rc;
}

} // namespace

int asj_resolve_opts(const asj_opts *opts, int64_t n_build, asj_resolved *r)
{
    asj_opts o = {};
    if (opts) o = *opts;
    r->plain = (o.flags & ASJ_PLAIN) != 0;
    r->verify = (o.flags & ASJ_NO_VERIFY) == 0;
    if (r->plain && !r->verify) return ASJ_EINVAL;
    if (o.flags & ASJ_FINGERPRINT) return ASJ_EUNSUPPORTED; // single joins only
    r->kind = join_kind(o.flags);
    if (r->kind < 0) return ASJ_EINVAL;
    if (asj_kind_marks_build(r->kind)) return ASJ_EUNSUPPORTED; // right / full outer: asj_join, asj_probe, batches
    r->sig = asj_sig_params{16, 2};
    if (!r->plain) {
        const int rc = resolve_sig(o.sig, &r->sig);
        if (rc != ASJ_OK) return rc;
        if (sig64(r->sig)) return ASJ_EUNSUPPORTED; // 64-bit signatures: asj_join / asj_probe only
    }
    return resolve_auto(0, n_build, o, &r->lf, &r->kpw, &r->split, &r->grid_rounds);
}

const uint16_t *asj_device_tables(int *dev)
{
    int d = 0;
    if (ensure_init(&d) != ASJ_OK) return nullptr;
    if (dev) *dev = d;
    return g_dev[d].tab;
}

namespace {

constexpr int kNotLocal = 1; // join_local_single: not this path

// asj_join with at most ASJ_LOCAL_ROWS build rows: the build keys are signed
// into a scratch array and every probing block builds the table in LDS (no
// device-memory table, no insert).  Returns kNotLocal when the options ask
// for a path it does not take (device-memory tables, the split schedule,
// 64-bit signatures, the fingerprint control).
// Scratch layout of one such join: status word | build signatures | probe
// status word | right-outer marks, each part 256-byte aligned.
struct LocalLayout {
    size_t sig, pst, rm, bytes;
};
LocalLayout local_layout(int64_t n_build, int64_t rwords)
{
    LocalLayout L;
    L.sig = 256;
    L.pst = align256(L.sig + 4 * (size_t)(n_build > 0 ? n_build : 1));
    L.rm = align256(L.pst + 4);
    L.bytes = align256(L.rm + 4 * (size_t)(rwords > 0 ? rwords : 1));
    return L;
}

// fixed: the caller's scratch (asj_join_noalloc: nothing is allocated,
// ASJ_SORTED is refused); NULL: one stream-ordered allocation.
int join_local_single(const asj_keys *r, const asj_keys *s, const asj_opts *opts, asj_pair *out, int64_t out_cap,
                      int64_t *out_count, int64_t *cand_count, hipStream_t st, uint8_t *fixed = nullptr)
{
    if (!keys_ok(r) || r->n > ASJ_LOCAL_ROWS) return kNotLocal;
    asj_opts o = {};
    if (opts) o = *opts;
    if (o.flags & (ASJ_GLOBAL_TABLES | ASJ_FINGERPRINT)) return kNotLocal;
    const int plain = (o.flags & ASJ_PLAIN) != 0;
    const int verify = (o.flags & ASJ_NO_VERIFY) == 0;
    if (plain && !verify) return kNotLocal; // the regular path reports the error
    const int kind = join_kind(o.flags);
    if (kind < 0) return kNotLocal;
    asj_sig_params sig = {16, 2};
    if (!plain && resolve_sig(o.sig, &sig) != ASJ_OK) return kNotLocal;
    if (!plain && sig64(sig)) return kNotLocal;
    float lf;
    int kpw, split, rounds;
    if (resolve_auto(0, r->n, o, &lf, &kpw, &split, &rounds) != ASJ_OK || split) return kNotLocal;
    int dev = 0;
    int rc = ensure_init(&dev);
    if (rc != ASJ_OK) return rc;
    const bool marks = asj_kind_marks_build(kind);
    const int64_t rwords = marks ? (r->n + 3) / 4 : 0;
    const LocalLayout L = local_layout(r->n, rwords);
    uint8_t *blk = fixed;
    hipError_t e = hipSuccess;
    if (fixed) {
        if (L.bytes > ASJ_NOALLOC_SCRATCH_BYTES || (o.flags & ASJ_SORTED)) return ASJ_EINVAL;
    } else {
        e = hipMallocAsync((void **)&blk, L.bytes, st);
        if (e != hipSuccess) return hip_fail(e);
    }
    int32_t *status = (int32_t *)blk;
    uint32_t *sig_r = (uint32_t *)(blk + L.sig);
    int32_t *pstatus = (int32_t *)(blk + L.pst);
    uint8_t *rmatch = marks ? blk + L.rm : nullptr;
    const int validate = (o.flags & ASJ_VALIDATE) != 0;
    int out_rc = ASJ_OK;
    do {
        tim_begin("table_init", st);
        e = asj_launch_local_init(out_count, cand_count, status, (uint32_t *)rmatch, rwords, st);
        if (e == hipSuccess && validate) {
            e = asj_launch_fill_i32(pstatus, 1, 0, st);
            if (e == hipSuccess) e = asj_launch_validate(r->offsets, r->n, status, st);
            if (e == hipSuccess && s->n > 0) e = asj_launch_validate(s->offsets, s->n, pstatus, st);
        }
        tim_end(st);
        if (e != hipSuccess) { out_rc = hip_fail(e); break; }
        tim_begin(plain ? "hash_build" : "sign_build", st);
        e = launch_sign_for(r, sig, plain, sig_r, g_dev[dev].tab, st, status, nullptr, 1, nullptr, 0);
        tim_end(st);
        if (e != hipSuccess) { out_rc = hip_fail(e); break; }
        asj_probe_args a = {};
        a.rdata = r->data;
        a.roff = r->offsets;
        a.rids = r->ids;
        a.rn = r->n;
        a.rsig = sig_r;
        a.keys_per_window = kpw;
        a.sdata = s->data;
        a.soff = s->offsets;
        a.sids = s->ids;
        a.n = s->n;
        a.out = out;
        a.cap = out_cap;
        a.out_count = out_count;
        a.cand_count = cand_count;
        a.table_status = status;
        a.probe_status = validate ? pstatus : nullptr;
        a.grid_rounds = rounds;
        a.plain = plain;
        a.verify = verify;
        a.kind = kind;
        a.rmatch = rmatch;
        const int mode = plain ? ASJ_MODE_PLAIN : (sig.f == 16 ? ASJ_MODE_SIG16 : ASJ_MODE_SIG8);
        // launched without probe keys too: it reports a failed validation
        tim_begin(plain ? "hash_probe_verify" : "sign_probe_verify", st);
        e = asj_launch_probe_local_single(&a, mode, plain ? 1 : sig.nsym, g_dev[dev].tab, st);
        tim_end(st);
        if (e != hipSuccess) { out_rc = hip_fail(e); break; }
        if (rmatch) {
            tim_begin("unmatched_build", st);
            e = asj_launch_unmatched_build(rmatch, r->ids, r->n, out, out_cap, out_count, status,
                                           validate ? pstatus : nullptr, 0, nullptr, nullptr, st);
            tim_end(st);
            if (e != hipSuccess) { out_rc = hip_fail(e); break; }
        }
        if ((o.flags & ASJ_SORTED) && out_cap > 0) {
            void *sort_tmp = nullptr;
            e = hipMallocAsync(&sort_tmp, asj_sort_scratch_bytes(out_cap), st);
            if (e != hipSuccess) { out_rc = hip_fail(e); break; }
            tim_begin("sort", st);
            e = asj_launch_sort_pairs(out, out_count, out_cap, sort_tmp, st);
            tim_end(st);
            (void)hipFreeAsync(sort_tmp, st);
            if (e != hipSuccess) { out_rc = hip_fail(e); break; }
        }
    } while (0);
    if (!fixed) (void)hipFreeAsync(blk, st);
    return out_rc;
}

} // namespace

extern "C" {

int asj_signature(const asj_keys *keys, asj_sig_params p, uint32_t *sig_out, hipStream_t st)
{
    TimingScope ts;
    if (!keys_ok(keys) || (keys->n > 0 && !sig_out)) return ASJ_EINVAL;
    asj_sig_params sig;
    int rc = resolve_sig(p, &sig);
    if (rc != ASJ_OK) return rc;
    int dev = 0;
    rc = ensure_init(&dev);
    if (rc != ASJ_OK) return rc;
    const int kpw = 0; // windows sized by the kernel from the keys' mean length
    if (sig64(sig)) // little-endian 64-bit signatures: the low word, then the high word
        TIMED("signature",
              launch_sign_for(keys, sig, 0, sig_out, g_dev[dev].tab, st, nullptr, sig_out + 1, 2, nullptr, kpw));
    else
        TIMED("signature", launch_sign_for(keys, sig, 0, sig_out, g_dev[dev].tab, st, nullptr, nullptr, 1, nullptr, kpw));
    return ASJ_OK;
}

int asj_build(const asj_keys *r, const asj_opts *opts, asj_table **table_out, hipStream_t st)
{
    TimingScope ts;
    return build_impl(r, opts, table_out, st);
}

int asj_probe(const asj_table *t, const asj_keys *s, asj_pair *out, int64_t out_cap, int64_t *out_count,
              int64_t *cand_count, hipStream_t st)
{
    TimingScope ts;
    return probe_impl(t, s, out, out_cap, out_count, cand_count, st);
}

int asj_join(const asj_keys *r, const asj_keys *s, const asj_opts *opts, asj_pair *out, int64_t out_cap,
             int64_t *out_count, int64_t *cand_count, hipStream_t st)
{
    TimingScope ts;
    if (!keys_ok(s) || !out_count || out_cap < 0 || (out_cap > 0 && !out)) return ASJ_EINVAL;
    const int lrc = join_local_single(r, s, opts, out, out_cap, out_count, cand_count, st);
    if (lrc != kNotLocal) return lrc;
    asj_table *t = nullptr;
    int rc = build_impl(r, opts, &t, st, out_count, cand_count); // the build's first launch clears the counters
    if (rc != ASJ_OK) return rc;
    rc = probe_impl(t, s, out, out_cap, out_count, cand_count, st, true);
    int rc2 = table_free_impl(t);
    return rc != ASJ_OK ? rc : rc2;
}

int asj_join_noalloc(const asj_keys *r, const asj_keys *s, const asj_opts *opts, asj_pair *out, int64_t out_cap,
                     int64_t *out_count, int64_t *cand_count, hipStream_t st)
{
    TimingScope ts;
    if (!keys_ok(r) || !keys_ok(s) || !out_count || out_cap < 0 || (out_cap > 0 && !out)) return ASJ_EINVAL;
    if (r->n > ASJ_NOALLOC_MAX_BUILD_ROWS) return ASJ_EINVAL; // beyond the scratch array
    asj_opts o = {};
    if (opts) o = *opts;
    // options that would allocate: sorting, a device-memory table, the split schedule
    if (o.flags & (ASJ_SORTED | ASJ_GLOBAL_TABLES | ASJ_PROBE_SPLIT)) return ASJ_EINVAL;
    o.flags |= ASJ_PROBE_FUSED; // also when the autotuner recorded the split schedule for this size
    const int plain = (o.flags & ASJ_PLAIN) != 0, verify = (o.flags & ASJ_NO_VERIFY) == 0;
    if ((plain && !verify) || join_kind(o.flags) < 0) return ASJ_EINVAL;
    if (o.flags & ASJ_FINGERPRINT) return ASJ_EUNSUPPORTED;
    if (!plain) {
        asj_sig_params sig;
        const int src = resolve_sig(o.sig, &sig);
        if (src != ASJ_OK) return src;
        if (sig64(sig)) return ASJ_EUNSUPPORTED;
    }
    float lf;
    int kpw, split, rounds;
    if (resolve_auto(0, r->n, o, &lf, &kpw, &split, &rounds) != ASJ_OK) return ASJ_EINVAL;
    int dev = 0;
    const int rc = ensure_init(&dev);
    if (rc != ASJ_OK) return rc;
    const int lrc = join_local_single(r, s, &o, out, out_cap, out_count, cand_count, st, g_dev[dev].scratch);
    return lrc == kNotLocal ? ASJ_EINVAL : lrc; // (every option set left reaches the LDS-table path)
}

int asj_table_status(const asj_table *t)
{
    if (!t) return ASJ_EINVAL;
    if (hipStreamSynchronize(t->stream) != hipSuccess) return ASJ_EHIP;
    int32_t v = 0;
    if (hipMemcpy(&v, t->status, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return ASJ_EHIP;
    return v == 0 ? ASJ_OK : (int)v;
}

int64_t asj_table_capacity(const asj_table *t) { return t ? t->capacity : -1; }

int asj_table_free(asj_table *t) { return table_free_impl(t); }

const char *asj_strerror(int code)
{
    switch (code) {
    case ASJ_OK: return "ok";
    case ASJ_EINVAL: return "invalid argument";
    case ASJ_ENOMEM: return "device allocation failed";
    case ASJ_EOVERFLOW: return "result larger than the output capacity";
    case ASJ_ETABLEFULL: return "hash table full";
    case ASJ_EHIP: return "HIP runtime error";
    case ASJ_EUNSUPPORTED: return "unsupported parameters";
    default: return "unknown error";
    }
}

int asj_timing_enable(int on)
{
    g_tim.on = on != 0;
    g_tim.count = 0;
    return ASJ_OK;
}

int asj_timing_read(float *ms, const char **names, int cap)
{
    const int n = g_tim.count;
    if (n == 0) return 0;
    if (hipEventSynchronize(g_tim.ev[2 * n - 1]) != hipSuccess) return ASJ_EHIP;
    for (int i = 0; i < n && i < cap; i++) {
        float v = 0.0f;
        if (hipEventElapsedTime(&v, g_tim.ev[2 * i], g_tim.ev[2 * i + 1]) != hipSuccess) return ASJ_EHIP;
        if (ms) ms[i] = v;
        if (names) names[i] = g_tim.names[i];
    }
    g_tim.count = 0;
    return n;
}

int asj_util_read(const void *src, int64_t bytes, uint32_t *out_word, int grid, hipStream_t st)
{
    if (bytes < 0 || (bytes > 0 && (!src || !out_word)) || ((uintptr_t)src & 15u)) return ASJ_EINVAL;
    if (grid <= 0) grid = 256 * 8;
    int dev = 0;
    int rc = ensure_init(&dev);
    if (rc != ASJ_OK) return rc;
    TimingScope ts;
    TIMED("read", asj_launch_read(src, bytes, out_word, grid, st));
    return ASJ_OK;
}

int asj_util_copy(void *dst, const void *src, int64_t bytes, hipStream_t st)
{
    if (bytes < 0 || (bytes > 0 && (!dst || !src))) return ASJ_EINVAL;
    if (((uintptr_t)dst | (uintptr_t)src) & 15u) return ASJ_EINVAL;
    int dev = 0;
    int rc = ensure_init(&dev);
    if (rc != ASJ_OK) return rc;
    TimingScope ts;
    TIMED("copy", asj_launch_copy(dst, src, bytes, st));
    return ASJ_OK;
}


int64_t asj_batch_workspace_bytes(int32_t njoins, int64_t n_build, int64_t n_probe, const asj_opts *opts)
{
    int plain, verify, kpw, split, local_only = 0;
    asj_sig_params sig;
    float lf;
    if (batch_opts(opts, n_build, &plain, &verify, &sig, &lf, &kpw, &split, nullptr, nullptr, nullptr, nullptr,
                   &local_only) != ASJ_OK)
        return -1;
    BatchLayout L;
    if (!batch_layout(njoins, n_build, n_probe, kpw, lf, &L, local_only != 0)) return -1;
    return (int64_t)L.bytes;
}

int asj_join_batch(const asj_batch *b, const asj_opts *opts, hipStream_t st)
{
    TimingScope ts;
    if (!b || b->njoins < 1 || !keys_ok(&b->r) || !keys_ok(&b->s) || !b->r_seg || !b->s_seg || !b->out_seg ||
        !b->out_count || !b->out)
        return ASJ_EINVAL;
    int plain, verify, kpw, split;
    asj_sig_params sig;
    float lf;
    int validate, kind, local, local_only;
    int rounds = 2;
    int rc = batch_opts(opts, b->r.n, &plain, &verify, &sig, &lf, &kpw, &split, &validate, &kind, &rounds, &local,
                        &local_only);
    if (rc != ASJ_OK) return rc;
    if (split) local = 0; // the split schedule signs the probe keys first: device-memory tables only
    BatchLayout L;
    if (!batch_layout(b->njoins, b->r.n, b->s.n, kpw, lf, &L, local_only != 0)) return ASJ_EINVAL;
    int dev = 0;
    rc = ensure_init(&dev);
    if (rc != ASJ_OK) return rc;
    uint8_t *ws = (uint8_t *)b->workspace;
    bool owned = false;
    if (ws) {
        if (b->workspace_bytes < (int64_t)L.bytes || ((uintptr_t)ws & 255u)) return ASJ_EINVAL;
    } else {
        hipError_t e = hipMallocAsync((void **)&ws, L.bytes, st);
        if (e != hipSuccess) return hip_fail(e);
        owned = true;
    }
    asj_join_desc *desc = (asj_join_desc *)(ws + L.desc);
    int64_t *rows_done = (int64_t *)(ws + L.rows_done);
    uint64_t *tot = (uint64_t *)(ws + L.tot);
    int32_t *status = (int32_t *)(ws + L.status);
    int32_t *win_r = (int32_t *)(ws + L.win_r);
    asj_win *win_s = (asj_win *)(ws + L.win_s);
    int32_t *win_l = (int32_t *)(ws + L.win_l);
    uint32_t *sig_r = (uint32_t *)(ws + L.sig);
    uint32_t *sig_s = (uint32_t *)(ws + L.ssig);
    uint64_t *slots = (uint64_t *)(ws + L.slots);
    uint32_t *rcnt = (uint32_t *)(ws + L.rcnt);
    int32_t *rmap = (int32_t *)(ws + L.rmap);
    uint64_t *novf = (uint64_t *)(ws + L.novf);
    uint64_t *ovf = (uint64_t *)(ws + L.ovf);
    int out_rc = ASJ_OK;
    do {
        hipError_t e;
        tim_begin("batch_plan", st);
        e = asj_launch_batch_plan(b->r_seg, b->s_seg, b->njoins, b->r.n, b->s.n, L.slot_bound, lf, kpw,
                                  local ? ASJ_LOCAL_ROWS : -1, local_only, desc, rows_done, b->out_count,
                                  b->cand_count, b->done_clock, tot, status, local_only ? nullptr : rcnt,
                                  L.region_cap, novf, st);
        if (e == hipSuccess && validate) e = asj_launch_validate(b->r.offsets, b->r.n, status, st);
        if (e == hipSuccess && validate) e = asj_launch_validate(b->s.offsets, b->s.n, status, st);
        tim_end(st);
        if (e != hipSuccess) { out_rc = hip_fail(e); break; }
        // the window and region maps are written by the signature kernel
        // (or, without build keys, a kernel of their own); the segments are
        // built by regions, which write every slot (no fill)
        uint8_t *rmatch = asj_kind_marks_build(kind) ? ws + L.rmatch : nullptr;
        asj_batch_prep prep = {tot, desc, b->s_seg, b->njoins, kpw,
                               win_r, L.win_r_cap, win_s, L.win_s_cap, win_l, L.win_s_cap,
                               (uint32_t *)rmatch, rmatch ? (b->r.n + 3) / 4 : 0, rmap, L.region_cap};
        tim_begin(plain ? "hash_build" : "sign_build", st);
        e = launch_sign_for(&b->r, sig, plain, sig_r, g_dev[dev].tab, st, status, nullptr, 1, &prep, 0);
        tim_end(st);
        if (e != hipSuccess) { out_rc = hip_fail(e); break; }
        if (!local_only) { // otherwise no join has a device-memory table
            tim_begin("insert", st);
            e = asj_launch_region_build_batch(sig_r, b->r.n, b->r_seg, b->njoins, desc, win_r, tot, L.win_r_cap,
                                              rmap, L.region_cap, rcnt, ovf, novf, slots, status, st);
            tim_end(st);
            if (e != hipSuccess) { out_rc = hip_fail(e); break; }
        }
        asj_probe_args a = {};
        a.rdata = b->r.data;
        a.roff = b->r.offsets;
        a.rids = b->r.ids;
        a.rn = b->r.n;
        a.keys_per_window = kpw;
        a.sdata = b->s.data;
        a.soff = b->s.offsets;
        a.sids = b->s.ids;
        a.n = b->s.n;
        a.slots = slots;
        a.out = b->out;
        a.out_count = b->out_count;
        a.cand_count = b->cand_count;
        a.table_status = status;
        a.plain = plain;
        a.verify = verify;
        a.kind = kind;
        a.njoins = b->njoins;
        a.s_seg = b->s_seg;
        a.desc = desc;
        a.wins = win_s;
        a.nwin = tot + 2;
        a.nwin_cap = L.win_s_cap;
        a.out_seg = b->out_seg;
        a.rows_done = rows_done;
        a.done_clock = b->done_clock;
        a.grid_rounds = rounds;
        a.rmatch = rmatch;
        const int mode = plain ? ASJ_MODE_PLAIN : (sig.f == 16 ? ASJ_MODE_SIG16 : ASJ_MODE_SIG8);
        if (split && b->s.n > 0) {
            tim_begin(plain ? "hash_S" : "sign_S", st);
            e = launch_sign_for(&b->s, sig, plain, sig_s, g_dev[dev].tab, st, status, nullptr, 1, nullptr, kpw);
            tim_end(st);
            if (e != hipSuccess) { out_rc = hip_fail(e); break; }
            a.ssig = sig_s;
        }
        tim_begin(plain ? "hash_probe_verify" : (a.ssig ? "probe_verify" : "sign_probe_verify"), st);
        if (local) { // one launch for the windows of both kinds of table
            a.win_l = win_l;
            a.nwin_l = tot + 3;
            a.nwin_l_cap = L.win_s_cap;
            a.r_seg = b->r_seg;
            a.rsig = sig_r;
            e = asj_launch_probe_local(&a, mode, sig.nsym, g_dev[dev].tab, st);
        } else {
            e = asj_launch_probe(&a, mode, sig.nsym, g_dev[dev].tab, kProbeGridCap, st);
        }
        tim_end(st);
        if (e != hipSuccess) { out_rc = hip_fail(e); break; }
        if (rmatch) { // right and full outer joins: the build rows without a match
            tim_begin("unmatched_build", st);
            e = asj_launch_unmatched_build(rmatch, b->r.ids, b->r.n, b->out, 0, b->out_count, status, nullptr,
                                           b->njoins, b->r_seg, b->out_seg, st);
            tim_end(st);
            if (e != hipSuccess) { out_rc = hip_fail(e); break; }
        }
    } while (0);
    if (owned) (void)hipFreeAsync(ws, st);
    return out_rc;
}

int64_t asj_clock_khz(void)
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return -1;
    return (int64_t)v;
}

} // extern "C"
