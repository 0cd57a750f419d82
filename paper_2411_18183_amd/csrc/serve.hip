// Serving: probe requests against a resident build table (the probe phase
// of Section 3.2, Figure 2, for a stream of requests) with continuous
// batching.
//
// Requests are queued FIFO.  A scheduler thread admits the queue head when
// the device bytes it needs fit in the remaining HBM budget (a request that
// cannot fit even in an empty budget is refused at submission; the head
// never gets overtaken, so nobody starves), and packs everything admitted
// into one launch on a free stream slot: the requests' keys are copied in
// behind one another, one batched probe kernel runs all of them against the
// shared table (each request is one segment with its own output), and the
// results are copied back.  Requests that arrive while launches are running
// join the next launch on the next free slot, so their work overlaps on the
// device with the work already there.  Completion frees the budget and the
// slot and wakes the waiters.
//
// The scheduler only talks to the device through launch_batch() and
// slot_done(); with dry_run set those simulate a launch by its key count,
// so the admission and batching logic can be exercised without a GPU.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string.h>
#include <thread>
#include <unordered_map>
#include <vector>

#include "asj_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
    int64_t ticket = 0;
    const uint8_t *data = nullptr; // host
    const int64_t *off = nullptr;  // host, n + 1
    int64_t n = 0;
    asj_pair *out = nullptr; // host
    int64_t cap = 0;
    int64_t bytes = 0; // device footprint charged to the budget
    double t_arrive = 0, t_launch = -1, t_done = -1;
    int64_t count = 0;
    int status = ASJ_OK;
    bool done = false;
    bool claimed = false; // a caller waits on this ticket (one waiter per ticket)
    int batch_id = -1, batch_n = 0;
    double dev_ms = 0, kern_ms = 0; // device time of its launch: copies and kernel, kernel alone
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    // timing events of the launch: before its input copies, around its
    // kernel, after its output copies
    hipEvent_t t_in = nullptr, t_k0 = nullptr, t_k1 = nullptr, t_out = nullptr;
    bool busy = false;
    std::vector<Req *> reqs;
    uint8_t *pin = nullptr; // pinned staging: metadata up, counts down
    size_t pin_bytes = 0;
    size_t counts_off = 0;
    double dry_done = 0; // dry run: completion time (ms)
    int batch_id = -1;
};

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device bytes one request holds while in flight: its keys and offsets,
// probe ids, probe signatures (split schedule), probe windows (kpw keys
// each), output pairs, and its share of the per-batch segment, descriptor
// and counter arrays with their alignment.
int64_t request_bytes(int64_t n, int64_t data_bytes, int64_t cap, int kpw)
{
    return (int64_t)(al256((size_t)data_bytes) + al256(8 * (size_t)(n + 1)) + 2 * al256(4 * (size_t)n) +
                     al256(sizeof(asj_win) * (size_t)(n / kpw + 1)) + al256(8 * (size_t)cap) + 2048);
}

// Pinned staging a launch of K keys, J requests and W windows uses: the
// metadata block (offsets .. window map, laid out as on the device) and the
// counts read back.
size_t staging_bytes(int64_t K, int64_t J, int64_t W)
{
    const size_t meta = al256(8 * (size_t)(K + 1)) + al256(4 * (size_t)(K > 0 ? K : 1)) +
                        2 * al256(8 * (size_t)(J + 1)) + al256(sizeof(asj_join_desc) * (size_t)J) + 256 +
                        al256(sizeof(asj_win) * (size_t)(W > 0 ? W : 1));
    return al256(meta) + al256(8 * (size_t)J);
}

int grow_staging(Slot &sl, size_t bytes)
{
    if (sl.pin) (void)hipHostFree(sl.pin);
    sl.pin = nullptr;
    sl.pin_bytes = 0;
    if (hipHostMalloc((void **)&sl.pin, bytes, hipHostMallocDefault) != hipSuccess) return ASJ_ENOMEM;
    sl.pin_bytes = bytes;
    return ASJ_OK;
}

} // namespace

struct asj_server {
    asj_table tbl;
    asj_server_opts o;
    const uint16_t *tab = nullptr;
    int dev = 0;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<Req *> q;
    std::unordered_map<int64_t, Req *> reqs;
    int64_t next_ticket = 1;
    int64_t budget_used = 0;
    int64_t peak_budget = 0;
    std::vector<Slot> slots;
    std::thread th;
    bool stop = false;
    Clock::time_point t0;
    int batch_seq = 0;
    int64_t launches = 0;

    double now_ms() const { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }
};

namespace {

// Issue one launch for `batch` on slot `sl` (scheduler thread only).
int launch_batch(asj_server *S, Slot &sl, const std::vector<Req *> &batch)
{
    const int J = (int)batch.size();
    int64_t K = 0, D = 0, C = 0, W = 0;
    for (Req *r : batch) {
        K += r->n;
        D += r->off[r->n] - r->off[0];
        C += r->cap;
    }
    if (S->o.dry_run) {
        sl.dry_done = S->now_ms() + S->o.dry_ns_per_key * 1e-6 * (double)K;
        return ASJ_OK;
    }
    const int kpw = S->tbl.keys_per_window; // 1 .. 64 for every built table
    for (Req *r : batch) W += (r->n + kpw - 1) / kpw;
    // device layout
    const size_t o_data = 0;
    const size_t o_off = al256(o_data + (size_t)D);
    const size_t o_sid = al256(o_off + 8 * (size_t)(K + 1));
    const size_t o_sseg = al256(o_sid + 4 * (size_t)(K > 0 ? K : 1));
    const size_t o_oseg = al256(o_sseg + 8 * (size_t)(J + 1));
    const size_t o_desc = al256(o_oseg + 8 * (size_t)(J + 1));
    const size_t o_nwin = al256(o_desc + sizeof(asj_join_desc) * (size_t)J);
    const size_t o_win = al256(o_nwin + 8);
    const size_t o_cnt = al256(o_win + sizeof(asj_win) * (size_t)(W > 0 ? W : 1));
    const size_t o_done = al256(o_cnt + 8 * (size_t)J);
    const size_t o_out = al256(o_done + 8 * (size_t)J);
    const size_t o_ssig = al256(o_out + 8 * (size_t)(C > 0 ? C : 1)); // probe signatures (split schedule)
    const size_t dev_bytes = S->tbl.split ? al256(o_ssig + 4 * (size_t)(K > 0 ? K : 1)) : o_ssig;
    const size_t meta_bytes = o_cnt - o_off; // offsets .. descriptors, staged in one copy
    // pinned staging (metadata, then the counts read back); sized for a full
    // batch when the server starts, grown geometrically past that (pinning
    // and unpinning host memory is slow and may wait for the device)
    const size_t need = staging_bytes(K, J, W);
    if (sl.pin_bytes < need && grow_staging(sl, std::max(need, 2 * sl.pin_bytes)) != ASJ_OK) return ASJ_ENOMEM;
    sl.counts_off = al256(meta_bytes);
    uint8_t *meta = sl.pin;
    int64_t *h_off = (int64_t *)(meta + (o_off - o_off));
    int32_t *h_sid = (int32_t *)(meta + (o_sid - o_off));
    int64_t *h_sseg = (int64_t *)(meta + (o_sseg - o_off));
    int64_t *h_oseg = (int64_t *)(meta + (o_oseg - o_off));
    asj_join_desc *h_desc = (asj_join_desc *)(meta + (o_desc - o_off));
    uint64_t *h_nwin = (uint64_t *)(meta + (o_nwin - o_off));
    asj_win *h_win = (asj_win *)(meta + (o_win - o_off));
    int64_t row = 0, db = 0, ob = 0, wb = 0;
    for (int j = 0; j < J; j++) {
        const Req *r = batch[j];
        h_sseg[j] = row;
        h_oseg[j] = ob;
        h_desc[j].tbase = 0;
        h_desc[j].mask = (uint64_t)S->tbl.capacity - 1;
        h_desc[j].wbase = wb;
        h_desc[j].wbase_r = 0;
        h_desc[j].wbase_l = 0;
        h_desc[j].rbase = 0;
        const int64_t nw = (r->n + kpw - 1) / kpw;
        for (int64_t w = 0; w < nw; w++) {
            h_win[wb + w].join = j;
            h_win[wb + w].first = row + w * kpw;
            h_win[wb + w].rows = (int32_t)std::min((int64_t)kpw, r->n - w * kpw);
        }
        wb += nw;
        const int64_t base = r->off[0];
        for (int64_t k = 0; k < r->n; k++) {
            h_off[row + k] = db + (r->off[k] - base);
            h_sid[row + k] = (int32_t)k;
        }
        row += r->n;
        db += r->off[r->n] - base;
        ob += r->cap;
    }
    h_off[K] = D;
    h_sseg[J] = K;
    h_oseg[J] = C;
    *h_nwin = (uint64_t)W;

    uint8_t *d = nullptr;
    hipError_t e = hipMallocAsync((void **)&d, dev_bytes, sl.st);
    if (e != hipSuccess) return ASJ_ENOMEM;
    e = hipEventRecord(sl.t_in, sl.st);
    db = 0;
    for (int j = 0; j < J && e == hipSuccess; j++) {
        const Req *r = batch[j];
        const int64_t len = r->off[r->n] - r->off[0];
        if (len > 0) e = hipMemcpyAsync(d + o_data + db, r->data + r->off[0], (size_t)len, hipMemcpyHostToDevice, sl.st);
        db += len;
    }
    if (e == hipSuccess) e = hipMemcpyAsync(d + o_off, meta, meta_bytes, hipMemcpyHostToDevice, sl.st);
    if (e == hipSuccess) e = asj_launch_fill_i64((int64_t *)(d + o_cnt), (int64_t)((o_out - o_cnt) / 8), 0, sl.st); // counts, rows_done
    if (e == hipSuccess) {
        asj_probe_args a = {};
        a.rdata = S->tbl.r.data;
        a.roff = S->tbl.r.offsets;
        a.rids = S->tbl.r.ids;
        a.rn = S->tbl.r.n;
        a.keys_per_window = S->tbl.keys_per_window;
        a.sdata = d + o_data;
        a.soff = (const int64_t *)(d + o_off);
        a.sids = (const int32_t *)(d + o_sid);
        a.n = K;
        a.slots = S->tbl.slots;
        a.out = (asj_pair *)(d + o_out);
        a.out_count = (int64_t *)(d + o_cnt);
        a.cand_count = nullptr;
        a.table_status = S->tbl.status;
        a.plain = S->tbl.plain;
        a.verify = S->tbl.verify;
        a.kind = S->tbl.kind;
        a.njoins = J;
        a.s_seg = (const int64_t *)(d + o_sseg);
        a.desc = (const asj_join_desc *)(d + o_desc);
        a.wins = (const asj_win *)(d + o_win);
        a.nwin = (const uint64_t *)(d + o_nwin);
        a.nwin_cap = W;
        a.out_seg = (const int64_t *)(d + o_oseg);
        a.rows_done = (int64_t *)(d + o_done);
        a.done_clock = nullptr;
        a.grid_rounds = S->tbl.grid_rounds;
        const int mode = S->tbl.plain ? ASJ_MODE_PLAIN : (S->tbl.sig.f == 16 ? ASJ_MODE_SIG16 : ASJ_MODE_SIG8);
        if (S->tbl.split && K > 0) {
            const asj_keys keys = {a.sdata, a.soff, a.sids, K};
            e = asj_launch_sign(mode, S->tbl.plain ? 1 : S->tbl.sig.nsym, &keys, (uint32_t *)(d + o_ssig), S->tab,
                                256 * 16, sl.st, nullptr, nullptr, 1, nullptr, S->tbl.keys_per_window);
            a.ssig = (const uint32_t *)(d + o_ssig);
        }
        if (e == hipSuccess) e = hipEventRecord(sl.t_k0, sl.st);
        if (e == hipSuccess) e = asj_launch_probe(&a, mode, S->tbl.sig.nsym, S->tab, 256 * 16, sl.st);
        if (e == hipSuccess) e = hipEventRecord(sl.t_k1, sl.st);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(sl.pin + sl.counts_off, d + o_cnt, 8 * (size_t)J, hipMemcpyDeviceToHost, sl.st);
    ob = 0;
    for (int j = 0; j < J && e == hipSuccess; j++) {
        const Req *r = batch[j];
        if (r->cap > 0)
            e = hipMemcpyAsync(r->out, d + o_out + 8 * (size_t)ob, 8 * (size_t)r->cap, hipMemcpyDeviceToHost, sl.st);
        ob += r->cap;
    }
    if (e == hipSuccess) e = hipEventRecord(sl.t_out, sl.st);
    if (e == hipSuccess) e = hipEventRecord(sl.ev, sl.st);
    (void)hipFreeAsync(d, sl.st);
    return e == hipSuccess ? ASJ_OK : ASJ_EHIP;
}

bool slot_done(asj_server *S, Slot &sl)
{
    if (S->o.dry_run) return S->now_ms() >= sl.dry_done;
    return hipEventQuery(sl.ev) != hipErrorNotReady;
}

// Completion bookkeeping (called with the lock held).
void finish_slot(asj_server *S, Slot &sl, int status)
{
    const double t = S->now_ms();
    float dev_ms = 0.0f, kern_ms = 0.0f;
    if (!S->o.dry_run && status == ASJ_OK) {
        if (hipEventElapsedTime(&dev_ms, sl.t_in, sl.t_out) != hipSuccess) dev_ms = -1.0f;
        if (hipEventElapsedTime(&kern_ms, sl.t_k0, sl.t_k1) != hipSuccess) kern_ms = -1.0f;
    }
    for (size_t j = 0; j < sl.reqs.size(); j++) {
        Req *r = sl.reqs[j];
        r->dev_ms = dev_ms;
        r->kern_ms = kern_ms;
        if (!S->o.dry_run && status == ASJ_OK) r->count = ((const int64_t *)(sl.pin + sl.counts_off))[j];
        r->status = status;
        r->t_done = t;
        r->done = true;
        S->budget_used -= r->bytes;
    }
    sl.reqs.clear();
    sl.busy = false;
}

void scheduler(asj_server *S)
{
    if (!S->o.dry_run) (void)hipSetDevice(S->dev);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool finished = false;
        for (Slot &sl : S->slots) {
            if (sl.busy && slot_done(S, sl)) {
                int st = ASJ_OK;
                if (!S->o.dry_run && hipEventSynchronize(sl.ev) != hipSuccess) st = ASJ_EHIP;
                finish_slot(S, sl, st);
                finished = true;
            }
        }
        if (finished) S->cv_done.notify_all();
        // admit the queue head(s) into free slots
        for (;;) {
            if (S->q.empty()) break;
            Slot *free = nullptr;
            for (Slot &sl : S->slots)
                if (!sl.busy) {
                    free = &sl;
                    break;
                }
            if (!free) break;
            std::vector<Req *> batch;
            int64_t keys = 0, bytes = 0;
            while (!S->q.empty()) {
                Req *r = S->q.front();
                if (S->budget_used + bytes + r->bytes > S->o.hbm_budget) break;
                if (!batch.empty() &&
                    (keys + r->n > S->o.max_batch_keys || (int)batch.size() >= S->o.max_batch_requests))
                    break;
                batch.push_back(r);
                keys += r->n;
                bytes += r->bytes;
                S->q.pop_front();
            }
            if (batch.empty()) break; // the head waits for memory to be freed
            S->budget_used += bytes;
            S->peak_budget = std::max(S->peak_budget, S->budget_used);
            const int id = S->batch_seq++;
            const double t = S->now_ms();
            for (Req *r : batch) {
                r->t_launch = t;
                r->batch_id = id;
                r->batch_n = (int)batch.size();
            }
            free->busy = true;
            free->reqs = batch;
            free->batch_id = id;
            S->launches++;
            lk.unlock(); // device calls outside the lock; only this thread touches slots
            const int rc = launch_batch(S, *free, batch);
            lk.lock();
            if (rc != ASJ_OK) {
                if (!S->o.dry_run) (void)hipStreamSynchronize(free->st);
                finish_slot(S, *free, rc);
                S->cv_done.notify_all();
            }
        }
        bool busy = false;
        for (Slot &sl : S->slots) busy = busy || sl.busy;
        if (S->stop && S->q.empty() && !busy) break;
        if (busy) S->cv_sched.wait_for(lk, std::chrono::microseconds(20));
        else S->cv_sched.wait(lk, [S] { return S->stop || !S->q.empty(); });
    }
}

} // namespace

extern "C" {

int asj_server_create(const asj_table *t, const asj_server_opts *opts, asj_server **out)
{
    if (!out) return ASJ_EINVAL;
    *out = nullptr;
    asj_server_opts o = {};
    if (opts) o = *opts;
    if (!o.dry_run && !t) return ASJ_EINVAL;
    if (t && !t->plain && t->sig.f == 16 && t->sig.nsym == 4) return ASJ_EUNSUPPORTED; // 64-bit signatures
    if (t && t->fp) return ASJ_EUNSUPPORTED;                                            // fingerprint control
    if (t && asj_kind_marks_build(t->kind)) return ASJ_EUNSUPPORTED; // right / full outer: per-call build marks
    if (o.slots <= 0) o.slots = 4;
    if (o.hbm_budget <= 0) o.hbm_budget = 200ll << 30;
    if (o.max_batch_keys <= 0) o.max_batch_keys = 256ll << 10;
    if (o.max_batch_requests <= 0) o.max_batch_requests = 256;
    if (o.slots > 64) return ASJ_EINVAL;
    asj_server *S = new (std::nothrow) asj_server();
    if (!S) return ASJ_ENOMEM;
    S->o = o;
    if (t) S->tbl = *t;
    S->t0 = Clock::now();
    S->slots.resize((size_t)o.slots);
    if (!o.dry_run) {
        S->tab = asj_device_tables(&S->dev);
        if (!S->tab) {
            delete S;
            return ASJ_EHIP;
        }
        for (Slot &sl : S->slots) {
            if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&sl.t_in, hipEventDisableSystemFence) != hipSuccess ||
                hipEventCreateWithFlags(&sl.t_k0, hipEventDisableSystemFence) != hipSuccess ||
                hipEventCreateWithFlags(&sl.t_k1, hipEventDisableSystemFence) != hipSuccess ||
                hipEventCreateWithFlags(&sl.t_out, hipEventDisableSystemFence) != hipSuccess) {
                for (Slot &x : S->slots) {
                    for (hipEvent_t ev : {x.ev, x.t_in, x.t_k0, x.t_k1, x.t_out})
                        if (ev) (void)hipEventDestroy(ev);
                    if (x.st) (void)hipStreamDestroy(x.st);
                }
                delete S;
                return ASJ_EHIP;
            }
        }
        // staging for a full batch on every slot, allocated once
        const int kpw = t->keys_per_window >= 1 ? t->keys_per_window : ASJ_DEFAULT_KEYS_PER_WINDOW;
        const size_t full = staging_bytes(o.max_batch_keys, o.max_batch_requests,
                                          o.max_batch_keys / kpw + o.max_batch_requests);
        for (Slot &sl : S->slots) {
            if (grow_staging(sl, full) != ASJ_OK) {
                for (Slot &x : S->slots) {
                    if (x.pin) (void)hipHostFree(x.pin);
                    for (hipEvent_t ev : {x.ev, x.t_in, x.t_k0, x.t_k1, x.t_out}) (void)hipEventDestroy(ev);
                    (void)hipStreamDestroy(x.st);
                }
                delete S;
                return ASJ_ENOMEM;
            }
        }
        // the table's build must be complete before any probe on the slot streams
        if (hipStreamSynchronize(t->stream) != hipSuccess) {
            delete S;
            return ASJ_EHIP;
        }
    }
    S->th = std::thread(scheduler, S);
    *out = S;
    return ASJ_OK;
}

int asj_server_submit(asj_server *S, const uint8_t *data, const int64_t *offsets, int64_t n, asj_pair *out,
                      int64_t out_cap, int64_t *ticket)
{
    if (!S || !ticket || n < 0 || n >= (int64_t)INT32_MAX || !offsets || out_cap < 0 || (out_cap > 0 && !out))
        return ASJ_EINVAL;
    const int64_t data_bytes = offsets[n] - offsets[0];
    if (data_bytes < 0 || (data_bytes > 0 && !data)) return ASJ_EINVAL;
    for (int64_t k = 0; k < n; k++) // host offsets: checked here, before any copy is made from them
        if (offsets[k + 1] < offsets[k]) return ASJ_EINVAL;
    Req *r = new (std::nothrow) Req();
    if (!r) return ASJ_ENOMEM;
    r->data = data;
    r->off = offsets;
    r->n = n;
    r->out = out;
    r->cap = out_cap;
    r->bytes = request_bytes(n, data_bytes, out_cap, S->tbl.keys_per_window >= 1 ? S->tbl.keys_per_window
                                                                                   : ASJ_DEFAULT_KEYS_PER_WINDOW);
    std::lock_guard<std::mutex> lk(S->mu);
    if (r->bytes > S->o.hbm_budget) {
        delete r;
        return ASJ_ENOMEM; // could never be admitted
    }
    r->ticket = S->next_ticket++;
    r->t_arrive = S->now_ms();
    S->reqs[r->ticket] = r;
    S->q.push_back(r);
    *ticket = r->ticket;
    S->cv_sched.notify_one();
    return ASJ_OK;
}

int asj_server_wait(asj_server *S, int64_t ticket, asj_request_info *info)
{
    if (!S) return ASJ_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end() || it->second->claimed) return ASJ_EINVAL; // unknown, or another caller waits on it
    Req *r = it->second;
    r->claimed = true; // the only waiter: it alone erases and deletes the request
    S->cv_done.wait(lk, [r] { return r->done; });
    if (info) {
        info->status = r->status;
        info->count = r->count;
        info->t_arrive_ms = r->t_arrive;
        info->t_launch_ms = r->t_launch;
        info->t_done_ms = r->t_done;
        info->batch_id = r->batch_id;
        info->batch_requests = r->batch_n;
        info->t_device_ms = r->dev_ms;
        info->t_kernel_ms = r->kern_ms;
    }
    const int st = r->status;
    S->reqs.erase(ticket);
    delete r;
    return st;
}

int asj_server_stats(asj_server *S, asj_server_stats_t *st)
{
    if (!S || !st) return ASJ_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    st->queued = (int64_t)S->q.size();
    int64_t busy = 0;
    for (Slot &sl : S->slots) busy += sl.busy ? 1 : 0;
    st->busy_slots = busy;
    st->budget_used = S->budget_used;
    st->peak_budget_used = S->peak_budget;
    st->launches = S->launches;
    st->now_ms = S->now_ms();
    return ASJ_OK;
}

int asj_server_destroy(asj_server *S)
{
    if (!S) return ASJ_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_sched.notify_all();
    if (S->th.joinable()) S->th.join();
    for (Slot &sl : S->slots) {
        if (sl.pin) (void)hipHostFree(sl.pin);
        for (hipEvent_t ev : {sl.ev, sl.t_in, sl.t_k0, sl.t_k1, sl.t_out})
            if (ev) (void)hipEventDestroy(ev);
        if (sl.st) (void)hipStreamDestroy(sl.st);
    }
    for (auto &kv : S->reqs) delete kv.second;
    delete S;
    return ASJ_OK;
}

} // extern "C"
