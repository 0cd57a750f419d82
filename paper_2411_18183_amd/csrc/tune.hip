// Autotuner: times whole joins over a grid of table load factors, probe
// keys per window, both probe schedules and probe grid sizes (1, 2 or 4
// rounds of resident blocks) on the caller's relations, keeps
// the fastest, and records it per build-size class so that later calls that
// leave these options at zero use it.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "asj_internal.h"

namespace {

struct Key {
    int dev, batch, bucket, f, nsym, plain, verify;
    bool operator<(const Key &o) const
    {
        return std::tie(dev, batch, bucket, f, nsym, plain, verify) <
               std::tie(o.dev, o.batch, o.bucket, o.f, o.nsym, o.plain, o.verify);
    }
};

std::mutex g_tune_mu;
std::map<Key, asj_tuned> g_tuned;

int log2_bucket(int64_t n)
{
    int b = 0;
    while (b < 62 && (1LL << b) < n) b++;
    return b;
}

Key make_key(int batch, int64_t n_build, const asj_opts &o)
{
    Key k = {};
    (void)hipGetDevice(&k.dev);
    k.batch = batch;
    k.bucket = log2_bucket(n_build);
    k.plain = (o.flags & ASJ_PLAIN) ? 1 : (o.flags & ASJ_FINGERPRINT) ? 2 : 0;
    k.verify = (o.flags & ASJ_NO_VERIFY) == 0;
    k.f = k.plain ? 0 : (o.sig.f ? o.sig.f : 16);
    k.nsym = k.plain ? 0 : (o.sig.nsym ? o.sig.nsym : 2);
    return k;
}

constexpr float kLoadFactors[] = {0.25f, 0.35f, 0.5f, 0.7f};
// few keys per window for long keys: 131k keys of 4 KB in windows of 64 give
// one block per compute unit
constexpr int kKeysPerWindow[] = {4, 8, 16, 32, 64};
constexpr int kGridRounds[] = {1, 2, 4};
constexpr int kReps = 3;
// Grid pass: every configuration timed over kReps back-to-back calls.
// Second stage: the kFinalists fastest of them and the defaults, timed again
// as blocks of kBlockRuns back-to-back calls (one block each per pass,
// kPasses passes in alternating order), so that the choice among
// configurations a few percent apart does not rest on one short sample
// (the minimum over some sixty medians of three single calls, each call
// followed by a synchronization, had often been a lucky sample).
constexpr int kFinalists = 4;
constexpr int kBlockRuns = 8;
constexpr int kPasses = 2;

int64_t capacity_for(int64_t n, float lf)
{
    int64_t cap = 64;
    while ((double)cap * lf < (double)n) cap <<= 1;
    return cap;
}

// Milliseconds per call over kReps back-to-back calls after one untimed
// call (the result of run() is checked on every call).
template <class Run>
int time_runs(Run run, hipStream_t st, hipEvent_t e0, hipEvent_t e1, float *ms)
{
    int rc = run();
    if (rc != ASJ_OK) return rc;
    if (hipEventRecord(e0, st) != hipSuccess) return ASJ_EHIP;
    for (int i = 0; i < kReps; i++) {
        rc = run();
        if (rc != ASJ_OK) return rc;
    }
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return ASJ_EHIP;
    if (hipEventElapsedTime(ms, e0, e1) != hipSuccess) return ASJ_EHIP;
    *ms /= kReps;
    return ASJ_OK;
}

// Milliseconds per call over kBlockRuns back-to-back calls (the stream
// stays busy: no host round trip between them).
template <class Run>
int time_block(Run run, hipStream_t st, hipEvent_t e0, hipEvent_t e1, float *ms)
{
    if (hipEventRecord(e0, st) != hipSuccess) return ASJ_EHIP;
    for (int i = 0; i < kBlockRuns; i++) {
        const int rc = run();
        if (rc != ASJ_OK) return rc;
    }
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return ASJ_EHIP;
    if (hipEventElapsedTime(ms, e0, e1) != hipSuccess) return ASJ_EHIP;
    *ms /= kBlockRuns;
    return ASJ_OK;
}

// The grid: every load factor that gives a distinct table capacity for
// n_build rows (all four for a batch, whose segments differ), every keys per
// window, both schedules, every grid size.
std::vector<asj_opts> grid(const asj_opts &base, int64_t n_build, bool batch)
{
    std::vector<asj_opts> g;
    std::vector<int64_t> caps;
    const uint32_t flags = base.flags & ~(ASJ_PROBE_FUSED | ASJ_PROBE_SPLIT);
    for (float lf : kLoadFactors) {
        if (!batch) {
            const int64_t c = capacity_for(n_build, lf);
            if (std::find(caps.begin(), caps.end(), c) != caps.end()) continue;
            caps.push_back(c);
        }
        for (int kpw : kKeysPerWindow)
            for (uint32_t sched : {ASJ_PROBE_FUSED, ASJ_PROBE_SPLIT})
                for (int rounds : kGridRounds) {
                    if (sched == ASJ_PROBE_SPLIT && base.sig.f == 16 && base.sig.nsym == 4) continue; // fused only
                    if (sched == ASJ_PROBE_SPLIT && (base.flags & ASJ_LOCAL_ONLY)) continue;         // LDS tables: fused
                    asj_opts o = base;
                    o.load_factor = lf;
                    o.keys_per_window = kpw;
                    o.grid_rounds = rounds;
                    o.flags = flags | sched;
                    g.push_back(o);
                }
    }
    return g;
}

template <class RunWith>
int tune(const asj_opts &base, int64_t n_build, bool batch, RunWith run_with, asj_tune_result *res, hipStream_t st)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreateWithFlags(&e0, hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&e1, hipEventDisableSystemFence) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return ASJ_EHIP;
    }
    int rc = ASJ_OK;
    asj_opts defaults = base;
    defaults.load_factor = 0.5f;
    defaults.keys_per_window = ASJ_DEFAULT_KEYS_PER_WINDOW;
    defaults.grid_rounds = 2;
    defaults.flags = (base.flags & ~(ASJ_PROBE_FUSED | ASJ_PROBE_SPLIT)) | ASJ_PROBE_FUSED;
    float def_ms = 0.0f, best_ms = 0.0f;
    asj_opts best = defaults;
    int trials = 0;
    // grid pass: ms per call of each configuration, the defaults first
    struct Timed {
        float ms;
        asj_opts o;
        bool is_default;
    };
    std::vector<Timed> timed;
    rc = time_runs([&] { return run_with(defaults); }, st, e0, e1, &def_ms);
    if (rc == ASJ_OK) {
        timed.push_back({def_ms, defaults, true});
        for (const asj_opts &o : grid(base, n_build, batch)) {
            float ms = 0.0f;
            rc = time_runs([&] { return run_with(o); }, st, e0, e1, &ms);
            if (rc != ASJ_OK) break;
            trials++;
            timed.push_back({ms, o, false});
        }
    }
    if (rc == ASJ_OK) { // second stage: the finalists and the defaults, on one measure
        std::stable_sort(timed.begin(), timed.end(), [](const Timed &x, const Timed &y) { return x.ms < y.ms; });
        std::vector<size_t> fin;
        for (size_t i = 0; i < timed.size(); i++)
            if ((int)fin.size() < kFinalists || timed[i].is_default) fin.push_back(i);
        std::vector<float> sum(fin.size(), 0.0f);
        for (int pass = 0; pass < kPasses && rc == ASJ_OK; pass++)
            for (size_t i = 0; i < fin.size() && rc == ASJ_OK; i++) {
                const size_t k = pass % 2 ? fin.size() - 1 - i : i;
                float ms = 0.0f;
                rc = time_block([&] { return run_with(timed[fin[k]].o); }, st, e0, e1, &ms);
                sum[k] += ms;
            }
        if (rc == ASJ_OK) {
            size_t bi = 0;
            for (size_t i = 0; i < fin.size(); i++) {
                if (sum[i] < sum[bi]) bi = i;
                if (timed[fin[i]].is_default) def_ms = sum[i] / kPasses;
            }
            best = timed[fin[bi]].o;
            best_ms = sum[bi] / kPasses;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != ASJ_OK) return rc;
    asj_tuned t = {best.load_factor, best.keys_per_window, (best.flags & ASJ_PROBE_SPLIT) ? 1 : 0, best.grid_rounds};
    asj_tuned_store(batch ? 1 : 0, n_build, base, t);
    if (res) {
        res->best = best;
        res->best_ms = best_ms;
        res->default_ms = def_ms;
        res->trials = trials;
    }
    return ASJ_OK;
}

bool tunable(const asj_opts &o)
{
    return !((o.flags & ASJ_PROBE_FUSED) && (o.flags & ASJ_PROBE_SPLIT)) && o.load_factor >= 0.0f &&
           o.load_factor < 1.0f && o.keys_per_window <= ASJ_WAVE && o.grid_rounds <= 8;
}

} // namespace

bool asj_tuned_lookup(int batch, int64_t n_build, const asj_opts &o, asj_tuned *t)
{
    const Key k = make_key(batch, n_build, o);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(k);
    if (it == g_tuned.end()) return false;
    *t = it->second;
    return true;
}

void asj_tuned_store(int batch, int64_t n_build, const asj_opts &o, const asj_tuned &t)
{
    const Key k = make_key(batch, n_build, o);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[k] = t;
}

extern "C" {

int asj_autotune(const asj_keys *r, const asj_keys *s, const asj_opts *opts, asj_pair *out, int64_t out_cap,
                 int64_t *out_count, asj_tune_result *res, hipStream_t st)
{
    asj_opts base = {};
    if (opts) base = *opts;
    if (!r || !s || !out_count || out_cap < 0 || (out_cap > 0 && !out) || !tunable(base)) return ASJ_EINVAL;
    return tune(base, r->n, false,
                [&](const asj_opts &o) { return asj_join(r, s, &o, out, out_cap, out_count, nullptr, st); }, res, st);
}

int asj_autotune_batch(const asj_batch *b, const asj_opts *opts, asj_tune_result *res, hipStream_t st)
{
    asj_opts base = {};
    if (opts) base = *opts;
    if (!b || !tunable(base)) return ASJ_EINVAL;
    asj_batch trial = *b;
    trial.workspace = nullptr; // every configuration sizes its own (stream-ordered, pooled) workspace
    trial.workspace_bytes = 0;
    return tune(base, b->r.n, true, [&](const asj_opts &o) { return asj_join_batch(&trial, &o, st); }, res, st);
}

void asj_autotune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
}

} // extern "C"
