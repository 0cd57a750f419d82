// Probe side of the join in one kernel: Sign(s) for every probe tuple,
// Probe(H_sign, s), candidate verification and output compaction
// (Section 3.2, Figure 2: sign and probe every tuple of S and output the
// matching tuples; Section 2: matching tuples are concatenated into T).
//
// A wave takes a window of up to 64 probe keys, one key per lane (fewer keys
// per window make the verification re-read of a key come sooner after its
// signing read, while the bytes are still in the L2 cache).
//   1. The window's keys are signed (sign_window.h), so the keys' bytes are
//      still cache-resident when verification reads them again, and no
//      signature array goes through memory.
//   2. Each lane walks its key's run of slots from the home slot
//      mix32(signature) to the first empty slot, reading the aligned group
//      of four slots (32 bytes) that holds the current slot; every slot whose
//      stored signature equals the key's is a candidate (the paper outputs
//      candidates directly; here each one is compared byte by byte unless
//      verification is switched off).  The wave advances all walks in rounds
//      of at most one candidate per lane.
//   3. A round rejects candidates whose length differs and cuts the
//      remaining pairs into ceil(len / 64) chunks laid out back to back:
//      passes of 64 chunks, one per lane, compare both keys and flag
//      mismatching pairs in LDS.  The last chunk of a key of at least 64
//      bytes is the key's final 64 bytes (overlapping its neighbour), so
//      every compared chunk is a full, unguarded, unmasked read.
//   4. Surviving pairs are staged in a per-wave LDS buffer (ballot +
//      popcount prefix) and written out in bulk after one atomic reservation
//      per flush; a single output counter hit once per round and wave had
//      cost 11% of the kernel.
// The baseline simple hash join runs the same kernel with the plain key hash
// and treats every occupied slot as a candidate (no signature stored); its
// byte comparison stops after the first 64 bytes when they differ.
// In batch mode windows never span two joins: a window reads its join from
// the window map, probes that join's table segment, appends to that join's
// output segment, and the wave that finishes a join's last probe row stamps
// its completion clock.
#include "sign_window.h"

namespace {

// Block size: 8 waves when the kernel signs (one copy of the GF tables in
// LDS serves more waves), 4 waves when the signatures are given (no tables;
// the smaller block fits the register-limited wave count per CU exactly).
template <int PRESIGNED>
struct Shape {
    static constexpr int block = PRESIGNED ? 256 : 512;
    static constexpr int waves = block / ASJ_WAVE;
};
constexpr int kStage = 256; // staged result pairs per wave; flushed once more than kStage - 64 wait

typedef uint64_t asj_u64x2 __attribute__((ext_vector_type(2), aligned(16)));
typedef uint64_t asj_u64x2a8 __attribute__((ext_vector_type(2), aligned(8)));

struct Walk {
    uint64_t h;     // next slot to examine
    uint64_t qb;    // base slot of the cached group of four
    uint64_t q[4];  // cached group
    bool walking;   // the run has not ended yet
};

// Advance a lane's walk to its next candidate; true with *r = build row.
template <int PLAIN>
__device__ __forceinline__ bool next_candidate(const uint64_t *__restrict__ slots, uint64_t mask, uint32_t sg,
                                               Walk &w, uint32_t &r)
{
    bool has = false;
    while (w.walking) {
        const uint64_t qb = w.h & ~3ull;
        if (qb != w.qb) {
            const asj_u64x2 *g = (const asj_u64x2 *)(slots + qb);
            const asj_u64x2 lo = g[0], hi = g[1];
            w.q[0] = lo.x;
            w.q[1] = lo.y;
            w.q[2] = hi.x;
            w.q[3] = hi.y;
            w.qb = qb;
        }
        const int p = (int)(w.h - qb);
        bool stop = false;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            if (!stop && t >= p) {
                const uint64_t sl = w.q[t];
                if (sl == ASJ_EMPTY_SLOT) {
                    w.walking = false;
                    stop = true;
                } else if (PLAIN || (uint32_t)(sl >> 32) == sg) {
                    has = true;
                    r = (uint32_t)sl;
                    stop = true;
                    w.h = (qb + t + 1) & mask;
                    if (t < 3 && w.q[t + 1] == ASJ_EMPTY_SLOT) w.walking = false; // run ends here
                }
            }
        }
        if (stop) break;
        w.h = (qb + 4) & mask;
    }
    return has;
}

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, ASJ_WAVE);
    return v;
}

template <int MODE, int NSYM, int PLAIN, int VERIFY, int BATCH, int PRESIGNED>
// At most 128 registers (4 waves per SIMD): above that only one block fits a
// CU.
__global__ __launch_bounds__(Shape<PRESIGNED>::block, 4) void probe_kernel(asj_probe_args a,
                                                                         const uint16_t *__restrict__ gtab)
{
    constexpr int kBlock = Shape<PRESIGNED>::block;
    constexpr int kWaves = Shape<PRESIGNED>::waves;
    // four GF(2^16) components: the table holds the low word (components 1,
    // 2), a candidate must also match the build row's high word
    constexpr bool kHi = MODE == ASJ_MODE_SIG16 && NSYM == 4 && !PRESIGNED;
    __shared__ uint16_t tab[PRESIGNED ? 2 : asj::TabWords<MODE>::value];
    __shared__ int64_t kst[kWaves][ASJ_WAVE];  // probe key starts
    __shared__ int64_t krs[kWaves][ASJ_WAVE];  // candidate build key starts
    __shared__ int32_t kln[kWaves][ASJ_WAVE];  // key lengths
    __shared__ int32_t kex[kWaves][ASJ_WAVE];  // exclusive prefix of chunk counts
    __shared__ uint32_t kacc[kWaves][ASJ_WAVE]; // signature accumulators, then mismatch flags
    __shared__ uint32_t kacc2[kHi ? kWaves : 1][ASJ_WAVE]; // high-word accumulators
    __shared__ asj_pair kout[kWaves][kStage];   // result pairs staged before one output reservation

    if (*a.table_status != 0 || (a.probe_status && *a.probe_status != 0)) { // the whole grid leaves
        if (blockIdx.x == 0) {
            if (!BATCH && threadIdx.x == 0) *a.out_count = -1;
            if (BATCH)
                for (int j = threadIdx.x; j < a.njoins; j += kBlock) a.out_count[j] = -1;
        }
        return;
    }
    if (!PRESIGNED) asj::load_tables<MODE, kBlock>(tab, gtab);

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / ASJ_WAVE);
    const int lane = threadIdx.x % ASJ_WAVE;
    const uint64_t lanemask_lt = (1ull << lane) - 1ull;
    int64_t *wst = kst[wave];
    int64_t *wrs = krs[wave];
    int32_t *wln = kln[wave];
    int32_t *wex = kex[wave];
    uint32_t *wacc = kacc[wave];
    int64_t wave_cand = 0;
    asj_pair *wout = kout[wave];
    int nstage = 0;     // staged pairs (wave-uniform)
    int stage_join = 0; // join of the current window (batch mode)
    // reserve output space for the staged pairs with one atomic and copy them out
    auto flush = [&]() {
        if (nstage == 0) return;
        int64_t *cnt_p = a.out_count;
        asj_pair *out_p = a.out;
        int64_t cap_p = a.cap;
        if (BATCH) {
            const int64_t o0 = a.out_seg[stage_join];
            cnt_p = a.out_count + stage_join;
            out_p = a.out + o0;
            cap_p = a.out_seg[stage_join + 1] - o0;
        }
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd((unsigned long long *)cnt_p, (unsigned long long)nstage);
        base = __shfl(base, 0, ASJ_WAVE);
        asj_wave_sync();
        for (int t = lane; t < nstage; t += ASJ_WAVE) {
            const int64_t idx = (int64_t)base + t;
            if (idx < cap_p) out_p[idx] = wout[t];
        }
        asj_wave_sync();
        nstage = 0;
    };

    const bool pairs_out = a.kind == ASJ_KIND_INNER || a.kind == ASJ_KIND_LEFT; // the matching pairs themselves
    // where the probe keys' and (for the plain join's first-chunk compare)
    // the build keys' bytes end: short keys are read wide before these
    const int64_t send = a.n > 0 ? a.soff[a.n] : 0;
    const int64_t rend = (PLAIN && a.rn > 0) ? a.roff[a.rn] : 0;
    const int kpw = a.keys_per_window;
    const int64_t nwin = BATCH ? min((int64_t)*a.nwin, a.nwin_cap) : (a.n + kpw - 1) / kpw;
    const int64_t stride = (int64_t)gridDim.x * kWaves;
    // What starts the next window -- its map entry (batch), or its keys'
    // offsets and ids (single join) -- is requested while the current window
    // is processed, so a window does not begin with a chain of dependent
    // loads.  Vector loads (every lane asks for the same entry), so that the
    // requests wait in the in-order vector queue and not in the counter the
    // LDS operations share with scalar loads.
    asj_win pre_w = {0, 0, 0};
    int64_t pre_o0 = 0, pre_o1 = 0;
    int32_t pre_id = 0;
    auto prefetch = [&](int64_t w) {
        if (w >= nwin) return;
        if (BATCH) {
            pre_w = a.wins[w];
        } else {
            const int64_t kk = w * kpw + lane;
            if (lane < kpw && kk < a.n) {
                pre_o0 = a.soff[kk];
                pre_o1 = a.soff[kk + 1];
                pre_id = a.sids ? a.sids[kk] : (int32_t)kk;
            }
        }
    };
    prefetch((int64_t)blockIdx.x * kWaves + wave);
    for (int64_t win = (int64_t)blockIdx.x * kWaves + wave; win < nwin; win += stride) {
        // the window's rows, its join and table segment
        int64_t k0 = win * kpw;
        int rows = (int)min((int64_t)kpw, a.n - k0);
        int j = 0;
        const uint64_t *slots = a.slots;
        uint64_t mask = a.mask;
        int64_t ss = 0;
        int ls = 0;
        int32_t sid = 0;
        if (BATCH) {
            j = __builtin_amdgcn_readfirstlane(pre_w.join);
            rows = __builtin_amdgcn_readfirstlane(pre_w.rows);
            k0 = ((int64_t)__builtin_amdgcn_readfirstlane((uint32_t)(pre_w.first >> 32)) << 32) |
                 (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)pre_w.first);
            const asj_join_desc d = a.desc[j];
            slots = a.slots + d.tbase;
            mask = d.mask;
            stage_join = j;
        }
        const int64_t k = k0 + lane;
        const bool valid = lane < rows && k >= 0 && k < a.n;
        if (BATCH) {
            if (valid) {
                ss = a.soff[k];
                ls = (int)(a.soff[k + 1] - ss);
                sid = a.sids ? a.sids[k] : (int32_t)k;
            }
        } else if (valid) {
            ss = pre_o0;
            ls = (int)(pre_o1 - pre_o0);
            sid = pre_id;
        }
        prefetch(win + stride);
        uint32_t sg = 0, sg_hi = 0;
        if (PRESIGNED) {
            if (valid) sg = a.ssig[k];
        } else {
            sg = asj::sign_window<MODE, NSYM>(a.sdata, ss, ls, send, wst, wex, wacc, wln, tab,
                                              kacc2[kHi ? wave : 0], sg_hi);
        }

        Walk wk;
        wk.h = asj_mix32(sg) & mask;
        wk.qb = ~0ull;
        wk.walking = valid;
        int lane_cand = 0;
        bool matched = false; // this lane's key has a verified (or, unverified, signature-equal) match
        for (;;) {
            uint32_t r = 0;
            const bool walked = next_candidate<PLAIN>(slots, mask, sg, wk, r);
            const uint64_t hm = __ballot(walked);
            if (hm == 0) break;
            bool has = walked;
            if (kHi && has) has = a.rsig_hi[r] == sg_hi;
            wave_cand += __popcll(kHi ? __ballot(has) : hm);
            lane_cand += has ? 1 : 0;

            bool ok = has;
            if (VERIFY) {
                int64_t rs = 0;
                int lr = -1;
                if (has) {
                    const asj_u64x2a8 o = *(const asj_u64x2a8 *)(a.roff + r); // offsets r, r + 1
                    rs = (int64_t)o.x;
                    lr = (int)((int64_t)o.y - rs);
                }
                bool eq = has && lr == ls;
                if (PLAIN && eq) {
                    // The plain table offers every occupied slot as a candidate, so
                    // most equal-length pairs differ: each lane compares its pair's
                    // first 64 bytes (or whole key) alone, and only pairs that agree
                    // there go on to the chunk passes below.
                    uint32_t kr[16], ks[16], diff = 0;
                    if (ls >= ASJ_CHUNK) {
                        asj_load_full(a.rdata, rs, kr);
                        asj_load_full(a.sdata, ss, ks);
                    } else {
                        asj_load_tail_fast(a.rdata, rs, ls, rend, kr);
                        asj_load_tail_fast(a.sdata, ss, ls, send, ks);
                    }
#pragma unroll
                    for (int t = 0; t < 16; t++) diff |= kr[t] ^ ks[t];
                    eq = diff == 0;
                }
                // the (remaining) chunks of every equal-length pair, one per lane
                constexpr int kFirst = PLAIN ? 1 : 0; // chunks already compared
                const int nch = eq ? max(0, (ls + ASJ_CHUNK - 1) / ASJ_CHUNK - kFirst) : 0;
                const int incl = asj_wave_incl_scan(nch);
                const int total = __shfl(incl, ASJ_WAVE - 1, ASJ_WAVE);
                wst[lane] = ss;
                wrs[lane] = rs;
                wln[lane] = ls;
                wex[lane] = incl - nch;
                wacc[lane] = 0;
                asj_wave_sync();
                for (int base = 0; base < total; base += ASJ_WAVE) {
                    const int x = base + lane;
                    if (x < total) {
                        const int i = asj_find_owner(wex, x);
                        const int c = x - wex[i] + kFirst;
                        const int L = wln[i];
                        uint32_t diff = 0;
                        if (L >= ASJ_CHUNK) {
                            // chunk c covers [64c, 64c + 64); the last one ends at
                            // the key's end, [L - 64, L), overlapping its neighbour
                            const int64_t k0 = (c + 1) * ASJ_CHUNK <= L ? (int64_t)c * ASJ_CHUNK : (int64_t)(L - ASJ_CHUNK);
                            uint32_t kr[16], ks[16];
                            asj_load_full(a.rdata, wrs[i] + k0, kr);
                            asj_load_full(a.sdata, wst[i] + k0, ks);
#pragma unroll
                            for (int t = 0; t < 16; t++) diff |= kr[t] ^ ks[t];
                        } else {
                            uint32_t kr[16], ks[16];
                            asj_load_tail(a.rdata, wrs[i], L, kr);
                            asj_load_tail(a.sdata, wst[i], L, ks);
#pragma unroll
                            for (int t = 0; t < 16; t++) diff |= kr[t] ^ ks[t];
                        }
                        if (diff) wacc[i] = 1u; // every writer stores the same value
                    }
                }
                asj_wave_sync();
                ok = eq && wacc[lane] == 0u;
                asj_wave_sync();
            }
            // stage the survivors in LDS; output space is reserved per flush
            matched = matched || ok;
            const bool emit = ok && pairs_out;
            const uint64_t m = __ballot(emit);
            if (emit) {
                asj_pair p;
                p.r_id = a.rids ? a.rids[r] : (int32_t)r;
                p.s_id = sid;
                wout[nstage + __popcll(m & lanemask_lt)] = p;
            }
            nstage += __popcll(m);
            if (nstage > kStage - ASJ_WAVE) flush();
        }
        if (a.kind != ASJ_KIND_INNER) {
            // semi: matched probe rows; anti and left outer: unmatched ones
            const bool emit = valid && (a.kind == ASJ_KIND_SEMI ? matched : !matched);
            const uint64_t m = __ballot(emit);
            if (emit) {
                asj_pair p;
                p.r_id = -1;
                p.s_id = sid;
                wout[nstage + __popcll(m & lanemask_lt)] = p;
            }
            nstage += __popcll(m);
            if (nstage > kStage - ASJ_WAVE) flush();
        }
        if (BATCH) {
            flush(); // a join's pairs are all out before its rows are counted done
            const int cands = wave_sum(lane_cand);
            const unsigned long long rows = __popcll(__ballot(valid));
            if (lane == 0 && rows) {
                if (a.cand_count && cands) atomicAdd((unsigned long long *)(a.cand_count + j), (unsigned long long)cands);
                if (a.done_clock) { // the wave that finishes a join's last rows stamps its completion
                    const unsigned long long before = atomicAdd((unsigned long long *)(a.rows_done + j), rows);
                    if ((int64_t)(before + rows) == a.s_seg[j + 1] - a.s_seg[j]) a.done_clock[j] = wall_clock64();
                }
            }
        }
    }
    flush();
    if (!BATCH && a.cand_count && lane == 0 && wave_cand)
        atomicAdd((unsigned long long *)a.cand_count, (unsigned long long)wave_cand);
}

// Blocks of `kernel` that the device holds at once (blocks per compute unit
// from the occupancy calculator x compute units); 0 when the runtime cannot
// say.
int64_t resident_blocks(const void *kernel, int block)
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

template <int MODE, int NSYM, int PLAIN, int VERIFY, int PRESIGNED>
hipError_t launch(const asj_probe_args *a, const uint16_t *tab, int grid_cap, hipStream_t st)
{
    const int64_t nwin = a->njoins > 0 ? a->nwin_cap : (a->n + a->keys_per_window - 1) / a->keys_per_window;
    constexpr int kBlock = Shape<PRESIGNED>::block;
    constexpr int kWaves = Shape<PRESIGNED>::waves;
    int64_t blocks = (nwin + kWaves - 1) / kWaves;
    if (blocks > grid_cap) blocks = grid_cap;
    if (a->grid_rounds > 0) { // the grid in rounds of resident blocks
        static const int64_t res_batch = resident_blocks(
            reinterpret_cast<const void *>(&probe_kernel<MODE, NSYM, PLAIN, VERIFY, 1, PRESIGNED>), kBlock);
        static const int64_t res_single = resident_blocks(
            reinterpret_cast<const void *>(&probe_kernel<MODE, NSYM, PLAIN, VERIFY, 0, PRESIGNED>), kBlock);
        const int64_t resident = a->njoins > 0 ? res_batch : res_single;
        if (resident > 0 && blocks > resident * a->grid_rounds) blocks = resident * a->grid_rounds;
    }
    if (blocks < 1) blocks = 1;
    if (a->njoins > 0)
        hipLaunchKernelGGL((probe_kernel<MODE, NSYM, PLAIN, VERIFY, 1, PRESIGNED>), dim3((unsigned)blocks),
                           dim3(kBlock), 0, st, *a, tab);
    else
        hipLaunchKernelGGL((probe_kernel<MODE, NSYM, PLAIN, VERIFY, 0, PRESIGNED>), dim3((unsigned)blocks),
                           dim3(kBlock), 0, st, *a, tab);
    return hipGetLastError();
}

template <int MODE, int NSYM>
hipError_t launch_sig(const asj_probe_args *a, const uint16_t *tab, int grid_cap, hipStream_t st)
{
    return a->verify ? launch<MODE, NSYM, 0, 1, 0>(a, tab, grid_cap, st)
                     : launch<MODE, NSYM, 0, 0, 0>(a, tab, grid_cap, st);
}

} // namespace

hipError_t asj_launch_probe(const asj_probe_args *a_in, int mode, int nsym, const uint16_t *tab, int grid_cap,
                            hipStream_t st)
{
    asj_probe_args fixed = *a_in;
    if (fixed.keys_per_window < 1 || fixed.keys_per_window > ASJ_WAVE) fixed.keys_per_window = ASJ_WAVE;
    const asj_probe_args *a = &fixed;
    if (nsym == 4 && mode == ASJ_MODE_SIG16) { // 64-bit signatures: fused schedule only
        if (a->ssig || !a->rsig_hi) return hipErrorInvalidValue;
        return launch_sig<ASJ_MODE_SIG16, 4>(a, tab, grid_cap, st);
    }
    if (a->ssig) { // signatures (or plain hashes) of the probe keys are given: no signing, no tables
        if (a->plain) return launch<ASJ_MODE_PLAIN, 1, 1, 1, 1>(a, tab, grid_cap, st);
        return a->verify ? launch<ASJ_MODE_SIG16, 2, 0, 1, 1>(a, tab, grid_cap, st)
                         : launch<ASJ_MODE_SIG16, 2, 0, 0, 1>(a, tab, grid_cap, st);
    }
    if (a->plain) return launch<ASJ_MODE_PLAIN, 1, 1, 1, 0>(a, tab, grid_cap, st);
    if (mode == ASJ_MODE_PLAIN) return launch<ASJ_MODE_PLAIN, 1, 0, 1, 0>(a, tab, grid_cap, st); // fingerprint
    if (mode == ASJ_MODE_SIG16 && nsym == 2) return launch_sig<ASJ_MODE_SIG16, 2>(a, tab, grid_cap, st);
    if (mode == ASJ_MODE_SIG16 && nsym == 1) return launch_sig<ASJ_MODE_SIG16, 1>(a, tab, grid_cap, st);
    if (mode == ASJ_MODE_SIG8 && nsym == 4) return launch_sig<ASJ_MODE_SIG8, 4>(a, tab, grid_cap, st);
    if (mode == ASJ_MODE_SIG8 && nsym == 2) return launch_sig<ASJ_MODE_SIG8, 2>(a, tab, grid_cap, st);
    return hipErrorInvalidValue;
}
