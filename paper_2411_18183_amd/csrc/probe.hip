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
// byte comparison stops after the first 16 bytes when they differ.
// In batch mode windows never span two joins: a window reads its join from
// the window map, probes that join's table segment, appends to that join's
// output segment, and the wave that finishes a join's last probe row stamps
// its completion clock.
// A batch's joins with few build rows are probed against LDS tables (the
// LOCAL form, which takes all of a batch's windows in one launch): the grid
// is split between the two kinds of window in proportion to their counts; a
// block of the LDS-table part takes an equal share of those windows and,
// for every join in its share, first builds the join's table in LDS from the
// build signatures (a bucket per value of the low bits of mix32(signature),
// entries ordered by bucket with a counting sort), so a walk is a few LDS
// reads and no device-memory table is written, initialised or read.  A
// single join with few build rows runs the LOCAL form too: every block
// builds the whole table, then takes every grid-th window.
// Right and full outer joins: every verified match marks its build row in a
// byte array, and unmatched_build_kernel appends the unmarked rows.
#include "sign_window.h"

namespace {

// Block size: 8 waves when the kernel signs (one copy of the GF tables in
// LDS serves more waves), 4 waves when the signatures are given (no tables;
// the smaller block fits the register-limited wave count per CU exactly),
// 16 with an LDS table (one block per CU holds the tables and the join's
// table).  stage = result pairs staged per wave; flushed once more than
// stage - 64 wait.
template <int PRESIGNED, int LOCAL>
struct Shape {
    static constexpr int block = LOCAL ? 1024 : PRESIGNED ? 256 : 512;
    static constexpr int waves = block / ASJ_WAVE;
    static constexpr int stage = LOCAL ? 128 : 256;
};
// LDS table buckets: the plain baseline keeps no signature per entry, so
// every entry of its bucket is a candidate; the LDS the signatures would
// take holds four times the buckets instead (0.6 entries per bucket at the
// size limit).
template <int PLAIN>
struct LocalBuckets {
    static constexpr int value = PLAIN ? 16384 : 4096;
};

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

// Next candidate of a lane's LDS-table bucket (entries cur .. end); true
// with *r = the entry's build row within its join.
template <int PLAIN>
__device__ __forceinline__ bool next_local(const uint32_t *lsig, const uint16_t *lrow, uint32_t sg, uint32_t &cur,
                                           uint32_t end, uint32_t &r)
{
    while (cur < end) {
        const uint32_t i = cur++;
        if (PLAIN || lsig[i] == sg) {
            r = lrow[i];
            return true;
        }
    }
    return false;
}

// The LDS table of build rows r0 .. r0 + nr (whole block; nr <=
// ASJ_LOCAL_ROWS): their signatures rsig[..] read once into registers,
// bucket counts, their exclusive prefix sums, then every entry placed at its
// bucket's next position, which leaves lend[b] at the end of bucket b (the
// bucket is the low bits of mix32(signature); lsig is unused for PLAIN).
template <int kBlock, int kBuckets, int PLAIN>
__device__ __forceinline__ void build_lds_table(const uint32_t *__restrict__ rsig, int64_t r0, int nr, uint32_t *lend,
                                                uint32_t *lsig, uint16_t *lrow, uint32_t *lwsum, int lane, int wave)
{
    constexpr int kPer = (ASJ_LOCAL_ROWS + kBlock - 1) / kBlock;
    uint32_t rsg[kPer];
#pragma unroll
    for (int q = 0; q < kPer; q++) {
        const int i = (int)threadIdx.x + q * kBlock;
        rsg[q] = i < nr ? rsig[r0 + i] : 0u;
    }
    __syncthreads(); // the previous table's lookups are over
    for (int b = threadIdx.x; b < kBuckets; b += kBlock) lend[b] = 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; q++)
        if ((int)threadIdx.x + q * kBlock < nr) atomicAdd(&lend[asj_mix32(rsg[q]) & (uint32_t)(kBuckets - 1)], 1u);
    __syncthreads();
    {
        constexpr int per = kBuckets / kBlock; // consecutive buckets per thread
        uint32_t c[per], sum = 0;
#pragma unroll
        for (int q = 0; q < per; q++) {
            c[q] = lend[threadIdx.x * per + q];
            sum += c[q];
        }
        const int incl = asj_wave_incl_scan((int)sum);
        if (lane == ASJ_WAVE - 1) lwsum[wave] = (uint32_t)incl;
        __syncthreads();
        uint32_t before = 0;
        for (int q = 0; q < wave; q++) before += lwsum[q];
        uint32_t run = before + (uint32_t)incl - sum;
#pragma unroll
        for (int q = 0; q < per; q++) {
            lend[threadIdx.x * per + q] = run;
            run += c[q];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; q++) {
        const int i = (int)threadIdx.x + q * kBlock;
        if (i < nr) {
            const uint32_t pos = atomicAdd(&lend[asj_mix32(rsg[q]) & (uint32_t)(kBuckets - 1)], 1u);
            if (!PLAIN) lsig[pos] = rsg[q];
            lrow[pos] = (uint16_t)i;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, ASJ_WAVE);
    return v;
}

template <int MODE, int NSYM, int PLAIN, int VERIFY, int BATCH, int PRESIGNED, int LOCAL>
// At most 128 registers (4 waves per SIMD): above that only one block fits a
// CU.
__global__ __launch_bounds__((Shape<PRESIGNED, LOCAL>::block), 4) void probe_kernel(
    asj_probe_args a, const uint16_t *__restrict__ gtab)
{
    constexpr int kBlock = Shape<PRESIGNED, LOCAL>::block;
    constexpr int kWaves = Shape<PRESIGNED, LOCAL>::waves;
    constexpr int kStage = Shape<PRESIGNED, LOCAL>::stage;
    constexpr int kBuckets = LocalBuckets<PLAIN>::value;
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
    // LDS table of the current join: bucket b holds entries lend[b-1] ..
    // lend[b] (lend[-1] = 0) with the build rows' signatures and rows
    __shared__ uint32_t lend[LOCAL ? kBuckets : 1];
    __shared__ uint32_t lsig[LOCAL && !PLAIN ? ASJ_LOCAL_ROWS : 1];
    __shared__ uint16_t lrow[LOCAL ? ASJ_LOCAL_ROWS : 1];
    __shared__ uint32_t lwsum[LOCAL ? kWaves : 1];

    if (*a.table_status != 0 || (a.probe_status && *a.probe_status != 0)) { // the whole grid leaves
        if (blockIdx.x == 0) {
            if (!BATCH && threadIdx.x == 0) *a.out_count = -1;
            if (BATCH)
                for (int j = threadIdx.x; j < a.njoins; j += kBlock) a.out_count[j] = -1;
        }
        return;
    }
    const int kpw = a.keys_per_window;
    // Windows of this launch: every ngrid * kWaves-th device-table window
    // from gblk * kWaves + wave on (gblk = block index, ngrid = grid) and,
    // LOCAL, the share [w_lo, w_hi) of the LDS-table windows.  LOCAL splits
    // the grid between the two kinds in proportion to their window counts:
    // blocks 0 .. gl - 1 take equal shares of the LDS-table windows, the
    // others the device-table windows (a one-block grid takes both).  A
    // block without windows leaves at once, before it loads the tables.
    int64_t nwin = BATCH ? min((int64_t)*a.nwin, a.nwin_cap) : (a.n + kpw - 1) / kpw;
    int64_t w_lo = 0, w_hi = 0, gblk = blockIdx.x, ngrid = gridDim.x;
    bool do_glob = true;
    // a single join against an LDS table: every block builds the whole table
    // (at most ASJ_LOCAL_ROWS build rows) and takes windows like a single join
    constexpr bool kLocalSingle = LOCAL && !BATCH;
    if (LOCAL && BATCH) {
        const int64_t nl = min((int64_t)*a.nwin_l, a.nwin_l_cap);
        const int64_t G = gridDim.x, b = blockIdx.x;
        int64_t gl = 0;
        if (nl > 0) gl = nwin == 0 ? G : min(G - 1, max((int64_t)1, (G * nl + (nl + nwin) / 2) / (nl + nwin)));
        if (G == 1) {
            w_hi = nl;
        } else if (b < gl) {
            w_lo = nl * b / gl;
            w_hi = nl * (b + 1) / gl;
            do_glob = false;
        } else {
            gblk = b - gl;
            ngrid = G - gl;
        }
    }
    if (do_glob && gblk * kWaves >= nwin) do_glob = false;
    if (!do_glob && w_lo >= w_hi) return;
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
    int64_t join_cand = 0; // candidates of stage_join not yet added to its count (batch mode)
    // reserve output space for the staged pairs with one atomic and copy them out
    // (every lambda below is inlined at each use: a call would spill the
    // kernel's registers)
    auto flush = [&]() __attribute__((always_inline)) {
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
    // batch mode: the staged pairs and the candidate count of stage_join out
    // before the wave's windows move to another join
    auto flush_join = [&]() __attribute__((always_inline)) {
        flush();
        if (BATCH && join_cand) {
            if (lane == 0) atomicAdd((unsigned long long *)(a.cand_count + stage_join), (unsigned long long)join_cand);
            join_cand = 0;
        }
    };

    // the matching pairs themselves (every kind but the semi- and anti-join)
    const bool pairs_out = a.kind != ASJ_KIND_SEMI && a.kind != ASJ_KIND_ANTI;
    // where the probe keys' bytes end: short keys are read wide before it
    const int64_t send = a.n > 0 ? a.soff[a.n] : 0;
    // What starts the next window -- its map entry (batch), or its keys'
    // offsets and ids (single join, LDS-table windows) -- is requested while
    // the current window is processed, so a window does not begin with a
    // chain of dependent loads.  Vector loads (every lane asks for the same
    // entry), so that the requests wait in the in-order vector queue and not
    // in the counter the LDS operations share with scalar loads.
    asj_win pre_w = {0, 0, 0};
    int64_t pre_o0 = 0, pre_o1 = 0;
    int32_t pre_id = 0;
    int64_t pre_end = 0; // LDS-table windows: end of the current join's probe rows
    // w = the next window (lw, an LDS-table window: its first row, < 0 for none)
    auto prefetch = [&](int64_t w, bool lw) __attribute__((always_inline)) {
        if (LOCAL && lw) {
            const int64_t kk = w + lane;
            if (w >= 0 && lane < kpw && kk < pre_end) {
                pre_o0 = a.soff[kk];
                pre_o1 = a.soff[kk + 1];
                pre_id = a.sids ? a.sids[kk] : (int32_t)kk;
            }
            return;
        }
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

    // One window: probe rows k0 .. k0 + rows (of join j in batch mode)
    // against the table segment (slots, mask) or, lw, the block's LDS table
    // of the join, whose build rows start at row rbase; the next window's
    // prefetch is issued once this one's rows are read.
    auto window = [&](int j, int64_t k0, int rows, const uint64_t *slots, uint64_t mask, int64_t rbase,
                      int64_t next, bool lw) __attribute__((always_inline)) {
        const int64_t k = k0 + lane;
        const bool valid = lane < rows && k >= 0 && k < a.n;
        int64_t ss = 0;
        int ls = 0;
        int32_t sid = 0;
        if (BATCH && !(LOCAL && lw)) {
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
        prefetch(next, lw);
        uint32_t sg = 0, sg_hi = 0;
        if (PRESIGNED) {
            if (valid) sg = a.ssig[k];
        } else {
            sg = asj::sign_window<MODE, NSYM>(a.sdata, ss, ls, send, wst, wex, wacc, wln, tab, gtab,
                                              kacc2[kHi ? wave : 0], sg_hi);
        }

        Walk wk;
        wk.h = asj_mix32(sg) & mask;
        wk.qb = ~0ull;
        wk.walking = valid;
        uint32_t lcur = 0, lstop = 0; // LDS table: the lane's bucket
        if (LOCAL && lw && valid) {
            const uint32_t bk = asj_mix32(sg) & (uint32_t)(kBuckets - 1);
            lcur = bk ? lend[bk - 1] : 0u;
            lstop = lend[bk];
        }
        int lane_cand = 0;
        bool matched = false; // this lane's key has a verified (or, unverified, signature-equal) match
        for (;;) {
            uint32_t r = 0;
            bool walked;
            if (LOCAL && lw) {
                walked = next_local<PLAIN>(lsig, lrow, sg, lcur, lstop, r);
                r += (uint32_t)rbase;
            } else {
                walked = next_candidate<PLAIN>(slots, mask, sg, wk, r);
            }
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
                    // equal-length pairs often differ: each lane compares its pair's
                    // first 16 bytes alone, and only pairs that agree there go on to
                    // the chunk passes below.  (Sixteen bytes: a 64-byte first chunk
                    // held two raw chunks in registers and made the kernels spill.)
                    uint32_t kr[4], ks[4], diff = 0;
                    asj_load_head16(a.rdata, rs, ls, kr);
                    asj_load_head16(a.sdata, ss, ls, ks);
#pragma unroll
                    for (int t = 0; t < 4; t++) diff |= kr[t] ^ ks[t];
                    eq = diff == 0;
                }
                // every chunk of every equal-length pair, one per lane
                constexpr int kFirst = 0; // chunks already compared
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
                            const int64_t c0 = (c + 1) * ASJ_CHUNK <= L ? (int64_t)c * ASJ_CHUNK : (int64_t)(L - ASJ_CHUNK);
                            uint32_t kr[16], ks[16];
                            asj_load_full(a.rdata, wrs[i] + c0, kr);
                            asj_load_full(a.sdata, wst[i] + c0, ks);
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
            if (ok && a.rmatch) a.rmatch[r] = 1; // right and full outer joins: this build row has a match
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
        if (a.kind != ASJ_KIND_INNER && a.kind != ASJ_KIND_RIGHT) {
            // semi: matched probe rows; anti, left and full outer: unmatched ones
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
            // staged pairs and the candidate count stay with the wave until
            // its windows move to another join (or the stage fills); only
            // the completion clocks need a join's pairs out after every
            // window, before its rows are counted done
            if (a.done_clock) {
                flush();
                const unsigned long long nrows = __popcll(__ballot(valid));
                if (lane == 0 && nrows) { // the wave that finishes a join's last rows stamps its completion
                    const unsigned long long before = atomicAdd((unsigned long long *)(a.rows_done + j), nrows);
                    if ((int64_t)(before + nrows) == a.s_seg[j + 1] - a.s_seg[j]) a.done_clock[j] = wall_clock64();
                }
            }
            if (a.cand_count) join_cand += (uint32_t)__builtin_amdgcn_readfirstlane(wave_sum(lane_cand));
        }
    };


    if constexpr (LOCAL && BATCH) {
        // this block's share of the LDS-table windows, join by join
        for (int64_t w = w_lo; w < w_hi;) { // block-uniform
            const int j = __builtin_amdgcn_readfirstlane(a.win_l[w]);
            const int64_t wb = a.desc[j].wbase_l;
            const int64_t s0 = a.s_seg[j], s1 = a.s_seg[j + 1];
            const int64_t r0 = a.r_seg[j];
            const int nr = (int)min((int64_t)ASJ_LOCAL_ROWS, max((int64_t)0, a.r_seg[j + 1] - r0));
            const int64_t w_end = min(w_hi, wb + (s1 - s0 + kpw - 1) / kpw);
            if (w_end <= w) break; // a map entry outside its join's windows: nothing sane to do
            // this wave's first window of the join
            pre_end = s1;
            if (w + wave < w_end) prefetch(s0 + (w + wave - wb) * kpw, true);
            build_lds_table<kBlock, kBuckets, PLAIN>(a.rsig, r0, nr, lend, lsig, lrow, lwsum, lane, wave);
            stage_join = j;
            for (int64_t win = w + wave; win < w_end; win += kWaves) {
                const int64_t k0 = s0 + (win - wb) * kpw;
                const int64_t nxt = win + kWaves < w_end ? k0 + (int64_t)kWaves * kpw : -1;
                window(j, k0, (int)min((int64_t)kpw, s1 - k0), nullptr, 0, r0, nxt, true);
            }
            flush_join(); // the next join's pairs go to another output segment
            w = w_end;
        }
    }
    if (do_glob) {
        const int64_t stride = ngrid * kWaves;
        const int64_t first = gblk * kWaves + wave;
        if constexpr (kLocalSingle) { // the table, and the first window's rows (prefetch takes rows here)
            pre_end = a.n;
            prefetch(first < nwin ? first * kpw : -1, true);
            build_lds_table<kBlock, kBuckets, PLAIN>(a.rsig, 0, (int)min((int64_t)ASJ_LOCAL_ROWS, a.rn), lend, lsig,
                                                     lrow, lwsum, lane, wave);
        } else {
            prefetch(first, false);
        }
        for (int64_t win = first; win < nwin; win += stride) {
            // the window's rows, its join and table segment
            int64_t k0 = win * kpw;
            int rows = (int)min((int64_t)kpw, a.n - k0);
            int j = 0;
            const uint64_t *slots = a.slots;
            uint64_t mask = a.mask;
            if (BATCH) {
                j = __builtin_amdgcn_readfirstlane(pre_w.join);
                rows = __builtin_amdgcn_readfirstlane(pre_w.rows);
                k0 = ((int64_t)__builtin_amdgcn_readfirstlane((uint32_t)(pre_w.first >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)pre_w.first);
                const asj_join_desc d = a.desc[j];
                slots = a.slots + d.tbase;
                mask = d.mask;
                if (j != stage_join) flush_join();
                stage_join = j;
            }
            if constexpr (kLocalSingle)
                window(0, k0, rows, nullptr, 0, 0, win + stride < nwin ? (win + stride) * kpw : -1, true);
            else
                window(j, k0, rows, slots, mask, 0, win + stride, false);
        }
    }
    if constexpr (BATCH) {
        flush_join();
    } else {
        // The waves' last staged pairs and their candidate counts go out
        // with one output reservation and one count per block: the waves of
        // a grid finish together, and one atomic per wave on the same two
        // words made a queue at the end of the kernel (44 us of a 200 us
        // probe of 131k keys of 4 KB, one grid round).  Every wave of the
        // block gets here (the only returns above are the block's).
        __shared__ int32_t bn[kWaves];
        __shared__ int64_t bc[kWaves];
        __shared__ unsigned long long bbase;
        if (lane == 0) {
            bn[wave] = nstage;
            bc[wave] = wave_cand;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t tn = 0, tc = 0;
            for (int w = 0; w < kWaves; w++) {
                tn += bn[w];
                tc += bc[w];
            }
            bbase = tn ? atomicAdd((unsigned long long *)a.out_count, (unsigned long long)tn) : 0ull;
            if (a.cand_count && tc) atomicAdd((unsigned long long *)a.cand_count, (unsigned long long)tc);
        }
        __syncthreads();
        int64_t base = (int64_t)bbase;
        for (int w = 0; w < wave; w++) base += bn[w];
        for (int t = lane; t < nstage; t += ASJ_WAVE)
            if (base + t < a.cap) a.out[base + t] = wout[t];
    }
}

// (r_id, -1) for each build row without a match (see
// asj_launch_unmatched_build).  A block of 1024 lanes takes 1024 consecutive
// rows per step.  When they lie in one join (always for a single join), the
// block reserves output space for its unmatched rows with one atomic: the
// blocks start together, and an atomic per wave on the same count made a
// queue (192 us for 1M build rows, 17 us with one per block).  A step that
// spans joins has each wave reserve once per join among its rows.
constexpr int kUnmatchedBlock = 1024;

__device__ __forceinline__ int join_of_row(const int64_t *__restrict__ r_seg, int32_t J, int64_t r)
{
    int lo = 0, hi = J; // r_seg[lo] <= r < r_seg[hi] throughout (r_seg[0] = 0, r_seg[J] = m)
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (r_seg[mid] <= r) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kUnmatchedBlock) void unmatched_build_kernel(const uint8_t *__restrict__ rmatch,
                                                                          const int32_t *__restrict__ rids,
                                                                          int64_t m, asj_pair *__restrict__ out,
                                                                          int64_t cap,
                                                                          int64_t *__restrict__ out_count,
                                                                          const int32_t *__restrict__ status1,
                                                                          const int32_t *__restrict__ status2,
                                                                          int32_t J,
                                                                          const int64_t *__restrict__ r_seg,
                                                                          const int64_t *__restrict__ out_seg)
{
    if ((status1 && *status1 != 0) || (status2 && *status2 != 0)) return;
    constexpr int kW = kUnmatchedBlock / ASJ_WAVE;
    __shared__ uint32_t wcnt[kW];
    __shared__ unsigned long long bbase;
    const int lane = threadIdx.x % ASJ_WAVE, wave = threadIdx.x / ASJ_WAVE;
    const uint64_t lanemask_lt = (1ull << lane) - 1ull;
    for (int64_t b0 = (int64_t)blockIdx.x * kUnmatchedBlock; b0 < m; b0 += (int64_t)gridDim.x * kUnmatchedBlock) {
        const int64_t r = b0 + threadIdx.x; // (the loop and jf, jl are block-uniform)
        const bool emit = r < m && rmatch[r] == 0;
        const int jf = J > 0 ? join_of_row(r_seg, J, b0) : 0;
        const int jl = J > 0 ? join_of_row(r_seg, J, min(b0 + kUnmatchedBlock, m) - 1) : 0;
        if (jf == jl) { // one join: one reservation for the block
            const uint64_t bal = __ballot(emit);
            if (lane == 0) wcnt[wave] = (uint32_t)__popcll(bal);
            __syncthreads();
            if (threadIdx.x == 0) {
                uint32_t t = 0;
                for (int w = 0; w < kW; w++) t += wcnt[w];
                bbase = t ? atomicAdd((unsigned long long *)(out_count + jf), (unsigned long long)t) : 0ull;
            }
            __syncthreads();
            if (emit) {
                int64_t o0 = 0, cp = cap;
                if (J > 0) {
                    o0 = out_seg[jf];
                    cp = out_seg[jf + 1] - o0;
                }
                int64_t idx = (int64_t)bbase + __popcll(bal & lanemask_lt);
                for (int w = 0; w < wave; w++) idx += wcnt[w];
                if (idx < cp) {
                    asj_pair p;
                    p.r_id = rids ? rids[r] : (int32_t)r;
                    p.s_id = -1;
                    out[o0 + idx] = p;
                }
            }
            __syncthreads(); // wcnt and bbase are the next step's
            continue;
        }
        const int j = emit ? join_of_row(r_seg, J, r) : 0;
        uint64_t pend = __ballot(emit);
        while (pend) { // one reservation per join among the wave's rows
            const int leader = __ffsll((unsigned long long)pend) - 1;
            const int jw = __shfl(j, leader, ASJ_WAVE);
            const bool mine = emit && j == jw;
            const uint64_t grp = __ballot(mine);
            const int64_t o0 = out_seg[jw], cp = out_seg[jw + 1] - o0;
            unsigned long long b = 0;
            if (lane == leader) b = atomicAdd((unsigned long long *)(out_count + jw), (unsigned long long)__popcll(grp));
            b = __shfl(b, leader, ASJ_WAVE);
            if (mine) {
                const int64_t idx = (int64_t)b + __popcll(grp & lanemask_lt);
                if (idx < cp) {
                    asj_pair p;
                    p.r_id = rids ? rids[r] : (int32_t)r;
                    p.s_id = -1;
                    out[o0 + idx] = p;
                }
            }
            pend &= ~grp;
        }
    }
}

template <int MODE, int NSYM, int PLAIN, int VERIFY, int PRESIGNED>
hipError_t launch(const asj_probe_args *a, const uint16_t *tab, int grid_cap, hipStream_t st)
{
    const int64_t nwin = a->njoins > 0 ? a->nwin_cap : (a->n + a->keys_per_window - 1) / a->keys_per_window;
    constexpr int kBlock = Shape<PRESIGNED, 0>::block;
    constexpr int kWaves = Shape<PRESIGNED, 0>::waves;
    int64_t blocks = (nwin + kWaves - 1) / kWaves;
    if (blocks > grid_cap) blocks = grid_cap;
    if (a->grid_rounds > 0) { // the grid in rounds of resident blocks
        static const int64_t res_batch = asj_resident_blocks(
            reinterpret_cast<const void *>(&probe_kernel<MODE, NSYM, PLAIN, VERIFY, 1, PRESIGNED, 0>), kBlock);
        static const int64_t res_single = asj_resident_blocks(
            reinterpret_cast<const void *>(&probe_kernel<MODE, NSYM, PLAIN, VERIFY, 0, PRESIGNED, 0>), kBlock);
        const int64_t resident = a->njoins > 0 ? res_batch : res_single;
        if (resident > 0 && blocks > resident * a->grid_rounds) blocks = resident * a->grid_rounds;
    }
    if (blocks < 1) blocks = 1;
    if (a->njoins > 0)
        hipLaunchKernelGGL((probe_kernel<MODE, NSYM, PLAIN, VERIFY, 1, PRESIGNED, 0>), dim3((unsigned)blocks),
                           dim3(kBlock), 0, st, *a, tab);
    else
        hipLaunchKernelGGL((probe_kernel<MODE, NSYM, PLAIN, VERIFY, 0, PRESIGNED, 0>), dim3((unsigned)blocks),
                           dim3(kBlock), 0, st, *a, tab);
    return hipGetLastError();
}

// All windows of a batch with LDS tables: grid_rounds x the resident blocks
// (one per compute unit), split between the two kinds of window on the
// device.
template <int MODE, int NSYM, int PLAIN, int VERIFY>
hipError_t launch_local(const asj_probe_args *a, const uint16_t *tab, hipStream_t st)
{
    constexpr int kBlock = Shape<0, 1>::block;
    static const int64_t resident =
        asj_resident_blocks(reinterpret_cast<const void *>(&probe_kernel<MODE, NSYM, PLAIN, VERIFY, 1, 0, 1>), kBlock);
    if (resident <= 0) return hipErrorInvalidValue; // the kernel does not fit a compute unit
    int64_t blocks = resident * (a->grid_rounds > 0 ? a->grid_rounds : 1);
    const int64_t most = (a->nwin_cap + a->nwin_l_cap) / Shape<0, 1>::waves + 2;
    if (blocks > most) blocks = most;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((probe_kernel<MODE, NSYM, PLAIN, VERIFY, 1, 0, 1>), dim3((unsigned)blocks), dim3(kBlock), 0,
                       st, *a, tab);
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

hipError_t asj_launch_unmatched_build(const uint8_t *rmatch, const int32_t *rids, int64_t m, asj_pair *out, int64_t cap,
                                      int64_t *out_count, const int32_t *status1, const int32_t *status2,
                                      int32_t njoins, const int64_t *r_seg, const int64_t *out_seg, hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    if (!rmatch || !out_count || (njoins > 0 && (!r_seg || !out_seg))) return hipErrorInvalidValue;
    int64_t blocks = (m + kUnmatchedBlock - 1) / kUnmatchedBlock;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(unmatched_build_kernel, dim3((unsigned)blocks), dim3(kUnmatchedBlock), 0, st, rmatch, rids, m,
                       out, cap, out_count, status1, status2, njoins, r_seg, out_seg);
    return hipGetLastError();
}

// A single join against LDS tables: every block builds the whole table of
// the a->rn <= ASJ_LOCAL_ROWS build rows from a->rsig, then takes every
// grid-th window; grid_rounds x the resident blocks at most.
template <int MODE, int NSYM, int PLAIN, int VERIFY>
hipError_t launch_local_single(const asj_probe_args *a, const uint16_t *tab, hipStream_t st)
{
    constexpr int kBlock = Shape<0, 1>::block;
    constexpr int kWaves = Shape<0, 1>::waves;
    static const int64_t resident =
        asj_resident_blocks(reinterpret_cast<const void *>(&probe_kernel<MODE, NSYM, PLAIN, VERIFY, 0, 0, 1>), kBlock);
    if (resident <= 0) return hipErrorInvalidValue;
    const int64_t nwin = (a->n + a->keys_per_window - 1) / a->keys_per_window;
    int64_t blocks = (nwin + kWaves - 1) / kWaves;
    const int64_t most = resident * (a->grid_rounds > 0 ? a->grid_rounds : 1);
    if (blocks > most) blocks = most;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((probe_kernel<MODE, NSYM, PLAIN, VERIFY, 0, 0, 1>), dim3((unsigned)blocks), dim3(kBlock), 0,
                       st, *a, tab);
    return hipGetLastError();
}

hipError_t asj_launch_probe_local_single(const asj_probe_args *a_in, int mode, int nsym, const uint16_t *tab,
                                         hipStream_t st)
{
    asj_probe_args fixed = *a_in;
    if (fixed.keys_per_window < 1 || fixed.keys_per_window > ASJ_WAVE) fixed.keys_per_window = ASJ_WAVE;
    const asj_probe_args *a = &fixed;
    if (!a->rsig || a->njoins != 0 || a->ssig || a->rn > ASJ_LOCAL_ROWS || !a->table_status)
        return hipErrorInvalidValue;
    if (a->plain) return launch_local_single<ASJ_MODE_PLAIN, 1, 1, 1>(a, tab, st);
#define ASJ_LOCAL_SIG(M, N)                                                                                       \
    if (mode == M && nsym == N)                                                                                   \
        return a->verify ? launch_local_single<M, N, 0, 1>(a, tab, st) : launch_local_single<M, N, 0, 0>(a, tab, st);
    ASJ_LOCAL_SIG(ASJ_MODE_SIG16, 2)
    ASJ_LOCAL_SIG(ASJ_MODE_SIG16, 1)
    ASJ_LOCAL_SIG(ASJ_MODE_SIG8, 4)
    ASJ_LOCAL_SIG(ASJ_MODE_SIG8, 2)
#undef ASJ_LOCAL_SIG
    return hipErrorInvalidValue;
}

hipError_t asj_launch_probe_local(const asj_probe_args *a_in, int mode, int nsym, const uint16_t *tab, hipStream_t st)
{
    asj_probe_args fixed = *a_in;
    if (fixed.keys_per_window < 1 || fixed.keys_per_window > ASJ_WAVE) fixed.keys_per_window = ASJ_WAVE;
    const asj_probe_args *a = &fixed;
    if (!a->win_l || !a->nwin_l || !a->r_seg || !a->rsig || !a->wins || !a->nwin || a->njoins < 1 || a->ssig)
        return hipErrorInvalidValue;
    if (a->plain) return launch_local<ASJ_MODE_PLAIN, 1, 1, 1>(a, tab, st);
#define ASJ_LOCAL_SIG(M, N)                                                                                       \
    if (mode == M && nsym == N)                                                                                   \
        return a->verify ? launch_local<M, N, 0, 1>(a, tab, st) : launch_local<M, N, 0, 0>(a, tab, st);
    ASJ_LOCAL_SIG(ASJ_MODE_SIG16, 2)
    ASJ_LOCAL_SIG(ASJ_MODE_SIG16, 1)
    ASJ_LOCAL_SIG(ASJ_MODE_SIG8, 4)
    ASJ_LOCAL_SIG(ASJ_MODE_SIG8, 2)
#undef ASJ_LOCAL_SIG
    return hipErrorInvalidValue;
}
