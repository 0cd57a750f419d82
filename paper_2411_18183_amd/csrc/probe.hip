// Probe(H_sign, s), candidate verification and output compaction
// (Section 3.2, Figure 2: probe the table with every tuple of S and output
// the matching tuples; Section 2: matching tuples are concatenated into T).
//
// One wave handles a window of 64 probe keys, one key per lane.  Each lane
// walks its key's run of slots from the home slot mix32(signature) until the
// first empty slot; every slot whose stored signature equals the key's is a
// candidate (the paper outputs candidates directly; here each one is also
// compared byte by byte unless verification is switched off).  The wave
// advances all walks in rounds of at most one candidate per lane:
//   1. candidates whose length differs from the probe key are rejected;
//   2. the remaining pairs are cut into full 64-byte key-relative chunks,
//      laid out back to back; passes of 64 chunks compare one chunk per lane
//      and flag mismatching pairs in LDS; each lane then compares its own
//      pair's partial last chunk;
//   3. surviving pairs are appended to the output with one atomic add per
//      wave and round (ballot + popcount prefix).
// The baseline simple hash join walks the same way but treats every
// occupied slot as a candidate (no stored signature to filter with).
#include "asj_internal.h"

namespace {

constexpr int kBlock = 512;
constexpr int kWaves = kBlock / ASJ_WAVE;

template <int PLAIN, int VERIFY>
__global__ __launch_bounds__(kBlock) void probe_kernel(asj_probe_args a)
{
    __shared__ int64_t crs[kWaves][ASJ_WAVE]; // candidate build key start
    __shared__ int64_t css[kWaves][ASJ_WAVE]; // probe key start
    __shared__ int32_t cex[kWaves][ASJ_WAVE]; // exclusive prefix of full-chunk counts
    __shared__ uint32_t cbad[kWaves][ASJ_WAVE];

    if (*a.table_status != 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *a.out_count = -1;
        return;
    }
    const int wave = threadIdx.x / ASJ_WAVE;
    const int lane = threadIdx.x % ASJ_WAVE;
    const uint64_t lanemask_lt = (1ull << lane) - 1ull;
    int64_t wave_cand = 0;

    const int64_t nwin = (a.n + ASJ_WAVE - 1) / ASJ_WAVE;
    for (int64_t w = (int64_t)blockIdx.x * kWaves + wave; w < nwin; w += (int64_t)gridDim.x * kWaves) {
        const int64_t k = w * ASJ_WAVE + lane;
        const bool valid = k < a.n;
        int64_t ss = 0;
        int32_t ls = 0;
        uint32_t sg = 0;
        uint64_t h = 0;
        int32_t sid = 0;
        if (valid) {
            ss = a.soff[k];
            ls = (int32_t)(a.soff[k + 1] - ss);
            sg = a.sig_s[k];
            h = asj_mix32(sg) & a.mask;
            sid = a.sids ? a.sids[k] : (int32_t)k;
        }
        bool walking = valid;
        for (;;) {
            bool has = false;
            uint32_t r = 0;
            while (walking) {
                const uint64_t slot = a.slots[h];
                if (slot == ASJ_EMPTY_SLOT) {
                    walking = false;
                    break;
                }
                h = (h + 1) & a.mask;
                if (PLAIN || (uint32_t)(slot >> 32) == sg) {
                    has = true;
                    r = (uint32_t)slot;
                    break;
                }
            }
            const uint64_t hm = __ballot(has);
            if (hm == 0) break;
            wave_cand += __popcll(hm);

            bool ok = has;
            if (VERIFY) {
                int64_t rs = 0;
                int32_t lr = -1;
                if (has) {
                    rs = a.roff[r];
                    lr = (int32_t)(a.roff[r + 1] - rs);
                }
                const bool eq = has && lr == ls;
                // full 64-byte chunks of every pair, 64 per pass, one per lane
                const int nfull = eq ? ls / ASJ_CHUNK : 0;
                const int incl = asj_wave_incl_scan(nfull);
                const int total = __shfl(incl, ASJ_WAVE - 1, ASJ_WAVE);
                crs[wave][lane] = rs;
                css[wave][lane] = ss;
                cex[wave][lane] = incl - nfull;
                cbad[wave][lane] = 0;
                asj_wave_sync();
                for (int base = 0; base < total; base += ASJ_WAVE) {
                    const int x = base + lane;
                    if (x < total) {
                        const int i = asj_find_owner(cex[wave], x);
                        const int64_t k0 = (int64_t)(x - cex[wave][i]) * ASJ_CHUNK;
                        uint32_t kr[16], ks[16];
                        asj_load_full(a.rdata, crs[wave][i] + k0, kr);
                        asj_load_full(a.sdata, css[wave][i] + k0, ks);
                        uint32_t diff = 0;
#pragma unroll
                        for (int t = 0; t < 16; t++) diff |= kr[t] ^ ks[t];
                        if (diff) cbad[wave][i] = 1u; // every writer stores the same value
                    }
                }
                // each lane compares its own pair's last, partial chunk
                bool tail_ok = true;
                const int rem = ls - nfull * ASJ_CHUNK;
                if (eq && rem > 0) {
                    const int64_t k0 = (int64_t)nfull * ASJ_CHUNK;
                    uint32_t kr[16], ks[16];
                    asj_load_tail(a.rdata, rs + k0, rem, kr);
                    asj_load_tail(a.sdata, ss + k0, rem, ks);
                    uint32_t diff = 0;
#pragma unroll
                    for (int t = 0; t < 16; t++) diff |= kr[t] ^ ks[t];
                    tail_ok = diff == 0;
                }
                asj_wave_sync();
                ok = eq && tail_ok && cbad[wave][lane] == 0u;
                asj_wave_sync();
            }
            const uint64_t om = __ballot(ok);
            if (om) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd((unsigned long long *)a.out_count, (unsigned long long)__popcll(om));
                base = __shfl(base, 0, ASJ_WAVE);
                if (ok) {
                    const int64_t idx = (int64_t)base + __popcll(om & lanemask_lt);
                    if (idx < a.cap) {
                        asj_pair p;
                        p.r_id = a.rids ? a.rids[r] : (int32_t)r;
                        p.s_id = sid;
                        a.out[idx] = p;
                    }
                }
            }
        }
    }
    if (a.cand_count && lane == 0 && wave_cand)
        atomicAdd((unsigned long long *)a.cand_count, (unsigned long long)wave_cand);
}

template <int PLAIN, int VERIFY>
hipError_t launch(const asj_probe_args *a, int grid_cap, hipStream_t st)
{
    const int64_t nwin = (a->n + ASJ_WAVE - 1) / ASJ_WAVE;
    int64_t blocks = (nwin + kWaves - 1) / kWaves;
    if (blocks > grid_cap) blocks = grid_cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((probe_kernel<PLAIN, VERIFY>), dim3((unsigned)blocks), dim3(kBlock), 0, st, *a);
    return hipGetLastError();
}

} // namespace

hipError_t asj_launch_probe(const asj_probe_args *a, int grid_cap, hipStream_t st)
{
    if (a->plain) return launch<1, 1>(a, grid_cap, st);
    if (a->verify) return launch<0, 1>(a, grid_cap, st);
    return launch<0, 0>(a, grid_cap, st);
}
