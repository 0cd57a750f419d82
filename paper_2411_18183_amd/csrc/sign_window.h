// Per-window signing shared by the signature kernel and the fused probe
// kernel (included by sign.hip and probe.hip).
//
// Work decomposition.  A key of len bytes is read as floor(len / 64) full
// key-relative chunks of 64 bytes plus, when len % 64 != 0, one tail chunk.
// A wave takes a window of 64 consecutive keys.  It lays the full chunks of
// all 64 keys out back to back and processes them in passes of 64, one
// chunk per lane, so short and long keys (16 B .. 10 KB and beyond) keep
// every lane busy with identical, unpredicated code; a last pass gives lane
// i the tail chunk of key i.  A lane reads its chunk with 16-byte loads,
// realigns it to key-relative words, folds it into a partial signature,
// scales the partial to the chunk's position in the key and XORs it (GF
// addition) into the key's accumulator in LDS.
//
// Chunk arithmetic (GF(2^16), components j = 1 .. 4).  Component j of a chunk
// is sum_u p_u alpha^(j u) over its 32 symbols.  Instead of one log/antilog
// multiplication per symbol, the lane runs Horner's rule over groups of
// symbols with an unreduced accumulator: shifting by one bit is
// multiplication by alpha = x, so a group (16 symbols for j = 1, 8 for
// j = 2) costs shifts and XORs only, and the 16 bits that overflow are
// folded back with two byte-indexed table lookups (T[b] = b x^16).  Scaling
// a chunk to its position multiplies by alpha^(32 j c) for chunk index c,
// digit by digit with constant tables (c = d0 + 8 d1 + 64 blk).
// With four components (a 64-bit signature) the low word is the two-
// component signature and the high word holds components 3 and 4, whose
// groups are 4 symbols (x^12, x^16 per Horner step); their position factors
// alpha^(96c) and alpha^(128c) are products of the component 1 and 2 tables,
// so no further tables are needed.
#pragma once

#include "asj_internal.h"

namespace asj {

// (low half of w) << S and (high half of w) << S in one instruction each
// (sub-dword operand select, S an inline constant); VALU only.
template <int S>
__device__ __forceinline__ uint32_t shl_lo16(uint32_t w)
{
    uint32_t r;
    asm("v_lshlrev_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_0"
        : "=v"(r) : "n"(S), "v"(w));
    return r;
}
template <int S>
__device__ __forceinline__ uint32_t shl_hi16(uint32_t w)
{
    uint32_t r;
    asm("v_lshlrev_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_1"
        : "=v"(r) : "n"(S), "v"(w));
    return r;
}
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// XOR over words t = 0..T of (low symbol << STEP t) and (high symbol <<
// STEP t + OFF): one Horner group with an unreduced accumulator.
template <int T, int STEP, int OFF>
__device__ __forceinline__ uint32_t fold_group(const uint32_t *w)
{
    if constexpr (T < 0) {
        return 0u;
    } else {
        const uint32_t u = fold_group<T - 1, STEP, OFF>(w);
        return xor3(u, shl_lo16<STEP * T>(w[T]), shl_hi16<STEP * T + OFF>(w[T]));
    }
}

// Multiplication by alpha^(2048 J blk) for a chunk's 64-chunk block index
// blk > 2 (keys longer than 12 KB): one device-memory pair per non-zero
// octal digit of blk (at most seven), so that a chunk's cost does not grow
// with its position in a long key.  Blocks 1 and 2 take the LDS pair once
// or twice instead (the callers' loop).
template <int J>
__device__ __forceinline__ uint32_t scale_blk16_far(uint32_t v, const uint16_t *__restrict__ gtab, int blk)
{
    for (int k = 0; blk > 0; k++, blk >>= 3) {
        const int d = blk & 7;
        if (d) v = asj_cmul16(v, gtab + ASJ_TAB_HI_BASE + asj_tab_hi(J, k, d) * ASJ_TAB_WORDS);
    }
    return v;
}

// GF(2^16): components 1 and 2 of one 64-byte chunk, positions relative to
// the chunk start; returns s1 | s2 << 16 (s2 = 0 when nsym == 1).
template <int NSYM>
__device__ __forceinline__ uint32_t chunk_sig16(const uint32_t kd[16], const uint16_t *__restrict__ tab,
                                                const uint16_t *__restrict__ gtab, int c)
{
    const uint16_t *red = tab + ASJ_TAB_RED * ASJ_TAB_WORDS;
    uint32_t a1 = 0, a2 = 0;
    // component 1: two groups of 16 symbols; p_v (v = 0..15 in the group)
    // shifted by v stays below 2^31, plus the accumulator times x^16
#pragma unroll
    for (int g = 1; g >= 0; g--) {
        const uint32_t u = fold_group<7, 2, 1>(kd + 8 * g);
        const uint32_t t1 = (a1 << 16) ^ u;
        a1 = (t1 & 0xFFFFu) ^ asj_cmul16(t1 >> 16, red);
    }
    if (NSYM >= 2) {
        // component 2: four groups of 8 symbols; p_v shifted by 2v stays below 2^30
#pragma unroll
        for (int q = 3; q >= 0; q--) {
            const uint32_t u = fold_group<3, 4, 2>(kd + 4 * q);
            const uint32_t t2 = (a2 << 16) ^ u;
            a2 = (t2 & 0xFFFFu) ^ asj_cmul16(t2 >> 16, red);
        }
    }
    // position of the chunk in the key: multiply by alpha^(32 j c)
    const int d0 = c & 7, d1 = (c >> 3) & 7;
    a1 = asj_cmul16(a1, tab + asj_tab_d0(1, d0) * ASJ_TAB_WORDS);
    a1 = asj_cmul16(a1, tab + asj_tab_d1(1, d1) * ASJ_TAB_WORDS);
    if (NSYM >= 2) {
        a2 = asj_cmul16(a2, tab + asj_tab_d0(2, d0) * ASJ_TAB_WORDS);
        a2 = asj_cmul16(a2, tab + asj_tab_d1(2, d1) * ASJ_TAB_WORDS);
    }
    int blk = c >> 6;
    if (blk > 2) {
        a1 = scale_blk16_far<1>(a1, gtab, blk);
        if (NSYM >= 2) a2 = scale_blk16_far<2>(a2, gtab, blk);
        blk = 0;
    }
    for (; blk > 0; blk--) {
        a1 = asj_cmul16(a1, tab + asj_tab_blk(1) * ASJ_TAB_WORDS);
        if (NSYM >= 2) a2 = asj_cmul16(a2, tab + asj_tab_blk(2) * ASJ_TAB_WORDS);
    }
    return a1 | (a2 << 16);
}

// Multiplication by alpha^(32 j c) for j = 1, 2 (the position factors of
// components 1 and 2); components 3 and 4 apply them in combination.
template <int J>
__device__ __forceinline__ uint32_t scale16(uint32_t v, const uint16_t *__restrict__ tab,
                                            const uint16_t *__restrict__ gtab, int c)
{
    v = asj_cmul16(v, tab + asj_tab_d0(J, c & 7) * ASJ_TAB_WORDS);
    v = asj_cmul16(v, tab + asj_tab_d1(J, (c >> 3) & 7) * ASJ_TAB_WORDS);
    int blk = c >> 6;
    if (blk > 2) {
        v = scale_blk16_far<J>(v, gtab, blk);
        blk = 0;
    }
    for (; blk > 0; blk--) v = asj_cmul16(v, tab + asj_tab_blk(J) * ASJ_TAB_WORDS);
    return v;
}

// GF(2^16): components 3 and 4 of one 64-byte chunk; returns s3 | s4 << 16.
__device__ __forceinline__ uint32_t chunk_sig16_hi(const uint32_t kd[16], const uint16_t *__restrict__ tab,
                                                   const uint16_t *__restrict__ gtab, int c)
{
    const uint16_t *red = tab + ASJ_TAB_RED * ASJ_TAB_WORDS;
    uint32_t a3 = 0, a4 = 0;
    // eight groups of 4 symbols (2 words): p_v shifted by 3v (below 2^25)
    // plus the accumulator times x^12, and p_v shifted by 4v (below 2^28)
    // plus the accumulator times x^16
#pragma unroll
    for (int q = 7; q >= 0; q--) {
        const uint32_t t3 = (a3 << 12) ^ fold_group<1, 6, 3>(kd + 2 * q);
        a3 = (t3 & 0xFFFFu) ^ asj_cmul16(t3 >> 16, red);
        const uint32_t t4 = (a4 << 16) ^ fold_group<1, 8, 4>(kd + 2 * q);
        a4 = (t4 & 0xFFFFu) ^ asj_cmul16(t4 >> 16, red);
    }
    // positions: alpha^(96c) = alpha^(32c) alpha^(64c), alpha^(128c) = (alpha^(64c))^2
    a3 = scale16<2>(scale16<1>(a3, tab, gtab, c), tab, gtab, c);
    a4 = scale16<2>(scale16<2>(a4, tab, gtab, c), tab, gtab, c);
    return a3 | (a4 << 16);
}

// GF(2^8): byte symbols, NSYM components of 8 bits; component j of the chunk
// is sum_u b_u alpha^(j u), u = 0..63, then scaled by alpha^(64 j c).
template <int NSYM>
__device__ __forceinline__ uint32_t chunk_sig8(const uint32_t kd[16], const uint16_t *__restrict__ t8, int c)
{
    const uint16_t *ex = t8 + ASJ_TAB8_EXP, *lg = t8 + ASJ_TAB8_LOG, *red = t8 + ASJ_TAB8_RED;
    uint32_t acc[NSYM];
#pragma unroll
    for (int j = 0; j < NSYM; j++) acc[j] = 0;
#pragma unroll
    for (int t = 15; t >= 0; t--) {
        const uint32_t w = kd[t];
        const uint32_t b0 = w & 255u, b1 = (w >> 8) & 255u, b2 = (w >> 16) & 255u, b3 = w >> 24;
#pragma unroll
        for (int j = 1; j <= NSYM; j++) {
            // four symbols per word: Horner step by alpha^(4j), unreduced
            const uint32_t u = b0 ^ (b1 << j) ^ (b2 << (2 * j)) ^ (b3 << (3 * j));
            const uint32_t T = (acc[j - 1] << (4 * j)) ^ u; // < 2^(8 + 4j) <= 2^24
            uint32_t v = (T & 255u) ^ red[(T >> 8) & 255u];
            if (j > 2) v ^= red[256 + ((T >> 16) & 255u)];
            acc[j - 1] = v;
        }
    }
    uint32_t out = 0;
#pragma unroll
    for (int j = 1; j <= NSYM; j++) {
        uint32_t v = acc[j - 1];
        if (v) v = ex[(lg[v] + (uint32_t)((64ull * j * (uint64_t)c) % 255u)) % 255u];
        out |= v << (8 * (j - 1));
    }
    return out;
}

// Plain multiplicative hash of one chunk, seeded by its index (baseline).
__device__ __forceinline__ uint32_t chunk_plain(const uint32_t kd[16], int c)
{
    uint32_t h = 0x9E3779B9u * (uint32_t)(c + 1);
#pragma unroll
    for (int t = 0; t < 16; t++) {
        h = (h ^ kd[t]) * 0x85EBCA77u;
        h ^= h >> 15;
    }
    return h;
}

template <int MODE, int NSYM>
__device__ __forceinline__ uint32_t chunk_value(const uint32_t kd[16], const uint16_t *tab,
                                                const uint16_t *__restrict__ gtab, int c)
{
    if (MODE == ASJ_MODE_SIG16) return chunk_sig16<NSYM>(kd, tab, gtab, c);
    if (MODE == ASJ_MODE_SIG8) return chunk_sig8<NSYM>(kd, tab, c);
    return chunk_plain(kd, c);
}

// Words of the constant tables a block keeps in LDS for each mode.
template <int MODE>
struct TabWords {
    static constexpr int value = MODE == ASJ_MODE_SIG16 ? ASJ_NTAB16 * ASJ_TAB_WORDS
                                 : MODE == ASJ_MODE_SIG8 ? ASJ_NTAB8 * ASJ_TAB_WORDS
                                                         : 2;
};

// Copy the mode's constant tables from device memory into LDS (whole block).
template <int MODE, int BLOCK>
__device__ __forceinline__ void load_tables(uint16_t *tab, const uint16_t *__restrict__ gtab)
{
    if (MODE == ASJ_MODE_PLAIN) return;
    constexpr int words = TabWords<MODE>::value;
    const uint16_t *src = gtab + (MODE == ASJ_MODE_SIG8 ? ASJ_TAB8_BASE : 0);
    for (int i = threadIdx.x; i < words / 2; i += BLOCK)
        reinterpret_cast<uint32_t *>(tab)[i] = reinterpret_cast<const uint32_t *>(src)[i];
    __syncthreads();
}

// Signature (or finalized plain hash) of each lane's key for a window of up
// to 64 keys, one per lane: key bytes data[s, s + len) (len = 0 for lanes
// without a key); end = where the relation's key bytes end (offsets[n]).
// wown is the wave's 64-entry LDS scratch for the pass owners.
// wst/wex/wacc are the wave's 64-entry LDS scratch arrays; with four
// GF(2^16) components wacc2 (64 entries) accumulates the high word,
// returned in hi.  tab: the mode's constant tables in LDS; gtab: all of
// them in device memory (the pairs for chunks beyond the 192nd of a key).
template <int MODE, int NSYM>
__device__ __forceinline__ uint32_t sign_window(const uint8_t *__restrict__ data, int64_t s, int len, int64_t end,
                                                int64_t *wst, int32_t *wex, uint32_t *wacc, int32_t *wown,
                                                const uint16_t *tab, const uint16_t *__restrict__ gtab,
                                                uint32_t *wacc2, uint32_t &hi)
{
    constexpr bool kHi = MODE == ASJ_MODE_SIG16 && NSYM == 4;
    const int lane = threadIdx.x % ASJ_WAVE;
    const int nfull = len / ASJ_CHUNK;
    const int incl = asj_wave_incl_scan(nfull);
    const int total = __shfl(incl, ASJ_WAVE - 1, ASJ_WAVE);
    wst[lane] = s;
    wex[lane] = incl - nfull;
    wacc[lane] = 0;
    if (kHi) wacc2[lane] = 0;
    asj_wave_sync();
    // full chunks of all 64 keys, 64 per pass, one per lane: uniform code
    int carry = -1;
    for (int base = 0; base < total; base += ASJ_WAVE) {
        const int x = base + lane;
        const int i = asj_pass_owner(incl - nfull, nfull, base, wown, carry);
        if (x < total) {
            const int c = x - wex[i];
            uint32_t kd[16];
            asj_load_full(data, wst[i] + (int64_t)c * ASJ_CHUNK, kd);
            atomicXor(&wacc[i], chunk_value<MODE, NSYM>(kd, tab, gtab, c));
            if (kHi) atomicXor(&wacc2[i], chunk_sig16_hi(kd, tab, gtab, c));
        }
    }
    // tail pass: lane i takes key i's last, partial chunk
    uint32_t v = 0, vh = 0;
    const int rem = len - nfull * ASJ_CHUNK;
    if (rem > 0) {
        uint32_t kd[16];
        asj_load_tail_fast(data, s + (int64_t)nfull * ASJ_CHUNK, rem, end, kd);
        v = chunk_value<MODE, NSYM>(kd, tab, gtab, nfull);
        if (kHi) vh = chunk_sig16_hi(kd, tab, gtab, nfull);
    }
    asj_wave_sync();
    v ^= wacc[lane];
    if (kHi) hi = vh ^ wacc2[lane];
    asj_wave_sync();
    if (MODE == ASJ_MODE_PLAIN) v = asj_mix32(v ^ ((uint32_t)len * 0xC2B2AE3Du));
    return v;
}

} // namespace asj
