/*
 * Byte fillers for the seeded synthetic relations.
 *
 * Shared by the tests, the benchmark and (through them) both the oracle and
 * the HIP library as the source of inputs.  It contains no join or
 * signature arithmetic: only a counter-based random stream and the
 * alphabets of the workloads (printable ASCII, DNA bases, XML-like text).
 *
 * Random stream: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  Each row has its own
 * stream seeded from (seed, stream id, row), so rows can be filled in any
 * order and in parallel with identical results.
 */
#include <stdint.h>
#include <string.h>

static inline uint64_t sm64_next(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline uint64_t row_state(uint64_t seed, uint64_t stream, uint64_t row)
{
    uint64_t s = seed ^ (stream * 0xD1B54A32D192ED03ull);
    uint64_t a = sm64_next(&s);
    s = a ^ (row * 0xABC98388FB8FAC03ull);
    (void)sm64_next(&s);
    return s;
}

/* 16-bit draws from a 64-bit stream. */
typedef struct {
    uint64_t st, buf;
    int left;
} draw16_t;

static inline uint32_t d16(draw16_t *d)
{
    if (d->left == 0) {
        d->buf = sm64_next(&d->st);
        d->left = 4;
    }
    uint32_t v = (uint32_t)(d->buf & 0xFFFFu);
    d->buf >>= 16;
    d->left--;
    return v;
}

/* Exactly uniform integer in [0, k) for 1 <= k <= 65536 (multiply-shift
 * with rejection of the biased low range, after Lemire 2019). */
static inline uint32_t uniform_k(draw16_t *d, uint32_t k)
{
    uint32_t threshold = (65536u - k) % k; /* = 65536 mod k */
    for (;;) {
        uint32_t m = d16(d) * k;
        if ((m & 0xFFFFu) >= threshold) return m >> 16;
    }
}

/* Fill rows[t] (t < nrows) with bytes drawn uniformly from alphabet[0..asize),
 * after copying the first min(prefix_len, len) bytes from prefix. */
void fill_alphabet(uint8_t *data, const int64_t *off, const int64_t *rows, int64_t nrows,
                   uint64_t seed, uint64_t stream, const uint8_t *alphabet, int asize,
                   const uint8_t *prefix, int64_t prefix_len)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t t = 0; t < nrows; t++) {
        int64_t r = rows ? rows[t] : t;
        uint8_t *p = data + off[r];
        int64_t len = off[r + 1] - off[r];
        int64_t i = 0;
        for (; i < len && i < prefix_len; i++) p[i] = prefix[i];
        draw16_t d = {row_state(seed, stream, (uint64_t)r), 0, 0};
        if (asize == 4) { /* two bits per symbol: exactly uniform */
            uint64_t w = 0;
            int bits = 0;
            for (; i < len; i++) {
                if (bits == 0) {
                    w = sm64_next(&d.st);
                    bits = 64;
                }
                p[i] = alphabet[w & 3u];
                w >>= 2;
                bits -= 2;
            }
        } else {
            for (; i < len; i++) p[i] = alphabet[uniform_k(&d, (uint32_t)asize)];
        }
    }
}

/* XML-like text: seeded random nesting of <name> ... </name> tags taken
 * from a vocabulary (names[k] = vocab[voff[k] .. voff[k+1])), with runs of
 * printable content that contain no '<' or '>', cut to the row length. */
void fill_xml(uint8_t *data, const int64_t *off, const int64_t *rows, int64_t nrows,
              uint64_t seed, uint64_t stream, const uint8_t *vocab, const int64_t *voff, int nnames)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t t = 0; t < nrows; t++) {
        int64_t r = rows ? rows[t] : t;
        uint8_t *p = data + off[r];
        int64_t len = off[r + 1] - off[r];
        draw16_t d = {row_state(seed, stream, (uint64_t)r), 0, 0};
        int stack[8];
        int depth = 0;
        int64_t i = 0;
#define PUT(c)                     \
    do {                           \
        if (i < len) p[i++] = (c); \
    } while (0)
        while (i < len) {
            uint32_t act = uniform_k(&d, 100);
            if (depth < 8 && act < 35) { /* open a tag */
                int k = (int)uniform_k(&d, (uint32_t)nnames);
                stack[depth++] = k;
                PUT('<');
                for (int64_t c = voff[k]; c < voff[k + 1]; c++) PUT(vocab[c]);
                PUT('>');
            } else if (depth > 0 && act < 65) { /* close the innermost tag */
                int k = stack[--depth];
                PUT('<');
                PUT('/');
                for (int64_t c = voff[k]; c < voff[k + 1]; c++) PUT(vocab[c]);
                PUT('>');
            } else { /* content run of 1..12 printable characters except < > */
                uint32_t run = 1 + uniform_k(&d, 12);
                for (uint32_t c = 0; c < run; c++) {
                    uint32_t v = 0x20 + uniform_k(&d, 93); /* 95 printable minus 2 */
                    if (v >= '<') v++;                    /* skip '<' (0x3C) */
                    if (v >= '>') v++;                    /* skip '>' (0x3E) */
                    PUT((uint8_t)v);
                }
            }
        }
#undef PUT
    }
}

/* dst row dst_rows[t] <- src row src_rows[t]; lengths must already agree. */
void copy_rows(uint8_t *dst, const int64_t *doff, const int64_t *dst_rows,
               const uint8_t *src, const int64_t *soff, const int64_t *src_rows, int64_t k)
{
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t t = 0; t < k; t++) {
        int64_t a = dst_rows[t], b = src_rows[t];
        memcpy(dst + doff[a], src + soff[b], (size_t)(soff[b + 1] - soff[b]));
    }
}
