/*
 * Reference (oracle) implementation of the signature-accelerated equi-join.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It is deliberately plain, single-threaded and slow:
 * every function follows the paper's definitions step by step so that a
 * reader can check it against the paper by eye.  It shares no code, table
 * or constant generator with the HIP library.
 *
 * Paper: Mokadem, Hameurlain, Morvan, "Equi join query acceleration using
 * algebraic signatures" (IADIS 2008).
 *
 *   Section 3.1   GF(2^f), log/antilog multiplication, the n-symbol
 *                 algebraic signature sig_alpha(P) = (sum_i p_i alpha_j^i)_j.
 *   Section 3.2   Figure 2: sign R, build H_sign, probe with S, output
 *                 tuples whose signatures match, materialize T.
 *   Section 2     the simple hash join (build on R, probe with S, tuples
 *                 whose join attributes match are concatenated into T).
 *
 * Readings where the paper is silent (each one is listed with its reason in
 * the design notes of the repository):
 *   - field polynomials: GF(2^16) uses x^16+x^12+x^3+x+1 (0x1100B), GF(2^8)
 *     uses x^8+x^4+x^3+x^2+1 (0x11D); alpha = x is primitive in both
 *     (or_alpha_order() proves it at run time);
 *   - base: component j (1..n) evaluates at alpha^j;
 *   - symbol i is bytes 2i (low) and 2i+1 (high) for f = 16; an odd tail
 *     byte is zero-extended; for f = 8 symbol i is byte i;
 *   - the sum runs over symbol positions i = 0 .. l-1 (first symbol times
 *     alpha^0);
 *   - component j is stored in bits [(j-1)f, jf) of the packed signature;
 *   - exponents are taken modulo 2^f - 1 for keys longer than the bound
 *     l < 2^f - 1 (the change-detection guarantee lapses there; the join
 *     stays exact because candidates are verified);
 *   - a zero symbol contributes zero (log 0 is undefined).
 *
 * Parity pins: every function below is pinned by the not-gpu tests against
 * something other than itself (closed forms, field axioms, Reed-Solomon
 * codewords, brute force); none of them is "parity unpinned".
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* GF(2^f): elements are f-bit strings, addition is XOR (Section 3.1).       */
/* ------------------------------------------------------------------------ */

static uint32_t field_poly(int f) { return f == 16 ? 0x1100Bu : 0x11Du; }
static uint32_t field_order(int f) { return (1u << f) - 1u; } /* |GF*| */

/* Log/antilog tables (Section 3.1 multiplies with logarithm and antilogarithm tables).
 * exp[e] = alpha^e for 0 <= e < 2^f - 1; log[exp[e]] = e.  log[0] unused. */
static uint16_t exp16[65536], log16[65536];
static uint16_t exp8[256], log8[256];
static int tables_ok = 0;

/* Multiply by alpha = x: shift by one bit, subtract (XOR) the field
 * polynomial when the degree reaches f. */
static uint32_t times_alpha(int f, uint32_t v)
{
    v <<= 1;
    if (v >> f) v ^= field_poly(f);
    return v;
}

static int build_tables(int f, uint16_t *ex, uint16_t *lg)
{
    uint32_t ord = field_order(f);
    uint32_t v = 1;
    memset(lg, 0, sizeof(uint16_t) << f);
    for (uint32_t e = 0; e < ord; e++) {
        if (e > 0 && v == 1) return -1; /* alpha would not be primitive */
        ex[e] = (uint16_t)v;
        lg[v] = (uint16_t)e;
        v = times_alpha(f, v);
    }
    if (v != 1) return -1;
    ex[ord] = 1; /* alpha^(2^f-1) = 1, convenient for wrap-around */
    return 0;
}

int or_init(void)
{
    if (tables_ok) return 0;
    if (build_tables(16, exp16, log16) != 0) return -1;
    if (build_tables(8, exp8, log8) != 0) return -1;
    tables_ok = 1;
    return 0;
}

static const uint16_t *exp_table(int f) { return f == 16 ? exp16 : exp8; }
static const uint16_t *log_table(int f) { return f == 16 ? log16 : log8; }

uint32_t or_gf_exp(int f, uint32_t e) { return exp_table(f)[e % field_order(f)]; }
uint32_t or_gf_log(int f, uint32_t v) { return log_table(f)[v]; }

/* Multiplication through the log/antilog tables (Section 3.1). */
uint32_t or_mul_table(int f, uint32_t a, uint32_t b)
{
    if (a == 0 || b == 0) return 0;
    uint32_t e = ((uint32_t)log_table(f)[a] + log_table(f)[b]) % field_order(f);
    return exp_table(f)[e];
}

/* Multiplication by its textbook definition, independent of the tables:
 * carry-less product of the two polynomials over GF(2), then reduction
 * modulo the field polynomial. */
uint32_t or_mul_clmul(int f, uint32_t a, uint32_t b)
{
    uint64_t r = 0;
    for (int i = 0; i < f; i++)
        if ((b >> i) & 1u) r ^= (uint64_t)a << i;
    for (int d = 2 * f - 2; d >= f; d--)
        if ((r >> d) & 1u) r ^= (uint64_t)field_poly(f) << (d - f);
    return (uint32_t)r;
}

/* Multiplicative order of alpha, by brute force with the clmul multiply;
 * alpha is primitive iff this is 2^f - 1. */
uint32_t or_alpha_order(int f)
{
    uint32_t v = 1, k = 0;
    do {
        v = or_mul_clmul(f, v, 2u);
        k++;
    } while (v != 1u && k <= field_order(f) + 1u);
    return k;
}

/* ------------------------------------------------------------------------ */
/* Algebraic signature (Section 3.1).                                        */
/* ------------------------------------------------------------------------ */

static int64_t num_symbols(int f, int64_t len) { return f == 16 ? (len + 1) / 2 : len; }

/* Symbol p_i of a key of len bytes. */
static uint32_t symbol_at(int f, const uint8_t *b, int64_t len, int64_t i)
{
    if (f == 8) return b[i];
    uint32_t lo = b[2 * i];
    uint32_t hi = (2 * i + 1 < len) ? b[2 * i + 1] : 0u;
    return lo | (hi << 8);
}

/* Formulation 1, the definition term by term with log/antilog tables:
 *   s_j = XOR_{i=0}^{l-1} p_i * alpha^(j*i). */
static uint32_t component_def(int f, int j, const uint8_t *b, int64_t len)
{
    const uint16_t *ex = exp_table(f), *lg = log_table(f);
    uint64_t ord = field_order(f);
    uint32_t s = 0;
    int64_t l = num_symbols(f, len);
    for (int64_t i = 0; i < l; i++) {
        uint32_t p = symbol_at(f, b, len, i);
        if (p == 0) continue; /* zero symbol contributes zero */
        uint64_t e = ((uint64_t)lg[p] + (uint64_t)j * (uint64_t)i) % ord;
        s ^= ex[e];
    }
    return s;
}

/* Formulation 2, Horner's rule using only multiplication by alpha:
 *   s_j = (...((p_{l-1}) a^j + p_{l-2}) a^j + ...) a^j + p_0. */
static uint32_t component_horner(int f, int j, const uint8_t *b, int64_t len)
{
    uint32_t s = 0;
    for (int64_t i = num_symbols(f, len) - 1; i >= 0; i--) {
        for (int t = 0; t < j; t++) s = times_alpha(f, s);
        s ^= symbol_at(f, b, len, i);
    }
    return s;
}

/* Formulation 3, the key read as a polynomial P(y) = sum p_i y^i evaluated
 * at y = alpha^j, with powers and products by the clmul multiply. */
static uint32_t component_poly(int f, int j, const uint8_t *b, int64_t len)
{
    uint32_t beta = 1;
    for (int t = 0; t < j; t++) beta = or_mul_clmul(f, beta, 2u);
    uint32_t pw = 1, s = 0;
    int64_t l = num_symbols(f, len);
    for (int64_t i = 0; i < l; i++) {
        s ^= or_mul_clmul(f, symbol_at(f, b, len, i), pw);
        pw = or_mul_clmul(f, pw, beta);
    }
    return s;
}

/* Packed n-symbol signature of one key: component j in bits [(j-1)f, jf). */
static uint64_t signature_one(int method, int f, int nsym, const uint8_t *b, int64_t len)
{
    uint64_t sig = 0;
    for (int j = 1; j <= nsym; j++) {
        uint32_t c;
        if (method == 1) c = component_horner(f, j, b, len);
        else if (method == 2) c = component_poly(f, j, b, len);
        else c = component_def(f, j, b, len);
        sig |= (uint64_t)c << ((j - 1) * f);
    }
    return sig;
}

/* Signatures of n keys: key k is data[offsets[k] .. offsets[k+1]).
 * method 0 = definition (log/antilog), 1 = Horner, 2 = polynomial/clmul.
 * Returns 0, or -1 on bad parameters. */
int or_signature(int method, int f, int nsym, const uint8_t *data, const int64_t *offsets,
                 int64_t n, uint64_t *out)
{
    if (!tables_ok || (f != 8 && f != 16) || nsym < 1 || f * nsym > 64) return -1;
    for (int64_t k = 0; k < n; k++)
        out[k] = signature_one(method, f, nsym, data + offsets[k], offsets[k + 1] - offsets[k]);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Joins (Section 2, Section 3.2 Figure 2).                                  */
/* Output: (r_id, s_id) pairs as int32 pairs; ids == NULL means row index.   */
/* The full count is returned; pairs past `cap` are not written.             */
/* ------------------------------------------------------------------------ */

typedef struct {
    const uint8_t *data;
    const int64_t *off;
    const int32_t *ids;
    int64_t n;
} rel_t;

static int64_t key_len(const rel_t *r, int64_t k) { return r->off[k + 1] - r->off[k]; }
static const uint8_t *key_ptr(const rel_t *r, int64_t k) { return r->data + r->off[k]; }
static int32_t row_id(const rel_t *r, int64_t k) { return r->ids ? r->ids[k] : (int32_t)k; }

static int keys_equal(const rel_t *R, int64_t a, const rel_t *S, int64_t b)
{
    int64_t la = key_len(R, a);
    if (la != key_len(S, b)) return 0;
    return la == 0 || memcmp(key_ptr(R, a), key_ptr(S, b), (size_t)la) == 0;
}

static void emit(int32_t *pairs, int64_t cap, int64_t *cnt, int32_t r_id, int32_t s_id)
{
    if (*cnt < cap) {
        pairs[2 * *cnt] = r_id;
        pairs[2 * *cnt + 1] = s_id;
    }
    (*cnt)++;
}

/* The join by its definition: every (r, s) with byte-equal keys. */
int64_t or_join_nested(const uint8_t *rd, const int64_t *ro, const int32_t *rid, int64_t m,
                       const uint8_t *sd, const int64_t *so, const int32_t *sid, int64_t n,
                       int32_t *pairs, int64_t cap)
{
    rel_t R = {rd, ro, rid, m}, S = {sd, so, sid, n};
    int64_t cnt = 0;
    for (int64_t b = 0; b < n; b++)
        for (int64_t a = 0; a < m; a++)
            if (keys_equal(&R, a, &S, b)) emit(pairs, cap, &cnt, row_id(&R, a), row_id(&S, b));
    return cnt;
}

/* Chained hash table over m build rows: head[bucket] -> row, next[row] -> row. */
typedef struct {
    int64_t nb;
    int64_t *head;
    int64_t *next;
} chain_t;

static int chain_alloc(chain_t *h, int64_t m)
{
    h->nb = 1;
    while (h->nb < 2 * m) h->nb <<= 1;
    h->head = (int64_t *)malloc(sizeof(int64_t) * (size_t)h->nb);
    h->next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    if (!h->head || !h->next) {
        free(h->head);
        free(h->next);
        return -1;
    }
    for (int64_t i = 0; i < h->nb; i++) h->head[i] = -1;
    return 0;
}

static void chain_free(chain_t *h)
{
    free(h->head);
    free(h->next);
}

/* FNV-1a over the key bytes: the oracle's own plain hash h (Section 2). */
static uint64_t bytes_hash(const uint8_t *p, int64_t len)
{
    uint64_t h = 1469598103934665603ull;
    for (int64_t i = 0; i < len; i++) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

/* Simple hash join (Section 2): build H on R by hashing the join attribute,
 * probe with every S tuple, compare attributes byte by byte. */
int64_t or_join_hash(const uint8_t *rd, const int64_t *ro, const int32_t *rid, int64_t m,
                     const uint8_t *sd, const int64_t *so, const int32_t *sid, int64_t n,
                     int32_t *pairs, int64_t cap)
{
    rel_t R = {rd, ro, rid, m}, S = {sd, so, sid, n};
    chain_t H;
    if (chain_alloc(&H, m) != 0) return -1;
    for (int64_t a = m - 1; a >= 0; a--) { /* build phase */
        int64_t bk = (int64_t)(bytes_hash(key_ptr(&R, a), key_len(&R, a)) & (uint64_t)(H.nb - 1));
        H.next[a] = H.head[bk];
        H.head[bk] = a;
    }
    int64_t cnt = 0;
    for (int64_t b = 0; b < n; b++) { /* probe phase */
        int64_t bk = (int64_t)(bytes_hash(key_ptr(&S, b), key_len(&S, b)) & (uint64_t)(H.nb - 1));
        for (int64_t a = H.head[bk]; a >= 0; a = H.next[a])
            if (keys_equal(&R, a, &S, b)) emit(pairs, cap, &cnt, row_id(&R, a), row_id(&S, b));
    }
    chain_free(&H);
    return cnt;
}

/* Signature hash join (Section 3.2, Figure 2):
 *   for each r in R: compute Sign(r);  Build(R, H_sign);
 *   for each s in S: Probe(H_sign, s): every r whose signature equals
 *   Sign(s) is a candidate; output it.
 * With verify != 0 each candidate is also compared byte by byte, so the
 * output is exactly the equi-join; with verify == 0 the output is the
 * paper's literal one (pairs whose signatures match).
 * *n_cand receives the number of (r, s) pairs with equal signatures. */
int64_t or_join_sig(int f, int nsym, int verify,
                    const uint8_t *rd, const int64_t *ro, const int32_t *rid, int64_t m,
                    const uint8_t *sd, const int64_t *so, const int32_t *sid, int64_t n,
                    int32_t *pairs, int64_t cap, int64_t *n_cand)
{
    rel_t R = {rd, ro, rid, m}, S = {sd, so, sid, n};
    if (!tables_ok || (f != 8 && f != 16) || nsym < 1 || f * nsym > 64) return -1;
    uint64_t *sigR = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
    chain_t H;
    if (!sigR) return -1;
    if (chain_alloc(&H, m) != 0) {
        free(sigR);
        return -1;
    }
    for (int64_t a = 0; a < m; a++) /* pre-calculate Sign(r) */
        sigR[a] = signature_one(0, f, nsym, key_ptr(&R, a), key_len(&R, a));
    for (int64_t a = m - 1; a >= 0; a--) { /* Build(R, H_sign) */
        int64_t bk = (int64_t)(sigR[a] & (uint64_t)(H.nb - 1));
        H.next[a] = H.head[bk];
        H.head[bk] = a;
    }
    int64_t cnt = 0, cand = 0;
    for (int64_t b = 0; b < n; b++) { /* Probe(H_sign, s) */
        uint64_t sg = signature_one(0, f, nsym, key_ptr(&S, b), key_len(&S, b));
        int64_t bk = (int64_t)(sg & (uint64_t)(H.nb - 1));
        for (int64_t a = H.head[bk]; a >= 0; a = H.next[a]) {
            if (sigR[a] != sg) continue;
            cand++;
            if (!verify || keys_equal(&R, a, &S, b))
                emit(pairs, cap, &cnt, row_id(&R, a), row_id(&S, b));
        }
    }
    chain_free(&H);
    free(sigR);
    if (n_cand) *n_cand = cand;
    return cnt;
}
