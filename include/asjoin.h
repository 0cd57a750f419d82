/*
 * libasjoin -- signature-accelerated hash equi-join on one MI355X (gfx950).
 *
 * Computes T = Join(R, S) on the predicate r = s between two relations of
 * variable-length byte-string join attributes, following Mokadem, Hameurlain,
 * Morvan, "Equi join query acceleration using algebraic signatures":
 *
 *   Section 2     R (m tuples) is the smaller relation; a hash table is built
 *                 on R and probed with every tuple of S; matching tuples are
 *                 concatenated into the result T.
 *   Section 3.1   the algebraic signature: GF(2^f) symbols, the n-symbol
 *                 signature sig_alpha(P) = (sum_i p_i alpha^(j i))_{j=1..n},
 *                 4 bytes as two GF(2^16) components.
 *   Section 3.2   Figure 2: sign every r, Build(R, H_sign), sign every s,
 *                 Probe(H_sign, s), output on signature match, Materialize(T).
 *
 * Unlike the paper, every signature match is also verified byte by byte
 * (unless ASJ_NO_VERIFY), so the output is exactly the equi-join.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - All array arguments are DEVICE pointers on the current HIP device unless
 *   stated otherwise.  The caller owns every input and output buffer.
 * - Calls are asynchronous on `stream` (0 = the legacy default stream).  The
 *   return value reports host-side validation and launch errors only;
 *   conditions found on the device are reported through the device counters
 *   described with each call, or through asj_table_status().
 * - Return codes: ASJ_OK (0) or a negative ASJ_E* code; asj_strerror() names
 *   them.  No C++ exception and no abort crosses this interface.
 * - Thread safety: calls on different streams may run concurrently; a table
 *   is read-only after asj_build() and may be probed from several streams.
 */
#ifndef ASJOIN_H
#define ASJOIN_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define ASJ_OK 0
#define ASJ_EINVAL (-1)       /* bad argument (null pointer, negative size, bad parameters) */
#define ASJ_ENOMEM (-2)       /* device allocation failed */
#define ASJ_EOVERFLOW (-3)    /* more result pairs than the caller's capacity (see asj_probe) */
#define ASJ_ETABLEFULL (-4)   /* the hash table had no free slot for a build row */
#define ASJ_EHIP (-5)         /* a HIP runtime call failed */
#define ASJ_EUNSUPPORTED (-6) /* parameter combination not implemented on the GPU */

/* ---- option flags (asj_opts.flags) ---- */
#define ASJ_NO_VERIFY 0x1u /* paper-literal output (Section 3.2, Figure 2): every pair whose
                              signatures are equal, without comparing the key bytes */
#define ASJ_PLAIN 0x2u     /* baseline simple hash join (Section 2): a full-key multiplicative
                              hash instead of the signature; every occupied slot on the probe
                              path is compared by length and bytes (no stored fingerprint) */
#define ASJ_FINGERPRINT 0x200u /* control for the baseline: the same full-key multiplicative hash
                                as ASJ_PLAIN, but stored in the table as a 32-bit fingerprint and
                                compared like a signature before any key byte -- it isolates what
                                the algebraic signature adds over a non-algebraic fingerprint.
                                Single joins (asj_build / asj_probe / asj_join) only; with
                                ASJ_PLAIN or ASJ_NO_VERIFY: ASJ_EINVAL; asj_join_batch,
                                asj_join_host and the server: ASJ_EUNSUPPORTED. */
#define ASJ_PROBE_FUSED 0x4u /* probe schedule: each probe key is signed inside the probe kernel,
                                right before its table walk and verification */
#define ASJ_SORTED 0x10u      /* asj_join / asj_probe: the stored pairs (the first min(|T|, out_cap))
                                are returned sorted by (r_id, s_id) as signed integers, by a device
                                radix sort that reads |T| on the device (no host round trip; device
                                scratch of 16 bytes per out_cap entry, stream-ordered).  Not
                                supported by asj_join_batch (ASJ_EUNSUPPORTED). */
#define ASJ_VALIDATE 0x20u    /* check on the device, before any key byte is read, that every offsets
                                array starts at >= 0 and never decreases (R at build time, S at each
                                probe, both relations for asj_join_batch); on a violation nothing is
                                joined, |T| is reported as -1 (every out_count[j] for a batch) and,
                                for a bad build relation, asj_table_status returns ASJ_EINVAL.
                                (offsets[n] beyond the data buffer cannot be detected.) */
/* Join kind (at most one; none = the inner equi-join of Section 2 / 3.2).
 * The paper names outer joins and the semi-join as future work (Section 5);
 * here they are of the probe relation S with the build relation R, and a
 * probe-only row is reported as the pair (-1, s_id):
 *   ASJ_SEMI        S semi-join R: (-1, s_id) once per probe row with a match
 *   ASJ_ANTI        S anti-join R: (-1, s_id) for each probe row without one
 *   ASJ_LEFT_OUTER  every inner pair plus (-1, s_id) for each unmatched row
 *   ASJ_RIGHT_OUTER every inner pair plus (r_id, -1) for each build row that
 *                   no probe row matches (per asj_probe / asj_join call)
 *   ASJ_LEFT_OUTER | ASJ_RIGHT_OUTER  the full outer join: both
 * (left, right and semi-joins are named as future work in Section 5).
 * |T| counts the pairs written.  A match is key equality, or signature
 * equality under ASJ_NO_VERIFY.  Any other combination: ASJ_EINVAL.  The
 * right and full outer joins are offered by asj_join, asj_probe and
 * asj_join_batch (the server and asj_join_host: ASJ_EUNSUPPORTED); the
 * unmatched build rows are written after every probe row has been
 * processed, so overlapping asj_probe calls on one such table are fine but
 * each call reports the build rows that its own probe rows left unmatched. */
#define ASJ_SEMI 0x40u
#define ASJ_ANTI 0x80u
#define ASJ_LEFT_OUTER 0x100u
#define ASJ_RIGHT_OUTER 0x800u
#define ASJ_PROBE_SPLIT 0x8u /* probe schedule: the probe keys are signed by the signature kernel
                                into a device scratch array first (4 bytes per key), then a probe
                                kernel without signing walks and verifies.  Neither flag means
                                ASJ_PROBE_FUSED; both flags: ASJ_EINVAL.  The output is the
                                same either way. */
#define ASJ_GLOBAL_TABLES 0x400u /* asj_join_batch: every join's table is a segment of one
                                device-memory slot array; asj_join: the table is built in
                                device memory.  Without it, a join with at most 10240 build
                                rows gets no device-memory table: each block that probes it
                                builds the join's table in LDS from the build signatures
                                (same candidates, same output set).  The split schedule, the
                                fingerprint control, 64-bit signatures and asj_build always
                                use device-memory tables. */
#define ASJ_LOCAL_ONLY 0x1000u /* asj_join_batch (and asj_autotune_batch): the caller states that
                                every join has at most 10240 build rows, so every join is probed
                                against an LDS table and the device-memory table build (three
                                launches that would find nothing to build) is skipped.  Checked
                                on the device: a join above the limit fails the call as invalid
                                segments do (every count -1, no key read).  With
                                ASJ_GLOBAL_TABLES or ASJ_PROBE_SPLIT: ASJ_EINVAL (an automatic
                                schedule resolves to the fused one).  Other entry points ignore
                                it. */

/* A relation's join attributes: key k is data[offsets[k] .. offsets[k+1]).
 * offsets must be non-decreasing (k = 0..n).  The library reads only
 * 4-byte-aligned words that hold at least one byte of some key, so `data`
 * needs no padding.  ids[k] is the tuple id written to the output; ids ==
 * NULL means the row index k.  n < 2^31.  All three pointers are device
 * pointers (data may be NULL when every key is empty). */
typedef struct asj_keys {
    const uint8_t *data;
    const int64_t *offsets;
    const int32_t *ids;
    int64_t n;
} asj_keys;

/* One result tuple of T: the ids of the matching build and probe rows. */
typedef struct asj_pair {
    int32_t r_id;
    int32_t s_id;
} asj_pair;

/* Signature parameters (Section 3.1): symbol width f in bits and the number
 * of components n.  Supported: {16, 2} (the paper's 4-byte sig_alpha,2 over
 * GF(2^16), the default), {16, 1}, {8, 4}, {8, 2}, and {16, 4}: an 8-byte
 * signature (every change of up to four symbols detected, Section 3.1).
 * With {16, 4} the table slot holds the low word (components 1 and 2, i.e.
 * the {16, 2} signature) and the table keeps the high word of every build
 * row beside it; a candidate matches both.  {16, 4} is offered by
 * asj_signature, asj_build / asj_probe / asj_join and asj_autotune with the
 * fused probe schedule (ASJ_PROBE_SPLIT: ASJ_EUNSUPPORTED); asj_join_batch,
 * asj_join_host and the server return ASJ_EUNSUPPORTED for it. */
typedef struct asj_sig_params {
    int32_t f;
    int32_t nsym;
} asj_sig_params;

/* Join options.  sig = {0, 0} means {16, 2}; load_factor = table fill
 * bound (capacity = next power of two >= m / load_factor, at least 64);
 * keys_per_window = probe keys a wave takes at a time, 1..64;
 * grid_rounds = size of the probe kernel's grid in units of the blocks the
 * device holds at once, 1..8 (waves then take every grid-th window: one
 * round keeps every block resident for the whole launch, more rounds
 * balance windows of uneven cost).  Options left to the library --
 * load_factor <= 0, keys_per_window <= 0, grid_rounds <= 0, neither
 * ASJ_PROBE_FUSED nor ASJ_PROBE_SPLIT -- take the value asj_autotune (or
 * asj_autotune_batch for asj_join_batch) recorded on this device for the
 * same size class (build rows rounded up to a power of two, same signature
 * parameters and ASJ_PLAIN / ASJ_NO_VERIFY / ASJ_FINGERPRINT flags), else
 * the defaults 0.5, 64, 2 rounds and the fused schedule. */
typedef struct asj_opts {
    asj_sig_params sig;
    float load_factor;
    uint32_t flags;
    int32_t keys_per_window;
    int32_t grid_rounds;
} asj_opts;

/* Opaque build-side hash table H_sign (Section 3.2): an open-addressing
 * multimap of 64-bit slots (signature << 32 | build row), linear probing.
 * It owns its slot array and BORROWS the build relation's data, offsets
 * and ids, which the caller keeps alive and unchanged until asj_table_free. */
typedef struct asj_table asj_table;

/* Algebraic signature of every key (Section 3.1).
 *   keys     the relation (device arrays, see asj_keys)
 *   p        signature parameters; {0,0} means {16,2}
 *   sig_out  device uint32[keys->n] (uint32[2 keys->n] for {16,4}: one
 *            little-endian 64-bit signature per key); component j is stored
 *            in bits [(j-1)f, jf): for {16,2}, sig = s1 | s2 << 16
 * Errors: ASJ_EINVAL (null/negative), ASJ_EUNSUPPORTED (parameters),
 * ASJ_EHIP (launch). */
int asj_signature(const asj_keys *keys, asj_sig_params p, uint32_t *sig_out, hipStream_t stream);

/* Build phase (Section 3.2, Figure 2: pre-calculate Sign(r), Build(R, H_sign)).
 *   r          build relation (borrowed by the table, see asj_table)
 *   opts       may be NULL (defaults)
 *   table_out  receives the new table (host pointer to a handle)
 * The slot array is allocated stream-ordered on `stream`: 8 bytes per slot,
 * 4 per build row for the signatures (8 with 64-bit signatures), and, for
 * the tables of 327680 rows or more that are built region by region, 8 more
 * per row and at most 33 KB of build scratch, all held until
 * asj_table_free.  Whether every row found a slot is known only on the
 * device: asj_table_status() reports it.
 * Errors: ASJ_EINVAL, ASJ_EUNSUPPORTED, ASJ_ENOMEM, ASJ_EHIP. */
int asj_build(const asj_keys *r, const asj_opts *opts, asj_table **table_out, hipStream_t stream);

/* Probe phase (Section 3.2, Figure 2: Probe(H_sign, s) for every s, output
 * the matching tuples, Materialize(T)).
 *   t           table from asj_build (its build stream's work must be
 *               ordered before this call, e.g. the same stream)
 *   s           probe relation
 *   out         device asj_pair[out_cap] (may be NULL when out_cap == 0)
 *   out_cap     capacity of `out` in pairs
 *   out_count   device int64[1]; set to |T|, the full number of result
 *               pairs, even when it exceeds out_cap (pairs past out_cap are
 *               not written; call again with a larger buffer)
 *   cand_count  device int64[1] or NULL; set to the number of (r, s) pairs
 *               whose signatures are equal (the candidates verified), or to
 *               the number of slots compared for ASJ_PLAIN tables
 * The order of the pairs in `out` is unspecified.
 * Errors: ASJ_EINVAL, ASJ_EHIP. */
int asj_probe(const asj_table *t, const asj_keys *s, asj_pair *out, int64_t out_cap, int64_t *out_count,
              int64_t *cand_count, hipStream_t stream);

/* asj_build + asj_probe + asj_table_free in one stream-ordered call (the
 * whole of Figure 2).  Arguments as for those calls.  A full table is
 * reported as |T| = -1 in *out_count. */
int asj_join(const asj_keys *r, const asj_keys *s, const asj_opts *opts, asj_pair *out, int64_t out_cap,
             int64_t *out_count, int64_t *cand_count, hipStream_t stream);

/* ---- a join that allocates nothing ---- */

#define ASJ_NOALLOC_MAX_BUILD_ROWS 10240
#define ASJ_NOALLOC_SCRATCH_BYTES 65536

/* asj_join for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * calls no hipMalloc, hipFree or allocating library routine: the build side's
 * signatures, status words and right-outer marks live in a fixed device
 * array of ASJ_NOALLOC_SCRATCH_BYTES bytes that the library holds on every
 * device it runs on until the process ends (the GF constant tables, too,
 * live in the library's own device array).  Limits: at most
 * ASJ_NOALLOC_MAX_BUILD_ROWS build rows (r->n larger: ASJ_EINVAL), where the
 * table is built in LDS by every probing block exactly as asj_join builds
 * it for such build sides; the fused probe schedule only.
 * Arguments, output and errors are those of asj_join, except that
 * ASJ_SORTED, ASJ_GLOBAL_TABLES and ASJ_PROBE_SPLIT are refused
 * (ASJ_EINVAL) and the fingerprint control and 64-bit signatures are
 * ASJ_EUNSUPPORTED.  Every call on a device shares that device's one scratch
 * array, which each call clears before use: calls that overlap on one device
 * (different streams, or host threads) race and may report wrong results;
 * order them on one stream.  The first call of the process on a device
 * initialises the library there (constant tables, which synchronizes the
 * device): make it outside graph capture. */
int asj_join_noalloc(const asj_keys *r, const asj_keys *s, const asj_opts *opts, asj_pair *out, int64_t out_cap,
                     int64_t *out_count, int64_t *cand_count, hipStream_t stream);

/* ---- many independent joins in one launch sequence ---- */

/* A batch of J independent equi-joins T_j = Join(R_j, S_j) (each one is the
 * join of Section 2 / Figure 2 of Section 3.2).  All build rows of all joins
 * share one key arena and all probe rows another; join j owns build rows
 * r_seg[j] .. r_seg[j+1] of `r` and probe rows s_seg[j] .. s_seg[j+1] of
 * `s`.  Tuple ids come from r.ids / s.ids (typically row-local ids) or are
 * the global row indexes when those are NULL.
 *   r, s        build and probe relations (device, see asj_keys)
 *   r_seg       device int64[njoins + 1], non-decreasing, r_seg[0] = 0,
 *               r_seg[njoins] = r.n
 *   s_seg       device int64[njoins + 1], likewise over s
 *   njoins      J >= 1
 *   out         device asj_pair[]; join j writes out[out_seg[j] .. out_seg[j+1])
 *   out_seg     device int64[njoins + 1], non-decreasing
 *   out_count   device int64[njoins]: |T_j|, the full count even when it
 *               exceeds join j's segment (pairs past it are not written)
 *   cand_count  device int64[njoins] or NULL: signature-equal pairs per join
 *   done_clock  device uint64[njoins + 1] or NULL: done_clock[j] = device
 *               constant-clock time (asj_clock_khz) at which join j's last
 *               probe row was finished, done_clock[njoins] = time at which the
 *               batch started on the device
 *   workspace   device memory of at least asj_batch_workspace_bytes(...)
 *               bytes, or NULL to let the library allocate stream-ordered
 *               (with a workspace the call allocates nothing, so it can be
 *               captured into a HIP graph)
 * A join with more than 10240 build rows (every join with
 * ASJ_GLOBAL_TABLES or the split schedule) gets its own table segment
 * (capacity = next power of two >= |R_j| / load_factor, at least 64); the
 * others are probed against tables built in LDS.  Errors: ASJ_EINVAL, ASJ_ENOMEM,
 * ASJ_EUNSUPPORTED, ASJ_EHIP.  The segment arrays are read on the device
 * only: when they do not cover the relations exactly (r_seg[0] = 0,
 * r_seg[njoins] = r.n, no bound decreasing; likewise s_seg), or a segment
 * table fills up, nothing is joined and every out_count[j] is set to -1. */
typedef struct asj_batch {
    asj_keys r;
    asj_keys s;
    const int64_t *r_seg;
    const int64_t *s_seg;
    int32_t njoins;
    asj_pair *out;
    const int64_t *out_seg;
    int64_t *out_count;
    int64_t *cand_count;
    uint64_t *done_clock;
    void *workspace;
    int64_t workspace_bytes;
} asj_batch;

/* Device workspace needed by asj_join_batch for njoins joins over n_build
 * build rows and n_probe probe rows with these options (NULL = defaults);
 * -1 on bad arguments.  With ASJ_LOCAL_ONLY in the options the table-build
 * scratch (about 8 bytes per build row) is left out, and a workspace of that
 * size serves only calls that pass the flag (others refuse it: ASJ_EINVAL). */
int64_t asj_batch_workspace_bytes(int32_t njoins, int64_t n_build, int64_t n_probe, const asj_opts *opts);

int asj_join_batch(const asj_batch *b, const asj_opts *opts, hipStream_t stream);

/* ---- relations in host memory, beyond the device memory a call may use ---- */

/* Options of asj_join_host.
 *   hbm_budget  device bytes the call may hold at once (0: 80% of the free
 *               device memory).
 *   partitions  0: chosen by the library (1 while the build side and its
 *               table fit half the budget, else the smallest power of two
 *               whose partitions fit); else a power of two 1 .. 1024. */
typedef struct asj_host_opts {
    int64_t hbm_budget;
    int32_t partitions;
    int32_t reserved; /* 0 */
} asj_host_opts;

/* What asj_join_host did (all filled on ASJ_OK). */
typedef struct asj_host_stats {
    int32_t partitions;   /* 1: build side resident, probe side streamed */
    int32_t reserved;
    int64_t chunks;       /* host-to-device chunks in the partitioning pass (0 when partitions = 1) */
    int64_t pieces;       /* probe launches (one per piece of the probe side) */
    int64_t bytes_h2d;    /* bytes copied host -> device */
    int64_t bytes_d2h;    /* bytes copied device -> host */
    int64_t device_peak;  /* most device bytes held at once */
    double ms_partition;  /* host wall time of the partitioning pass */
    double ms_join;       /* host wall time of building and probing */
} asj_host_stats;

/* Join relations held in host memory (pinned memory gives the full host
 * link rate; pageable memory works), for build sides larger than the device
 * memory the call may use: the Grace hash join of Section 2 on one GPU, with
 * the signature as the partitioning hash.
 *   partitions = 1: R is copied to the device whole, signed and built once
 *     (Section 3.2, Figure 2); S streams through in pieces that fit the
 *     budget, each probed as asj_probe does, two pieces in flight.
 *   partitions P > 1: a partitioning pass streams R, then S, through the
 *     device in chunks; each key is signed and moved to partition
 *     mix32(signature) >> (32 - log2 P) (equal keys, and keys of equal
 *     signature, share a partition: Section 2's bucket property), and the
 *     partitioned chunks go back to library-owned pinned host memory with
 *     their signatures.  Then, per partition, R_p is copied in and inserted
 *     from its stored signatures, and the pieces of S_p are probed against
 *     it without signing again.  Host-link traffic: 3|R| + 3|S| bytes of keys
 *     plus 16 bytes per key each way (Section 4.1 counts the same three
 *     passes over each relation for its disk buckets).
 * Arguments:
 *   r, s       relations with HOST pointers (data, offsets, ids as in
 *              asj_keys; ids == NULL means the row index).
 *   opts       join options as for asj_join; ASJ_SORTED: ASJ_EUNSUPPORTED;
 *              the offsets are always checked on the host (ASJ_EINVAL).
 *   hopts      NULL = all defaults.
 *   out        HOST array of out_cap pairs (may be NULL when out_cap = 0);
 *              the first min(|T|, out_cap) pairs, in no particular order.
 *   out_count  HOST int64: |T| (all pairs, also those beyond out_cap).
 *   stats      NULL or filled as above.
 *   stream     device work is ordered after the stream's earlier work;
 *              the call returns when everything is done (it synchronizes).
 * Errors: ASJ_EINVAL (arguments, offsets), ASJ_ENOMEM (the budget cannot
 * hold one key with its buffers, a partition of R too large for the budget
 * even at 1024 partitions -- heavy duplicates -- or one probe row with more
 * pairs than a piece's output buffer), ASJ_ETABLEFULL, ASJ_EHIP. */
int asj_join_host(const asj_keys *r, const asj_keys *s, const asj_opts *opts, const asj_host_opts *hopts,
                  asj_pair *out, int64_t out_cap, int64_t *out_count, asj_host_stats *stats, hipStream_t stream);

/* asj_join_host keeps the pinned host regions of its last partitioned join
 * (about |R| + |S| key bytes plus 16 bytes per key) for the next call; this
 * frees them.  Calls made while another asj_join_host runs use private
 * regions instead.  Returns ASJ_OK. */
int asj_join_host_release(void);

/* ---- autotuning ---- */

/* Outcome of an autotuning run. */
typedef struct asj_tune_result {
    asj_opts best;    /* fastest options found (explicit values and schedule flag) */
    float best_ms;    /* time per call with `best`, over back-to-back calls */
    float default_ms; /* the same with the defaults (0.5, 64, 2 rounds, fused) */
    int32_t trials;   /* configurations timed besides the defaults */
} asj_tune_result;

/* Autotuner for asj_join: times whole joins of r and s (one untimed call,
 * then three back-to-back calls per configuration, HIP events on `stream`) over
 * the load factors {0.25, 0.35, 0.5, 0.7} that give distinct capacities,
 * keys_per_window {4, 8, 16, 32, 64}, both probe schedules and grid_rounds
 * {1, 2, 4}, with the signature parameters and ASJ_PLAIN / ASJ_NO_VERIFY /
 * ASJ_FINGERPRINT flags of `opts` (NULL = defaults; its load factor, keys
 * per window, grid rounds and schedule are ignored); times the four fastest
 * again, each as two blocks of eight back-to-back calls, and records the
 * fastest of those for later calls that leave these options to the library
 * (see asj_opts).  out, out_cap and out_count are the result buffers of the trial
 * joins (as for asj_join); `res` (may be NULL) receives the outcome.
 * Synchronizes the stream.  Errors: those of asj_join, ASJ_EINVAL. */
int asj_autotune(const asj_keys *r, const asj_keys *s, const asj_opts *opts, asj_pair *out, int64_t out_cap,
                 int64_t *out_count, asj_tune_result *res, hipStream_t stream);

/* The same for asj_join_batch over the batch `b` (all four load factors;
 * b's workspace is not used: each trial allocates its own, stream-ordered).
 * b's outputs receive the trial results. */
int asj_autotune_batch(const asj_batch *b, const asj_opts *opts, asj_tune_result *res, hipStream_t stream);

/* Forget every recorded tuning result. */
void asj_autotune_clear(void);

/* Frequency of the device constant clock used by done_clock, in kHz. */
int64_t asj_clock_khz(void);

/* ---- serving: probe requests against a resident build table ---- */

/* A request server over one built table (the probe phase of Section 3.2,
 * Figure 2, applied to a stream of probe relations).  Requests are admitted
 * first-in first-out when the device bytes they need fit in hbm_budget;
 * everything admitted while a stream slot is free is packed into one
 * batched probe launch (continuous batching: requests that arrive while
 * others are on the device join the next launch on the next free slot and
 * overlap with the running ones).  Results are identical to asj_probe on the
 * request alone. */
typedef struct asj_server asj_server;

typedef struct asj_server_opts {
    int32_t slots;              /* concurrent launches (HIP streams); <= 0 means 4 */
    int64_t hbm_budget;         /* device bytes admitted requests may hold; <= 0 means 200 GiB */
    int64_t max_batch_keys;     /* probe keys packed into one launch (a request larger than this
                                   still gets a launch of its own); <= 0 means 256Ki: requests are
                                   bound by their host-to-device copies, so packing large requests
                                   gains no throughput and a request completes only when its whole
                                   launch does */
    int32_t max_batch_requests; /* requests packed into one launch; <= 0 means 256 (1 = no packing) */
    int32_t dry_run;            /* nonzero: no device work; a launch completes after dry_ns_per_key
                                   nanoseconds per probe key (exercises the scheduler without a GPU;
                                   results are then empty) */
    double dry_ns_per_key;
} asj_server_opts;

/* Outcome of one request; times are milliseconds on the server's steady clock. */
typedef struct asj_request_info {
    int32_t status;         /* ASJ_OK or the error that ended the request */
    int64_t count;          /* |T| of the request, even when larger than its out_cap */
    double t_arrive_ms;     /* submission */
    double t_launch_ms;     /* admission into a launch */
    double t_done_ms;       /* results in the caller's buffer */
    int32_t batch_id;       /* launch sequence number */
    int32_t batch_requests; /* requests packed into that launch */
    double t_device_ms;     /* device time of that launch (HIP events): its input copies, kernel
                               and output copies */
    double t_kernel_ms;     /* the launch's probe kernel alone */
} asj_request_info;

typedef struct asj_server_stats_t {
    int64_t queued, busy_slots, budget_used, peak_budget_used, launches;
    double now_ms;
} asj_server_stats_t;

/* t: a built table (its build stream is synchronized here); the server
 * borrows it until asj_server_destroy.  t may be NULL with dry_run. */
int asj_server_create(const asj_table *t, const asj_server_opts *opts, asj_server **out);

/* Queue one request.  HOST pointers: probe key k is data[offsets[k] ..
 * offsets[k+1]) (offsets[0] may be non-zero), results go to out[0 ..
 * out_cap) as (r_id, s_id) with s_id the row index inside the request.
 * The caller keeps data, offsets and out alive and unchanged until
 * asj_server_wait returns for the ticket; pinned memory (hipHostMalloc)
 * lets the copies overlap.  Returns ASJ_ENOMEM at once for a request that
 * needs more than the whole budget, ASJ_EINVAL for offsets that decrease
 * (checked on the host before anything is queued). */
int asj_server_submit(asj_server *s, const uint8_t *data, const int64_t *offsets, int64_t n, asj_pair *out,
                      int64_t out_cap, int64_t *ticket);

/* Blocks until the request has finished; fills info (may be NULL), releases
 * the ticket and returns the request's status.  One waiter per ticket: a
 * second call for a ticket that another thread already waits on, or for a
 * released or unknown ticket, returns ASJ_EINVAL at once.  Waits must not
 * overlap asj_server_destroy. */
int asj_server_wait(asj_server *s, int64_t ticket, asj_request_info *info);

int asj_server_stats(asj_server *s, asj_server_stats_t *stats);

/* Finishes every queued request, then releases the server. */
int asj_server_destroy(asj_server *s);

/* Waits for the table's build work and returns ASJ_OK or ASJ_ETABLEFULL. */
int asj_table_status(const asj_table *t);

/* Number of slots of the table (a power of two), or -1 for NULL. */
int64_t asj_table_capacity(const asj_table *t);

/* Releases the table (stream-ordered on its build stream).  NULL is a no-op. */
int asj_table_free(asj_table *t);

/* Static description of a return code. */
const char *asj_strerror(int code);

/* ---- measurement support (not part of the join) ---- */

/* Per-kernel timing.  While enabled, every kernel phase that this thread
 * launches through the library is bracketed by two HIP events recorded on
 * the call's stream; up to 4096 records accumulate.  asj_timing_read()
 * waits for the last recorded event, fills ms[i] (milliseconds) and
 * names[i] (static phase names) for i < min(cap, count), clears the record
 * and returns the count (or a negative error).  asj_timing_enable() clears
 * the record as well. */
int asj_timing_enable(int on);
int asj_timing_read(float *ms, const char **names, int cap);

/* Plain device-to-device copy of `bytes` bytes with the library's own
 * kernel (used to calibrate hardware byte counters against a known size).
 * dst and src 16-byte aligned. */
int asj_util_copy(void *dst, const void *src, int64_t bytes, hipStream_t stream);

/* Streaming read of `bytes` bytes (16-byte aligned src) with `grid` blocks of
 * 256 threads (<= 0: 2048); XORs a fold of the data into *out_word (device).
 * Measures the achievable read bandwidth that the join kernels are held to. */
int asj_util_read(const void *src, int64_t bytes, uint32_t *out_word, int grid, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* ASJOIN_H */
