/*
 * wvprime.h -- C ABI of libwvprime.so: B_{p-3} mod p and E_{p-3} mod p for
 * primes p on an AMD MI355X (gfx950).
 *
 * Method (Booker, Hathi, Mossinghoff, Trudgian, "Wolstenholme and Vandiver
 * primes", arXiv:2101.11157):
 *   - A prime p >= 5 is a Wolstenholme prime iff p divides the numerator of
 *     B_{p-3} (Section 1, eqnGlaisher and the sentence after it) and a
 *     Vandiver prime iff p divides E_{p-3} (Section 1; Euler numbers from the
 *     EGF sec z).
 *   - Each residue is a linear combination of sums
 *         S(x, y) = sum_{x p < s < y p} s^-3   (Bernoulli side, Section 3)
 *         S(x, y) = sum_{x p < s < y p} s^-2   (Euler side, Section 5)
 *     given by one of the paper's specialised congruences (eqnBB1 ... eqnBB30,
 *     eqnEE3 ... eqnEE33), with each sum computed as c1/c0 of
 *     prod (z + s^3) or prod (z + s^2) (Section 3, eqnComputeS) and partial
 *     products joined by eqnCombinePairs.
 *
 * Every call returns an int status: WV_OK (0) or a negative error code.  No
 * C++ exception crosses this interface.  Calls on one context are not
 * thread-safe: use one context per host thread, or serialise.
 */
#ifndef WVPRIME_H
#define WVPRIME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define WV_OK         0
#define WV_EINVAL    -1  /* NULL pointer where one is required, lo > hi, bad id  */
#define WV_EDOMAIN   -2  /* p < 5 or p >= WV_P_MAX                              */
#define WV_ENOTPRIME -3  /* a non-prime in wv_eval_primes                       */
#define WV_ETRUNC    -4  /* caller's buffer too small; *n_out holds the need    */
#define WV_ENOMEM    -5  /* device allocation failed (context stays valid)      */
#define WV_EHIP      -6  /* a HIP runtime call failed (context stays valid)     */
#define WV_EBUSY     -7  /* a served request has not finished yet               */

/* Largest supported prime bound (exclusive): 2^40.  The long sums run in exact
 * double-precision modular arithmetic (residues held as integer-valued doubles,
 * products below 2^51 p) and the short ones, the reductions and the final
 * combination in 64-bit Montgomery arithmetic; the bounds of both assume
 * p < 2^40. */
#define WV_P_MAX (1ULL << 40)

/* Result flags. */
#define WV_FLAG_WOLSTENHOLME 1u  /* b == 0: p | B_{p-3} */
#define WV_FLAG_VANDIVER     2u  /* e == 0: p | E_{p-3} */

/* One prime's residues.  b = B_{p-3} mod p and e = E_{p-3} mod p (Euler numbers
 * in the secant convention), both canonical in [0, p).  The paper reports the
 * symmetric representative in (-p/2, p/2] (Section 3, notation before Table 2);
 * wv_symmetric() converts. */
typedef struct {
    uint64_t p;
    uint64_t b;
    uint64_t e;
    uint32_t flags;
    uint32_t reserved;
} wv_result;

static inline int64_t wv_symmetric(uint64_t r, uint64_t p) {
    return r > (p - 1) / 2 ? (int64_t)r - (int64_t)p : (int64_t)r;
}

/* Congruence identifiers.  Bernoulli side (Section 3): eqnBB1, eqnBB2, eqnBB6,
 * eqnBB9, eqnBB16, eqnBB22, eqnBB30.  Euler side (Section 5): eqnEE3, eqnEE5,
 * eqnEE9, eqnEE16, eqnEE24, eqnEE33.  Root forms used for p = 5 and 7, where the
 * specialised tables' left sides vanish: eqnV12 (Section 2, at k=(p-3)/2 its
 * left side is 5 B_{p-3}) and eqnE1 (Section 4, at k=1 its left side is
 * -4 E_{p-3}, sign read as (-1)^k). */
enum {
    WV_TABLE_BB1 = 0, WV_TABLE_BB2, WV_TABLE_BB6, WV_TABLE_BB9, WV_TABLE_BB16,
    WV_TABLE_BB22, WV_TABLE_BB30,
    WV_TABLE_EE3, WV_TABLE_EE5, WV_TABLE_EE9, WV_TABLE_EE16, WV_TABLE_EE24,
    WV_TABLE_EE33,
    WV_TABLE_V12, WV_TABLE_E1,
    WV_TABLE_COUNT
};

/* Opaque context: owns device buffers, one HIP stream, events and the
 * tuning cache.  Device memory grows on demand and is freed by wv_destroy. */
typedef struct wv_ctx wv_ctx;

/* Timings (milliseconds, HIP events on the context stream) and sizes of the
 * most recent wv_search_range / wv_eval_primes call. */
typedef struct {
    double ms_total;     /* first to last event of the call (device time)        */
    double ms_sieve;     /* segmented sieve and prime compaction (search only)   */
    double ms_plan;      /* per-prime plan: endpoints, coefficients, chunk scan  */
    double ms_sum;       /* term-sum kernel (the hot loop)                      */
    double ms_reduce;    /* per-sum reduction of chunk pairs                    */
    double ms_finalize;  /* per-prime combination, inverse, flags               */
    uint64_t n_primes;
    uint64_t n_sums;     /* (prime, sum) pairs                                  */
    uint64_t n_chunks;
    uint64_t n_terms;    /* total number of s values summed (both residues)     */
    uint64_t n_terms_b;  /* of which Bernoulli-side terms                       */
    uint64_t chunk_terms;/* terms per chunk used                                */
    uint32_t block_k_b;  /* terms per block in the hot loop, Bernoulli side    */
    uint32_t block_k_e;  /* terms per block in the hot loop, Euler side        */
    uint32_t grid;       /* workgroups of the term-sum launch                   */
    uint32_t reserved;
} wv_stats;

/* Create a context on HIP device `hip_device`.  *out receives the handle.
 * Errors: WV_EINVAL (out NULL or bad device), WV_EHIP, WV_ENOMEM. */
int wv_create(int hip_device, wv_ctx **out);

/* Release every resource of ctx (NULL is accepted). */
int wv_destroy(wv_ctx *ctx);

/* Choose the congruences used for primes p >= 11: b_table one of the BB ids
 * or a Bernoulli table defined with wv_define_table, e_table one of the EE ids
 * or a defined Euler table.  Default: WV_TABLE_BB30 and WV_TABLE_EE33 (the
 * cheapest printed ones, cost 227p/6480 and 27p/512).  Every valid choice gives
 * identical residues; only the work changes.  Errors: WV_EINVAL. */
int wv_set_tables(wv_ctx *ctx, int b_table, int e_table);

/* Define a congruence at run time (for instance one derived from eqnVandiver
 * or eqnEMac2 with the transformations of Proposition propTW, Section 2):
 *     lhs * X_{p-3} == sum_{i<n} coef[i] * S(xa[i]/xb[i], ya[i]/yb[i])  (mod p),
 * S(x, y) = sum_{x p < s < y p} s^-deg, deg 3 for X = B, 2 for X = E.
 * Integers are decimal strings of any length (optional leading '-'; lhs
 * nonzero); endpoints 0 <= x < y <= 1 with denominators below 2^63; n <= 65536.
 * The table serves the primes p >= min_p (min_p >= 11, above every prime the
 * derivation must avoid, such as subdivision factors) that do not divide lhs;
 * every other prime of a batch uses eqnBB30 / eqnEE33.  The congruence itself
 * is trusted, not checked.  *id
 * receives the id for wv_set_tables (at most 64 tables per context).
 * Errors: WV_EINVAL (malformed input), WV_ENOMEM, WV_EHIP. */
int wv_define_table(wv_ctx *ctx, int deg, const char *lhs, size_t n, const char *const *coef,
                    const uint64_t *xa, const uint64_t *xb, const uint64_t *ya, const uint64_t *yb,
                    uint64_t min_p, int *id);

/* Name the table that serves the primes a defined table `id` does not (those
 * below its min_p, or dividing its left side): `below` is a compiled table of
 * the same degree (not a root form) or a defined one with a smaller min_p, so
 * that every chain ends at a compiled table.  The default is eqnBB30 /
 * eqnEE33.  A chain of congruences from one greedy search (Section 2.2: more
 * rounds give more, shorter sums of fewer terms in total) lets each prime use
 * the one whose work, terms plus a fixed cost per sum, is least at its size;
 * the residues do not depend on the choice.  A batch allows for the most sums
 * per prime of any table on the chain.  Errors: WV_EINVAL (an id out of
 * range, a compiled `id`, another degree, a root form, or a defined `below`
 * whose min_p is not smaller), WV_EHIP. */
int wv_set_table_below(wv_ctx *ctx, int id, int below);

/* Set the number of terms each lane sums per chunk (0 = automatic: about
 * sqrt(2 * 4096 * T / lanes) for a batch of T terms, between 2^12 and 2^22,
 * which balances the set-up of each chunk against lanes idling when the last
 * chunks finish).  Each sum is cut into chunks of exactly this many terms plus
 * one shorter tail; the tails of all sums run after the full chunks, longest
 * first.  Must be a multiple of 64 when nonzero.  Results do not depend on it. */
int wv_set_chunk_terms(wv_ctx *ctx, uint64_t chunk_terms);

/* Choose the block shape of the term-sum kernel: kb terms per block on the
 * Bernoulli side and ke on the Euler side (compiled shapes: 1/1, 4/4, 8/8,
 * 12/16, 16/24, 20/28, 24/32, 26/34, 28/32, 28/36; default 28/36).  Each block
 * of k consecutive s is folded into the running pair as one factor of
 * eqnCombinePairs, whose two members come from the Taylor coefficients of
 * prod_j (x + j) stepped by finite differences.  Results do not depend on the
 * shape.
 * kb = ke = 0 returns to the default / autotuned choice.
 * Errors: WV_EINVAL for a shape that is not compiled. */
int wv_set_block(wv_ctx *ctx, int kb, int ke);

/* Progress of a long synchronous call: with a callback set, the term sums of
 * each batch run as consecutive launches of about terms_per_launch terms (0:
 * 2^44) and fn(user, done, total) is called on the calling thread after each
 * (done/total in chunks of the current batch).  NULL fn: one launch per batch.
 * Results do not depend on the split. */
typedef void (*wv_progress_fn)(void *user, uint64_t done, uint64_t total);
int wv_set_progress(wv_ctx *ctx, wv_progress_fn fn, void *user, uint64_t terms_per_launch);

/* Autotuner: times every compiled block shape with chunk sizes 2^16, 2^18 and
 * automatic (reported as 0) on sample primes just above p_hint (n_sample of them, 0: 16) and
 * keeps the fastest for primes in [2^k, 2^(k+1)), k = floor(log2 p_hint).
 * Synchronous calls on primes in a tuned range then use the tuned shape and
 * chunk unless wv_set_block / wv_set_chunk_terms force others.  The measured
 * rates go to rates[v*3 + j] (terms/s) when rates is non-NULL (room for
 * 3 x the number of compiled shapes).  Returns the chosen shape and chunk. */
int wv_autotune(wv_ctx *ctx, uint64_t p_hint, int n_sample, int *kb, int *ke, uint64_t *chunk_terms,
                double *rates);

/* Write / read the tuning cache (text lines: arch log2p kb ke chunk rate). */
int wv_tune_save(const wv_ctx *ctx, const char *path);
int wv_tune_load(wv_ctx *ctx, const char *path);

/* Number of primes p with 5 <= p and lo <= p < hi (segmented sieve on the
 * device).  The paper's searches run over the primes from 5 upwards (Section 3,
 * Results: 4,118,054,811 primes in [5, 1e11)); which sieve enumerates them is
 * not part of the method (the paper uses an external one).  Synchronous.
 * Errors: WV_EINVAL (n NULL, lo > hi), WV_EDOMAIN (hi > WV_P_MAX). */
int wv_count_primes(wv_ctx *ctx, uint64_t lo, uint64_t hi, uint64_t *n);

/* The search of Sections 3 and 5 over one interval (Theorem 1.1 reports its
 * hits below 1e11): for every prime p with max(lo,5) <= p < hi, B_{p-3} mod p
 * and E_{p-3} mod p from the configured congruences (Section 3: eqnBB1 ...
 * eqnBB30; Section 5: eqnEE3 ... eqnEE33; or defined ones), each sum
 * S(x, y) of eqnDefnS evaluated as c1/c0 by eqnComputeS and eqnCombinePairs,
 * and the flags of a Wolstenholme (b = 0) or Vandiver (e = 0) prime.
 * Sieve, then residues; a small interval (at most 64 sieve segments, an upper
 * bound on its prime count no larger than cap, little work) runs as one
 * replayed HIP graph sized by that bound, with the count taken on the device.
 * out[0..n) receives the results in ascending p, where n = *n_out; if cap < n
 * the call
 * writes nothing, sets *n_out = n and returns WV_ETRUNC.  hits (may be NULL
 * when hit_cap == 0) receives up to hit_cap primes whose flags are nonzero,
 * ascending; *n_hits (may be NULL) receives their total number.  All buffers
 * are host memory owned by the caller and not retained.
 * Errors: WV_EINVAL, WV_EDOMAIN (hi > WV_P_MAX), WV_ETRUNC, WV_ENOMEM, WV_EHIP. */
int wv_search_range(wv_ctx *ctx, uint64_t lo, uint64_t hi,
                    wv_result *out, size_t cap, size_t *n_out,
                    uint64_t *hits, size_t hit_cap, size_t *n_hits);

/* A prime whose symmetric residue is small (a "near miss"): the results of
 * Section 3 list the primes in (1e9, 1e11) with |<B_{p-3}>_p| < 50 (Table 2),
 * those of Section 5 the primes with |<E_{p-3}>_p| < 50 (Table 3); a hit
 * (residue 0) is the limiting case. */
typedef struct {
    uint64_t p;
    int64_t r;          /* symmetric residue in (-p/2, p/2] */
    uint32_t which;     /* WV_NEAR_B (Bernoulli) or WV_NEAR_E (Euler) */
    uint32_t reserved;
} wv_near;

enum { WV_NEAR_B = 1, WV_NEAR_E = 2 };

#define WV_MAX_BINS 65536u

/* Residue statistics over every prime p with max(lo,5) <= p < hi, without
 * returning the per-prime results (the distributions the histograms of
 * Sections 3 and 5 show: 2000 equal bins of <r>_p / p over (-1/2, 1/2]).
 * hist_b / hist_e (bins entries each, 1 <= bins <= WV_MAX_BINS) receive the
 * number of primes whose symmetric residue s of B_{p-3} (resp. E_{p-3}) falls
 * in bin k = floor((s/p + 1/2) * bins) = floor((2s + p) * bins / (2p)).
 * near receives the near misses |s| < near_bound (none for near_bound = 0)
 * sorted by (p, which); *n_near receives their total number; if it exceeds
 * near_cap, the first near_cap are written and the call returns WV_ETRUNC
 * after completing (histograms and *n_primes are then still valid).
 * *n_primes (may be NULL) receives the number of primes.  Host buffers owned
 * by the caller.  Errors: WV_EINVAL, WV_EDOMAIN, WV_ETRUNC, WV_ENOMEM, WV_EHIP. */
int wv_range_stats(wv_ctx *ctx, uint64_t lo, uint64_t hi, uint32_t bins, uint64_t near_bound,
                   uint64_t *hist_b, uint64_t *hist_e, wv_near *near, size_t near_cap, size_t *n_near,
                   uint64_t *n_primes);

/* ---- every index: irregular and E-irregular pairs (Section 1) --------------
 *
 * (p, 2k) is an irregular pair when p | B_{2k} and an E-irregular pair when
 * p | E_{2k} (secant convention), 2 <= 2k <= p - 3.  The residues come from
 * the paper's congruences for general index: B_{2k} from
 * C_k(a,b,c) B_{2k} == sum S_{2k-1}(x, y) (Section 2, with C_k(a,b,c) =
 * (a^{p-2k} + b^{p-2k} - c^{p-2k} - 1) / (4k)) for the family (2, b, b+1)
 * over sum_{m <= b/2} (m/(b+1), m/b): b = 3, i.e. (1/4, 1/3), and, for the k
 * where its C_k vanishes mod p, b = 4, 5, ... up to 64; E_t (t = 2k) from
 * eqnEMac2 (Section 4: (-1)^k' 4^(k'-1) (9^k' + 1) E_t == 2^t (S_t(0, 1/12)
 * - S_t(5/12, 1/2)), k' = (p - 1 - t)/2) and, where 9^k' == -1 (mod p), from
 * eqnE1 with the sign read as (-1)^k'.  The power sums of every exponent run
 * on the device: about p^2 / 8 terms per prime. */
#define WV_IRR_P_MAX (1ULL << 27)

typedef struct {
    uint64_t p;
    uint32_t two_k;   /* the index 2k */
    uint32_t kind;    /* 1: p | B_{2k} (irregular pair); 2: p | E_{2k} (E-irregular pair) */
} wv_irr_pair;

/* B_{2k} mod p and E_{2k} mod p for 2k = 2, 4, ..., p - 3 of one prime:
 * b[k-1] = B_{2k} mod p, e[k-1] = E_{2k} mod p in [0, p), k = 1 .. (p-3)/2
 * (caller-owned arrays of (p - 3) / 2 entries).  b[k-1] = UINT64_MAX marks a
 * k where every congruence of the chain degenerates.
 * Errors: WV_EINVAL (NULL), WV_EDOMAIN (p < 5 or p >= WV_IRR_P_MAX),
 * WV_ENOTPRIME, WV_ENOMEM, WV_EHIP. */
int wv_bernoulli_euler_all(wv_ctx *ctx, uint64_t p, uint64_t *b, uint64_t *e);

/* Kernel of the power sums behind wv_bernoulli_euler_all / wv_irregular_pairs:
 * 0 automatic (matrix cores for batches with every p < 2^24, where partial
 * sums of up to 1024 products, reduced mod p before they reach 2^53, stay
 * exact f64 integers; vector ALU otherwise),
 * 1 vector ALU always, 2 matrix cores where exact (same as 0).  Results do not
 * depend on it.  Errors: WV_EINVAL. */
int wv_set_irregular_path(wv_ctx *ctx, int path);

/* All irregular and E-irregular pairs of the primes p in [lo, hi) (p >= 5),
 * sorted by (p, 2k, kind) into out (caller-owned, cap entries).  *n_out: the
 * number of pairs; n_primes (optional): primes examined; n_unresolved
 * (optional): indices whose congruence chain degenerated (not reported as
 * pairs).  Short buffer: WV_ETRUNC with *n_out set, nothing written.
 * Errors: WV_EINVAL, WV_EDOMAIN (hi > WV_IRR_P_MAX), WV_ETRUNC, WV_ENOMEM
 * (also when one batch of primes yields more than 2^20 pairs), WV_EHIP. */
int wv_irregular_pairs(wv_ctx *ctx, uint64_t lo, uint64_t hi, wv_irr_pair *out, size_t cap, size_t *n_out,
                       uint64_t *n_primes, uint64_t *n_unresolved);

/* Batched search over nwin windows [lo[w], hi[w]) (may differ in size and
 * position): all windows are sieved together and all their primes go through
 * one plan and one persistent term-sum launch per batch (at most 2^19 primes,
 * 2^27 (prime, sum) slots and about 2^44 terms; a wide window at large p is
 * cut into sub-ranges that fall into several batches), with work split by
 * cost (equal-size chunks of the flat term space).  out
 * receives the results window by window, ascending p within a window;
 * win_off (nwin + 1 entries, may be NULL) receives each window's first index
 * and the total.  Short buffer: WV_ETRUNC with *n_out set, nothing written.
 * Errors as wv_search_range. */
int wv_search_windows(wv_ctx *ctx, const uint64_t *lo, const uint64_t *hi, size_t nwin,
                      wv_result *out, size_t cap, size_t *n_out, size_t *win_off);

/* Residues for n given primes (host memory), results in input order: the
 * same computation as wv_search_range (Sections 3 and 5, eqnDefnS,
 * eqnComputeS, eqnCombinePairs) for a caller-chosen list.  Each
 * p must satisfy 5 <= p < WV_P_MAX (else WV_EDOMAIN) and be prime (checked on
 * the host by deterministic Miller-Rabin; else WV_ENOTPRIME).  n == 0 is a
 * no-op. */
int wv_eval_primes(wv_ctx *ctx, const uint64_t *primes, size_t n, wv_result *out);

/* Device-pointer variant of wv_eval_primes (the same residues: Sections 3
 * and 5, eqnDefnS, eqnComputeS, eqnCombinePairs): d_primes and d_out are
 * device memory (e.g. torch tensors) of n entries, d_out in the wv_result
 * layout; the work is enqueued on hip_stream (a hipStream_t;
 * NULL = the legacy default stream) and the call returns without waiting.
 * The batch is padded to a power of two and the whole sequence of kernels is
 * replayed from a captured HIP graph cached per padded size (captured on the
 * first call of each size, which waits for the context's own stream).
 * The primes are not validated: each must be a prime in [5, WV_P_MAX); a
 * value outside that range yields a result with flags = 0xFFFFFFFF, and so
 * does every prime of the call if the term sums report an internal error
 * (a wave stopped before the work ran out; not expected in a correct run).  The
 * caller keeps both buffers alive until the stream has passed this work.
 * Internal buffers of ctx are in use until then: do not issue another call on
 * ctx before synchronising hip_stream.  One batch: the padded size times the
 * sums per prime must not exceed 2^27 (WV_EINVAL otherwise; 2^21 primes with
 * the printed tables). */
int wv_eval_primes_async(wv_ctx *ctx, const uint64_t *d_primes, size_t n,
                         wv_result *d_out, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and the same arguments and results as wv_eval_primes_async, but
 * the call allocates nothing, captures no graph and never synchronises.
 * Every intermediate buffer lives in one fixed device array of
 * WV_STATIC_SCRATCH_BYTES that the library holds on each GPU it runs on until
 * the process ends (looked up by wv_create); ctx contributes only its
 * congruence tables and settings.  Limits: n <= WV_STATIC_MAX_PRIMES and n
 * times the sums per prime <= WV_STATIC_MAX_SLOTS (524288: 8322 primes with
 * the printed tables, 8 with the top rungs of the package's derived ladders,
 * whose lower rungs fit more); larger calls
 * return WV_EINVAL before enqueueing anything.  All calls on one GPU share
 * that GPU's array, which keeps the last call's contents: calls whose work
 * overlaps on one GPU (other streams, other contexts, other host threads)
 * race; order them on one stream or synchronise between them.  The words that
 * must start at zero are cleared by kernels of the call itself.
 * Errors: WV_EINVAL, WV_EHIP. */
#define WV_STATIC_MAX_PRIMES 65536ULL
#define WV_STATIC_MAX_SLOTS (1ULL << 19)
#define WV_STATIC_MAX_CHUNKS (1ULL << 20)
#define WV_STATIC_SCRATCH_BYTES (60ULL << 20)
int wv_eval_primes_static(wv_ctx *ctx, const uint64_t *d_primes, size_t n,
                          wv_result *d_out, void *hip_stream);

/* Testing aid: the individual sums S_j = sum_{x_j p < s < y_j p} s^-deg mod p
 * (Section 2, eqnDefnS; deg 3 on the Bernoulli side, 2 on the Euler side) of
 * the congruences the context uses for each prime, computed by the same
 * kernels as wv_eval_primes.  out_b[i*nb + j] receives the j-th Bernoulli
 * sum of primes[i] and out_e[i*ne + j] the j-th Euler sum, canonical in
 * [0, p); nb and ne are the numbers of sums of the configured congruences
 * (wv_table_info), and slots beyond the congruence used for a prime (p = 5, 7
 * use one-sum root forms) hold 0.  Same validation as wv_eval_primes; one
 * batch of at most 2^27 (prime, sum) slots (WV_EINVAL beyond). */
int wv_eval_sums(wv_ctx *ctx, const uint64_t *primes, size_t n, uint64_t *out_b, uint64_t *out_e);

/* ---- request server ---------------------------------------------------
 * Continuous batching of mixed requests (prime lists and intervals) on one
 * context.  Admitted requests keep their primes, per-sum plans and running
 * pairs (c0, c1) in a device pool; each step takes whole primes of the active
 * requests, about `step_terms` terms in all (an even share per request, the
 * rest to the smallest remaining work first, at least one prime), runs every
 * sum of those primes through the term-sum kernels and folds it into its
 * pair with eqnCombinePairs (Section 3).  Requests that arrive while others
 * run join at the next step; results do not depend on the interleaving (exact
 * arithmetic, associative product).  All device work goes on the context's
 * stream in call order (admission between steps); the host keeps no per-sum
 * state and copies from pinned staging.  Do not call other entry points on
 * the context between steps except wv_get_stats.  The congruences are those
 * set on the context at creation; the pool holds max_primes times their
 * sums, fewer than 2^32 (else WV_EINVAL). */
typedef struct wv_server wv_server;

typedef struct {
    uint64_t step_terms;   /* terms of work per step (0: 2^38, ~45 ms at p ~ 1e11) */
    uint32_t max_primes;   /* prime slots of the device pool (0: 65536, or fewer so that the pool
                              holds at most 2^30 (prime, sum) slots, at least 1024 primes) */
    uint32_t reserved;
} wv_server_config;

typedef struct {
    uint64_t submitted, completed, pending, active;
    uint64_t primes_done, terms_done, steps, readmits;
    double p50_ms, p99_ms, mean_ms, max_ms; /* submit-to-completion latency, requests completed without error */
    double busy_s;                          /* device time of the steps */
    double wall_s;                          /* since the first submit */
    uint64_t failed;                        /* requests that ended with an error (counted in completed) */
    uint64_t terms_done_b;                  /* Bernoulli-side (s^-3) terms of terms_done */
    double sum_s;                           /* device time of the term-sum kernel launches */
    uint32_t block_k_b, block_k_e;          /* block shape of the term-sum kernel */
} wv_server_stats;

int wv_server_create(wv_ctx *ctx, const wv_server_config *cfg, wv_server **out);
int wv_server_destroy(wv_server *srv);
/* Every prime of [lo, hi) (at most 2^26 integers wide).  The primes are counted
 * on the host at submission (a segmented sieve, no device work): a range
 * holding more primes than the pool (max_primes) is refused with WV_EINVAL and
 * nothing is queued.  At admission the device sieves the range again; a count
 * that disagrees ends the request with WV_EHIP. */
int wv_server_submit_range(wv_server *srv, uint64_t lo, uint64_t hi, uint64_t *id);
/* A list of primes (validated like wv_eval_primes; at most max_primes). */
int wv_server_submit_primes(wv_server *srv, const uint64_t *primes, size_t n, uint64_t *id);
/* Admit what fits, launch the next step of work, then wait for the step the
 * previous call launched: steps are pipelined two deep, so the caller's work
 * between calls and the host's planning overlap the device's work.  A
 * request is finalized at the end of the step that holds its last primes and
 * its results become available in the call that completes that step
 * (wv_server_result says WV_EBUSY until then).  A step holds about
 * step_terms terms (default 2^38, about 45 ms of the whole GPU at p ~ 1e11)
 * and at most 2^23 sums (2^22 while a request with at most an eighth of
 * step_terms left is active, so that it completes in a short step).
 * Admission takes requests pending for 2 s or more in
 * arrival order, then the smallest first (by number of primes), and plans at
 * most 2^24 sums per call; a request that does not fit in the pool waits
 * without blocking others.  A request whose admission fails ends with that error (see
 * wv_server_result) and frees its pool slots.  A failed step (HIP error, or
 * term sums that did not cover every chunk) returns its error after
 * restarting every active request from its plan, so no partial state of the
 * failed step survives (the step launched after it is discarded too); after
 * 3 failed steps with no step completed between them the active requests end
 * with the error instead.  The server stays usable either way. */
int wv_server_step(wv_server *srv, uint32_t *n_active, uint32_t *n_pending);
/* Results of a finished request (then forgotten); WV_EBUSY while it runs,
 * WV_ETRUNC (with *n_out) if cap is short.  A request that ended with an error
 * returns that error once (with *n_out = 0) and is forgotten.
 * latency_ms: submit to completion. */
int wv_server_result(wv_server *srv, uint64_t id, wv_result *out, size_t cap, size_t *n_out,
                     double *latency_ms);
int wv_server_get_stats(const wv_server *srv, wv_server_stats *out);
/* Testing aid: the step that ends `after_steps` steps from now reports a
 * failure after its GPU work (forced on the host), exercising the restart. */
int wv_server_inject_fault(wv_server *srv, int after_steps);

/* Statistics of the last search/eval call (synchronous calls only). */
int wv_get_stats(const wv_ctx *ctx, wv_stats *out);

/* Describe congruence `id`: number of sums, left-side multiplier and the exact
 * cost numerator/denominator (sum of y_i - x_i).  For tests. */
int wv_table_info(int id, int *n_sums, int64_t *lhs, uint64_t *cost_num, uint64_t *cost_den);

/* Term i of congruence `id`: coefficient and the endpoints x = xa/xb, y = ya/yb. */
int wv_table_term(int id, int i, int64_t *coef, uint32_t *xa, uint32_t *xb,
                  uint32_t *ya, uint32_t *yb);

/* Message for a status code (static storage). */
const char *wv_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* WVPRIME_H */
