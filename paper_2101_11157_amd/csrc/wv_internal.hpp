// wv_internal.hpp -- records shared by the device kernels and the host code
// of libwvprime.so, and the host-side launchers of the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "wvprime.h"

namespace wv {

constexpr int kSegLog = 20;                    // sieve segment: 2^20 integers
constexpr uint64_t kSegSpan = 1ull << kSegLog;
constexpr int kSegBits = 1 << (kSegLog - 1);   // odd integers per segment
constexpr int kSegWords = kSegBits / 32;       // 16384 words = 64 KiB of LDS
constexpr uint32_t kBaseLimit = 1u << 20;      // base primes below 2^20 cover p < 2^40
constexpr int kScanTile = 1024;                // elements per scan workgroup
constexpr int kMaxTableChain = 64;              // defined tables per context (and so per chain)

// One sieve segment: the 2^20 integers [L, L + 2^20) (L even), of which the
// window [lo, hi) keeps the primes p >= 5.  Segments of several windows can
// share one launch (batched search).
constexpr uint64_t kChunkSetup = 4096;         // set-up work of one chunk, in terms
constexpr uint64_t kChunkMin = 1ull << 12;
constexpr uint64_t kChunkMax = 1ull << 19;
constexpr int kTailBuckets = 64;                 // length classes of the tail chunks
constexpr int kTailClasses = 2 * kTailBuckets;   // (length class, side)

// Length class of a tail of rem in [1, C) terms; class 0 holds the longest.
// Classes are geometric, eight per octave below C (lengths within a class
// differ by at most 9 %), so that the 64 tails of a wave have nearly equal
// lengths also when the sums are much shorter than a chunk; tails below
// C / 2^8 share the last class.
constexpr int kTailPerOctave = 8;
__host__ __device__ inline uint32_t tail_bucket(uint64_t rem, uint64_t C) {
    const double x = log2((double)C / (double)rem) * kTailPerOctave;   // > 0 for rem < C
    return x >= kTailBuckets - 1 ? (uint32_t)(kTailBuckets - 1) : (uint32_t)x;
}

// Order of a tail among all tails: by length class, longest first, and
// within a class the s^-3 sums before the s^-2 sums, so that the 64 tails a
// wave takes run one code path (a wave holding both sides runs both loops).
__host__ __device__ inline uint32_t tail_class(uint64_t rem, uint64_t C, uint32_t deg) {
    return 2 * tail_bucket(rem, C) + (deg == 3 ? 0u : 1u);
}

// Automatic chunk size for T terms: sqrt(2 S T / w), clamped, where w counts
// the lanes of the grid (see k_pick_chunk).
__host__ __device__ inline uint64_t adaptive_chunk(uint64_t T, uint64_t w) {
    const double c = sqrt(2.0 * (double)kChunkSetup * (double)T / (double)(w ? w : 1));
    const uint64_t k = (uint64_t)c;
    return k < kChunkMin ? kChunkMin : (k > kChunkMax ? kChunkMax : k);
}

struct SegDesc {
    uint64_t L, lo, hi;
};

struct PrimeRec {      // 32 bytes
    uint64_t p;
    uint64_t r2;       // R^2 mod p
    uint64_t one;      // R mod p
    uint32_t ninv;     // -p^-1 mod 2^32
    uint8_t tb, te;    // congruences used
    uint8_t ok, pad;
};

struct SegRec {        // one (prime, sum)
    uint64_t lo;       // first s
    uint64_t len;      // number of s; 0 for an unused slot
    uint32_t prime;    // index in the batch
    uint32_t deg;      // 3 (B) or 2 (E)
};

struct Pair {
    uint64_t c0, c1;
};

// Request server: a step takes whole primes of the pool, span by span.  Span:
// primes [i0, i0 + cnt) of the request planned at pool sums seg0.. (its n
// primes laid out as a batch: B sums of prime i at i*nB + j, E sums at
// n*nB + i*nE + j), numbered q0.. among the step's primes.
struct StepSpan {
    uint64_t seg0;
    uint32_t nreq, i0, q0, cnt;
};

// A request finalized at the end of a step: pool slots [base, base + n), its
// results at out[out0 .. out0 + n).
struct FinReq {
    uint32_t base, n, out0, pad;
};

// A congruence  lhs * X_{p-3} == sum_i coef_i S(x_i, y_i)  (mod p) in device
// memory (compiled tables and tables defined at run time alike).  Integers of
// any size are little-endian base-2^32 limbs of the magnitude plus a sign.
struct TableTerm {      // 40 bytes
    uint64_t xa, xb, ya, yb;   // x = xa/xb < y = ya/yb
    uint32_t limb_off;         // coefficient magnitude: limbs[limb_off .. limb_off + nlimb)
    uint16_t nlimb;
    int16_t neg;
};

struct TableHead {      // 32 bytes
    int32_t deg, n;            // 3: s^-3 (B), 2: s^-2 (E); number of sums
    uint32_t term_off, lhs_off;
    uint16_t lhs_nlimb;
    int16_t lhs_neg;
    int32_t below;             // defined tables: the table for the other primes (-1 for compiled ones)
    uint64_t min_p;            // used for p >= min_p (and p not dividing lhs)
};

struct TableStore {
    const TableHead *head;
    const TableTerm *term;
    const uint32_t *limb;
};

// ---- launchers (wv_kernels.hip) ---------------------------------------------
// Every launcher enqueues on `st` and returns hipGetLastError().

hipError_t launch_base_sieve(hipStream_t st, uint32_t *out, uint32_t *n_out);
hipError_t launch_seg_sieve(hipStream_t st, const SegDesc *desc, unsigned ns, const uint32_t *bp, uint32_t n_bp,
                            uint32_t *bits_out, uint32_t *counts);
// primes of segment i at out[off[i] ..], written only below out[limit]
hipError_t launch_seg_compact(hipStream_t st, const SegDesc *desc, unsigned ns, const uint32_t *bits,
                              const uint64_t *off, uint64_t *out, uint64_t limit);
// off[0..ns] = exclusive prefix of counts[0..ns) (ns <= 1024); unless expect
// is UINT64_MAX, a total other than `expect` sets every off[i] = expect (a
// compaction then writes nothing) and primes[0..expect) = 0 (primes the plan
// rejects)
hipError_t launch_seg_offsets(hipStream_t st, const uint32_t *counts, unsigned ns, uint64_t expect, uint64_t *off,
                              uint64_t *primes);
// exclusive scan of n values into out[0..n], out[n] = total; tiles holds
// ceil(n / kScanTile) entries
hipError_t launch_scan(hipStream_t st, const uint64_t *in, uint64_t n, uint64_t *out, uint64_t *tiles);
// Plan of a batch of n primes with tables tb / te (per prime: fb / fe where
// p < min_p or p divides the table's lhs; the compiled root forms for p = 5, 7):
// PrimeRec, SegRec and term count per (prime, sum) slot, each slot's
// coefficient mod p (coefs, same layout as segs) and each prime's two lhs
// residues (lhsmod[2i], lhsmod[2i + 1]).
hipError_t launch_plan(hipStream_t st, const uint64_t *primes, uint32_t n, int tb, int te, int fb, int fe, int nB,
                       int nE, TableStore ts, PrimeRec *pr, SegRec *segs, uint64_t *terms, uint64_t *coefs,
                       uint64_t *lhsmod, uint32_t prime_base);
hipError_t launch_pick_chunk(hipStream_t st, const uint64_t *total_terms, uint64_t nseg, uint64_t chunk_cfg, uint64_t lanes,
                             uint64_t cap, uint64_t *chunk_out);
// Chunk layout (layout = {C, full chunks, tails}; layout[0] set by the pick):
// cnt[i] = full chunks of sum i, off = their exclusive prefix (off[nseg] =
// full chunks), tails[0..) = the sums whose length C does not divide, longest
// tail class first (tail_class: slots below nb_slots are s^-3 sums, the rest
// s^-2); *total_chunks = full chunks + tails.  hist holds 2 kTailClasses
// counters, scan_tiles as for launch_scan.
hipError_t launch_chunk_layout(hipStream_t st, const uint64_t *terms, uint64_t nseg, uint64_t nb_slots, uint64_t *layout,
                               uint64_t *cnt, uint64_t *off, uint64_t *scan_tiles, unsigned long long *hist,
                               uint32_t *tails, uint64_t *total_chunks);
hipError_t launch_set_u64(hipStream_t st, uint64_t *dst, int n, uint64_t value);
hipError_t launch_copy_u64(hipStream_t st, const uint64_t *src, uint64_t *dst, int n);
// Persistent term sums over the chunks [begin, min(end, total)) of a chunk
// layout; the counter at *counter must hold `begin` (a multiple of 64).  Full
// chunks leave pairs in partials, tails in seg_pairs[sum].  *err becomes
// nonzero if a wave stopped at its iteration bound before the chunks ran out
// (never in a correct run; the caller reports it as a failure).
int num_sum_variants();
int sum_variant_kb(int v);
int sum_variant_ke(int v);
hipError_t sum_variant_occupancy(int v, int *blocks_per_cu);
hipError_t launch_sum(hipStream_t st, int v, unsigned grid, const SegRec *segs, const uint64_t *off, uint32_t nseg,
                      const PrimeRec *pr, const uint64_t *layout, const uint32_t *tails, Pair *partials,
                      Pair *seg_pairs, unsigned long long *counter, uint64_t end, unsigned long long *err);
// seg_pairs[j] <- the pairs of sum j's full chunks joined with its tail's
hipError_t launch_reduce(hipStream_t st, const SegRec *segs, const uint64_t *off, uint32_t nseg, const PrimeRec *pr,
                         const Pair *partials, const uint64_t *layout, Pair *seg_pairs);
// err (may be null): the term-sum error word; when it is nonzero every result
// of the batch is marked invalid (flags = 0xFFFFFFFF)
hipError_t launch_finalize(hipStream_t st, TableStore ts, const PrimeRec *pr, const Pair *sp, const uint64_t *coefs,
                           const uint64_t *lhsmod, uint32_t n, int nB, int nE, wv_result *out,
                           const unsigned long long *err);
hipError_t launch_sum_values(hipStream_t st, const SegRec *segs, const PrimeRec *pr, const Pair *sp, uint64_t nseg,
                             uint64_t *out);
// acc[target[t]] <- acc[target[t]] (x) tp[t] (eqnCombinePairs), t < ntask
hipError_t launch_fold(hipStream_t st, const SegRec *tasks, const uint32_t *target, const Pair *tp, uint32_t ntask,
                       const PrimeRec *pr, Pair *acc);
hipError_t launch_fill_pairs(hipStream_t st, Pair *p, uint64_t n, uint64_t c0, uint64_t c1);
// The tasks of a request-server step: nq whole primes over nsp spans, B tasks
// of all of them first, then E tasks; tasks[t] = segs[g], terms[t] = its
// length, target[t] = g (its pool index).
hipError_t launch_step_expand(hipStream_t st, const StepSpan *sp, uint32_t nsp, uint32_t nq, int nB, int nE,
                              const SegRec *segs, SegRec *tasks, uint64_t *terms, uint32_t *target);
// Finalize (a workgroup per prime) for several requests of the pool at once
// (FinReq list, `total` primes): pool arrays pr, acc, coefs, lhsmod with
// nB + nE sums per prime
hipError_t launch_finalize_multi(hipStream_t st, TableStore ts, const PrimeRec *pr, const Pair *acc,
                                 const uint64_t *coefs, const uint64_t *lhsmod, const FinReq *fr, uint32_t nfr,
                                 uint32_t total, int nB, int nE, wv_result *out, const unsigned long long *err);
// out[i] = i < n ? src[i] : 0  (zero marks a padding slot the plan rejects)
hipError_t launch_copy_pad(hipStream_t st, const uint64_t *src, uint64_t n, uint64_t *dst, uint64_t n_pad);
hipError_t launch_copy_results(hipStream_t st, const wv_result *src, uint64_t n, wv_result *dst);
// hist[w * bins + k] += primes whose symmetric residue (w = 0: b, 1: e) falls
// in bin k; residues with |s| < bound appended at near[atomic (*near_n)++]
// (room for 2n entries)
hipError_t launch_stats(hipStream_t st, const wv_result *res, uint32_t n, uint32_t bins, uint64_t bound,
                        unsigned long long *hist, wv_near *near, unsigned long long *near_n);



}  // namespace wv
