// wv_ctx.hpp -- the context behind the opaque wv_ctx handle and the host-side
// pipeline helpers shared by the C ABI (wv_capi.hip), the autotuner
// (wv_tune.hip) and the request server (wv_server.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "wv_internal.hpp"
#include "wv_tables.hpp"
#include "wvprime.h"

#define WV_TRY(expr)                  \
    do {                              \
        int _rc = (expr);             \
        if (_rc != WV_OK) return _rc; \
    } while (0)

#define WV_HIP(expr)                                                                                  \
    do {                                                                                              \
        hipError_t _e = (expr);                                                                       \
        if (_e != hipSuccess) {                                                                       \
            if (getenv("WV_DEBUG"))                                                                   \
                fprintf(stderr, "wvprime: %s:%d %s: %s\n", __FILE__, __LINE__, #expr, hipGetErrorString(_e)); \
            return _e == hipErrorOutOfMemory ? WV_ENOMEM : WV_EHIP;                                   \
        }                                                                                             \
    } while (0)

namespace wv {

struct DevBuf {
    void *ptr = nullptr;
    size_t cap = 0;
};

template <class T>
T *as(DevBuf &b) { return reinterpret_cast<T *>(b.ptr); }

enum { EV_START, EV_SIEVE, EV_PLAN0, EV_PLAN, EV_SUM0, EV_SUM, EV_RED, EV_FINAL, EV_COUNT };

constexpr uint64_t kDefaultChunk = 0;            // 0: adaptive_chunk per batch
constexpr uint64_t kMaxChunks = 1ull << 27;      // partial pairs held at once (2 GiB)
constexpr uint64_t kMinChunks = 1ull << 16;
constexpr size_t kMaxBatchSegs = 64;             // sieve segments per search batch (4 MiB of bitmaps)
constexpr uint64_t kMaxBatchPrimes = 1ull << 19; // primes per search batch
constexpr uint64_t kMaxBatchSlots = 1ull << 27;  // (prime, sum) slots per batch (~10 GB of plan records)
constexpr double kMaxBatchTerms = 17592186044416.0;   // 2^44 terms per search batch (~3 s)
constexpr size_t kSieveLaunch = 1 << 16;         // segments per counting launch
constexpr int kDefaultVariant = 9;               // block shape 28/36

// scal words of a batch: [0] total terms, [1..3] chunk layout {chunk size,
// full chunks, tails}, [4] total chunks, [5] chunk counter, [6]
// Bernoulli-side terms, [7] term-sum error word (nonzero: a wave hit its
// iteration bound)
constexpr int kScalTerms = 0, kScalLayout = 1, kScalChunks = 4, kScalCounter = 5, kScalTermsB = 6, kScalErr = 7;

// Device buffers of one batch of primes (plan -> sums -> reduce -> finalize):
// the context's growable buffers, or a carve-up of a fixed scratch area.
struct BatchBufs {
    PrimeRec *pr;               // n
    SegRec *segs;               // nseg
    uint64_t *terms, *cnt;      // nseg
    uint64_t *off;              // nseg + 1
    uint64_t *tiles;            // ceil(nseg / kScanTile) + 1
    uint64_t *scal;             // 8
    Pair *partials;             // cap
    Pair *seg_pairs;            // nseg
    uint64_t *coefs;            // nseg
    uint64_t *lhsmod;           // 2 n
    uint32_t *tails;            // nseg
    unsigned long long *tail_hist;   // 2 kTailClasses
};

struct BatchShape {
    int tb, te;          // tables of the batch (a defined table's fallback when no prime reaches its min_p)
    uint32_t n;          // primes
    int nB, nE;          // slots per prime on each side
    uint64_t nseg;       // (prime, sum) slots
    uint64_t cap;        // partial-pair capacity
};

struct GraphEntry {
    uint64_t n_pad, gen;
    int variant, tb, te;
    uint64_t chunk;
    hipGraphExec_t exec;
    uint64_t ns = 0;       // search graphs: sieve segments (0: the eval graph)
    int tbl_b = -1, tbl_e = -1;   // search graphs: the batch's table choice
};

// Per-batch consumer of device results that never go to the host: residue
// histograms accumulated on the device, near misses gathered per batch.
struct StatsSink {
    uint32_t bins;
    uint64_t bound;
    std::vector<wv_near> near;   // host copy, all batches
};

struct TuneEntry {
    int log2p;           // primes in [2^log2p, 2^(log2p+1))
    int variant;
    uint64_t chunk;
    double terms_per_s;
};

}  // namespace wv

struct wv_ctx {
    int device = 0;
    char arch[64] = {};
    hipStream_t stream = nullptr;
    hipEvent_t ev[wv::EV_COUNT] = {};
    int tb = WV_TABLE_BB30, te = WV_TABLE_EE33;
    uint64_t chunk_cfg = 0;                       // user setting (0: automatic)
    uint64_t chunk_auto = wv::kDefaultChunk;      // automatic value (tuned; 0: adaptive)
    int variant = wv::kDefaultVariant;            // term-sum block shape
    bool shape_forced = false;
    int num_cus = 0;
    int sum_blocks[16] = {};                      // persistent grid per block shape
    uint32_t n_base = 0;
    uint64_t gen = 0;                             // bumped on every device reallocation
    wv::DevBuf base_primes, primes, pr, segs, terms, cnt, off, tiles, scal, partials, seg_pairs, results,
        seg_counts, seg_bits, seg_off, seg_desc, pad_primes, stats_hist, stats_near, coefs, lhsmod, tbl_head,
        tbl_term, tbl_limb, tails, tail_hist, irr_tasks, irr_units, irr_primes, irr_roff, irr_v, irr_fix,
        irr_counts, irr_pairs, irr_b, irr_e;
    // congruence registry: the compiled tables (ids < WV_TABLE_COUNT), then
    // those defined at run time; device copy in tbl_* (TableStore)
    std::vector<wv::TableHead> t_head;
    std::vector<wv::TableTerm> t_term;
    std::vector<uint32_t> t_limb;
    std::vector<double> t_cost;
    wv_stats stats{};
    wv_progress_fn progress = nullptr;
    void *progress_user = nullptr;
    uint64_t launch_terms = 1ull << 44;
    int irr_path = 0;                             // 0 automatic, 1 vector ALU, 2 matrix cores
    std::vector<wv::GraphEntry> graphs;
    std::vector<wv::TuneEntry> tune;
    void *scratch = nullptr;                      // this device's fixed scratch array (wv_eval_primes_static)
    wv_result *pin_res = nullptr;                 // pinned staging of results copied to the caller
    size_t pin_res_cap = 0;
};

namespace wv {

// lanes of the persistent term-sum grid of the current block shape
inline uint64_t sum_lanes(const wv_ctx *c) { return (uint64_t)c->sum_blocks[c->variant] * 256; }

constexpr int kMaxDefinedTables = kMaxTableChain;
constexpr size_t kMaxTableTerms = 1 << 16;

// table registry (wv_capi.hip)
int tables_init(wv_ctx *c);
int table_add(wv_ctx *c, int deg, const std::vector<uint32_t> &lhs_mag, bool lhs_neg,
              const std::vector<std::vector<uint32_t>> &coef_mag, const std::vector<bool> &coef_neg,
              const uint64_t *xa, const uint64_t *xb, const uint64_t *ya, const uint64_t *yb, uint64_t min_p,
              int *id);
TableStore table_store(wv_ctx *c);
// the printed table of id's degree (the last resort of the device's choice)
int table_fallback(const wv_ctx *c, int id);
// the table a batch of primes below pmax starts from on the side configured
// with id (defined tables hand the primes below their min_p down their chain)
int batch_table(const wv_ctx *c, int id, uint64_t pmax);
// slots and cost per p a side that starts from `id` must allow for: the
// largest over its chain of tables
int side_slots(const wv_ctx *c, int id);
double side_cost(const wv_ctx *c, int id);
// cost per p of the table of id's chain that serves a prime of size p
double prime_cost(const wv_ctx *c, int id, uint64_t p);

int ensure(wv_ctx *c, DevBuf &b, size_t bytes);
bool is_prime_u64(uint64_t n);
int check_device(wv_ctx *c);
// pmax: an upper bound on the batch's primes (sizes the partial-pair buffer)
int batch_shape(const wv_ctx *c, uint32_t n, uint64_t pmax, BatchShape *sh);
int prepare(wv_ctx *c, const BatchShape &sh);
// the context's batch buffers (after prepare)
BatchBufs ctx_bufs(wv_ctx *c);
// The three stages of a batch, enqueued on st with buffers b (sized for sh);
// nothing is allocated, every word that must start at zero is cleared by a
// kernel, so the sequence can be captured in a graph.
int enqueue_plan(wv_ctx *c, const BatchBufs &b, const uint64_t *d_primes, const BatchShape &sh, hipStream_t st);
int enqueue_sum(wv_ctx *c, const BatchBufs &b, const BatchShape &sh, hipStream_t st, uint64_t begin, uint64_t end);
int enqueue_finish(wv_ctx *c, const BatchBufs &b, const BatchShape &sh, hipStream_t st, wv_result *d_out);
int run_batch_sync(wv_ctx *c, const uint64_t *d_primes, uint32_t n, uint64_t pmax, wv_result *d_out);
// the segments of [lo, hi) (kSegSpan integers each), every one cut into
// sub-ranges of at most `piece` integers
void window_descs(uint64_t lo, uint64_t hi, std::vector<SegDesc> &d, uint64_t piece = kSegSpan);
// sub-range width whose primes near hi hold about half a search batch of work
uint64_t window_piece(const wv_ctx *c, uint64_t hi);
// st: the stream to use (nullptr: the context's); both wait for their own work
// (compact leaves the compaction enqueued on st)
int sieve_count(wv_ctx *c, const SegDesc *descs, size_t ns, bool keep_bits, uint32_t *counts,
                hipStream_t st = nullptr);
// descs_ready: c->seg_desc already holds descs[0..ns) (the sieve uploaded them)
int compact(wv_ctx *c, const SegDesc *descs, size_t ns, const uint32_t *counts, uint64_t *np_out,
            hipStream_t st = nullptr, bool descs_ready = false);
// out: host results (may be NULL when sink is set), written contiguously in
// desc order, or, with dest, the primes of descs[k] at out + dest[k];
// sink: device statistics; bits_ready: the counting pass kept the bitmaps of
// every descriptor, in this order, in c->seg_bits
int search_descs(wv_ctx *c, const std::vector<SegDesc> &descs, const std::vector<uint32_t> &counts,
                 wv_result *out, StatsSink *sink = nullptr, const uint64_t *dest = nullptr, bool bits_ready = false);
void pick_tuned(wv_ctx *c, uint64_t pmax);
// n results from the device to host memory `out` through the pinned staging
// buffer (a pageable copy costs several times more); waits on the context
// stream
int results_to_host(wv_ctx *c, const wv_result *d, size_t n, wv_result *out);
int pin_res_reserve(wv_ctx *c, size_t n);
// an upper bound on the primes in [lo, hi) (lo >= 5)
uint64_t prime_count_bound(uint64_t lo, uint64_t hi);
// Work (terms, estimated from the prime-count bound) below which a
// single-window search runs as one replayed graph (a few ms of the GPU).
constexpr double kGraphSearchTerms = 17179869184.0;
// Returns kGraphNotTaken (and does nothing) when the batch would exceed one
// batch's slots; the caller then takes the counted path.
constexpr int kGraphNotTaken = 1;
int search_graph(wv_ctx *c, const std::vector<SegDesc> &d, uint64_t n_bound, uint64_t pmax, wv_result *out,
                 size_t *n_out);
// device address of the fixed scratch array on `device` (current), looked up
// once per device (wv_static.hip)
int static_scratch_setup(int device, void **addr);

}  // namespace wv
