// wv_server.hip -- request server with continuous batching at prime
// granularity (the serving loop of the residue search).
//
// Requests (a prime list, or every prime of an interval) are admitted into a
// device pool of prime slots when a contiguous range of slots is free: their
// primes are planned into the pool (PrimeRec, one SegRec per (prime, sum)) and
// each sum gets an accumulator pair (c0, c1) = (1, 0) on the device.  Every
// step takes whole primes of the active requests -- a fair share of a budget
// of terms each, smallest remaining work first -- expands them into tasks (one
// per sum) on the device, runs them through the same term-sum and reduction
// kernels as a batch, and folds each task's pair into its sum's accumulator
// with eqnCombinePairs (Section 3).  A request whose last primes a step holds
// is finalized at the end of that step (Sections 3 and 5 congruences), its
// results copied out with the step's and its slots freed when the step
// completes.  New requests join at the next step, so short requests overtake
// long ones instead of queueing behind them.
//
// Steps alternate between two streams (the context's and the server's own),
// one per set of step buffers, so that the next step's term sums take over
// the compute units as the running step's last waves finish instead of after
// them.  A call of wv_server_step admits what fits (sieve, compaction, plan
// into the pool, on the stream of the step it launches next), launches that
// step and then waits for the step launched by the previous call; the host
// never waits for the device otherwise.  Events order what crosses the
// streams: a step waits for the admissions enqueued on the other stream, and
// a step that finalizes a request waits for the other stream's last fold
// before its finalize (every sum is folded by exactly one step, so the folds
// themselves never touch the same pair).  The host keeps no per-sum state: a
// request is its pool slots and the number of its primes handed out.
// Host-to-device copies come from pinned staging buffers, so no copy waits
// for the device.
//
// Because the pair product is associative and commutative and all arithmetic
// is exact, a request's residues do not depend on how its work was cut into
// steps or interleaved with other requests.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "step_share.hpp"
#include "wv_ctx.hpp"

using namespace wv;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum { REQ_PENDING = 0, REQ_ACTIVE = 1, REQ_DONE = 2 };

struct Request {
    uint64_t id = 0;
    bool is_range = false;
    uint64_t lo = 0, hi = 0;
    std::vector<uint64_t> primes;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int state = REQ_PENDING;
    int status = WV_OK;        // WV_OK, or the error that ended the request
    uint64_t n_primes = 0;     // primes of a range (counted at submission) or list length
    uint64_t pmax = 0;         // an upper bound on its primes
    uint32_t n = 0;            // primes in the pool
    uint32_t base = 0;         // first pool slot
    uint32_t next = 0;         // primes handed to launched steps
    double tpp = 0;            // estimated terms per prime
    std::vector<wv_result> results;
};

// Pinned host memory that grows (only while no queued copy reads it).
template <class T>
int pinned_reserve(T *&p, size_t &cap, size_t n) {
    if (n <= cap) return WV_OK;
    const size_t want = std::max<size_t>(n, cap + cap / 2);
    T *q = nullptr;
    if (hipHostMalloc((void **)&q, want * sizeof(T), hipHostMallocDefault) != hipSuccess) return WV_ENOMEM;
    if (p) (void)hipHostFree(p);
    p = q;
    cap = want;
    return WV_OK;
}

// One step's device buffers, its pinned staging (reused once the step has
// completed), its events and the requests it finalizes.
struct StepSet {
    DevBuf spans, tasks, terms, cnt, off, tiles, target, tpairs, partials, tails, hist, scal, fin, res;
    StepSpan *spans_h = nullptr;
    size_t spans_cap = 0;
    FinReq *fin_h = nullptr;
    size_t fin_cap = 0;
    wv_result *res_h = nullptr;
    size_t res_cap = 0;
    uint64_t *scal_h = nullptr;     // pinned: the step's scalars (kScal* words) once it has run
    hipEvent_t ev0 = nullptr, ev_sum0 = nullptr, ev_sum = nullptr, ev1 = nullptr;
    bool busy = false;              // launched and not yet completed
    uint64_t id = 0;                // step number (1, 2, ...)
    std::vector<Request *> finishing;   // requests finalized at the end of this step
    std::vector<uint32_t> fin_out;      // their first result in res
};

// Pinned staging of the host-to-device copies one call enqueues; the two
// halves alternate between calls, and a half is refilled only after the
// copies of its previous call have run (its event).
struct Upload {
    char *h = nullptr;
    size_t cap = 0, used = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
};

}  // namespace

struct wv_server {
    wv_ctx *c = nullptr;
    hipStream_t own = nullptr;  // the second stream (set 1's); set 0 uses the context's
    hipEvent_t ev_adm[2] = {}, ev_fold[2] = {}, ev_ref = nullptr;
    bool adm_pending[2] = {}, adm_recorded[2] = {}, fold_recorded[2] = {};
    double busy_end_ms = 0, sum_end_ms = 0;   // ends of the device intervals counted so far (from ev_ref)
    uint64_t step_terms = 1ull << 38;
    uint32_t pool = 1u << 16;
    int tb = 0, te = 0;        // congruences fixed at creation (the pool layout depends on them)
    int nB = 0, nE = 0, NS = 0;
    DevBuf pr, segs, acc, terms, coefs, lhsmod, plist;   // pool (plist: each slot's prime)
    DevBuf sdesc, scount, sbits, soff;                    // sieve of one range admission
    StepSet set[2];
    int next = 0;              // the set the next launch uses
    uint64_t launched = 0;     // steps launched
    Upload up[2];
    int up_cur = 0;
    std::vector<std::pair<uint32_t, uint32_t>> free_ranges;   // (first slot, count), sorted
    std::deque<Request *> pending;
    std::vector<Request *> active;
    std::map<uint64_t, Request *> all;
    std::vector<uint32_t> base_primes;   // odd primes up to base_limit for the host-side prime count
    uint64_t base_limit = 0;
    uint64_t next_id = 1;
    uint64_t submitted = 0, completed = 0, failed = 0, primes_done = 0, terms_done = 0, terms_done_b = 0, steps = 0,
             readmits = 0;
    double sum_s = 0;          // device time of the term-sum launches
    int fail_streak = 0;       // failed steps since the last step that completed
    double t_first = 0, busy_s = 0;
    std::vector<double> lat_ms;
    int64_t fault_after = -1;  // host-forced step failure (tests)
};

namespace {

hipStream_t stream_of(const wv_server *s, int k) { return k == 0 ? s->c->stream : s->own; }

// Upload staging per half at creation (it grows for larger prime lists).
constexpr size_t kUploadBytes = 1u << 20;

bool pool_alloc(wv_server *s, uint32_t n, uint32_t *base) {
    for (size_t i = 0; i < s->free_ranges.size(); i++) {
        auto &r = s->free_ranges[i];
        if (r.second >= n) {
            *base = r.first;
            r.first += n;
            r.second -= n;
            if (r.second == 0) s->free_ranges.erase(s->free_ranges.begin() + i);
            return true;
        }
    }
    return false;
}

void pool_free(wv_server *s, uint32_t base, uint32_t n) {
    if (n == 0) return;
    s->free_ranges.push_back({base, n});
    std::sort(s->free_ranges.begin(), s->free_ranges.end());
    std::vector<std::pair<uint32_t, uint32_t>> merged;
    for (auto &r : s->free_ranges) {
        if (!merged.empty() && merged.back().first + merged.back().second == r.first) merged.back().second += r.second;
        else merged.push_back(r);
    }
    s->free_ranges.swap(merged);
}

// Primes p with max(lo, 5) <= p < hi (the device sieve's convention), by a
// segmented sieve of the odd numbers on the host.
uint64_t count_primes_host(std::vector<uint32_t> &base, uint64_t &limit, uint64_t lo, uint64_t hi) {
    lo = std::max<uint64_t>(lo, 5);
    if (hi <= lo) return 0;
    uint64_t r = (uint64_t)std::sqrt((double)hi);
    while (r * r > hi) r--;
    while ((r + 1) * (r + 1) <= hi) r++;
    if (r > limit) {
        // odd primes up to r (r <= 2^20 for hi <= 2^40), then a sentinel whose
        // square exceeds every hi
        std::vector<uint8_t> comp(r + 1, 0);
        base.clear();
        for (uint64_t q = 3; q <= r; q += 2) {
            if (comp[q]) continue;
            base.push_back((uint32_t)q);
            for (uint64_t x = q * q; x <= r; x += 2 * q) comp[x] = 1;
        }
        base.push_back(UINT32_MAX);
        limit = r;
    }
    constexpr uint64_t kOdd = 1u << 20;   // odd numbers per block
    std::vector<uint8_t> comp(kOdd);
    uint64_t count = 0;
    for (uint64_t a = lo | 1; a < hi; a += 2 * kOdd) {
        const uint64_t b = std::min<uint64_t>(hi, a + 2 * kOdd);
        const uint64_t m = (b - a + 1) / 2;   // odd numbers a, a + 2, ... below b
        std::fill(comp.begin(), comp.begin() + m, 0);
        for (uint32_t q : base) {
            const uint64_t qq = (uint64_t)q * q;
            if (qq >= b) break;
            uint64_t x = std::max(qq, (a + q - 1) / q * q);
            if (!(x & 1)) x += q;
            for (; x < b; x += 2ull * q) comp[(x - a) / 2] = 1;
        }
        for (uint64_t i = 0; i < m; i++) count += !comp[i];
    }
    return count;
}

// Estimated terms per prime of size p (the congruence that applies at p).
double terms_per_prime(const wv_server *s, uint64_t p) {
    const wv_ctx *c = s->c;
    return (double)p * (c->t_cost[batch_table(c, s->tb, p)] + c->t_cost[batch_table(c, s->te, p)]) + s->NS;
}

// Stage n bytes for a host-to-device copy into the current upload half.
int stage_upload(wv_server *s, const void *src, size_t n, void *dst, hipStream_t st) {
    Upload &u = s->up[s->up_cur];
    if (u.used + n > u.cap) {
        if (u.used) return WV_EBUSY;   // full: the caller retries in a later call
        // nothing of this half is in flight (its event was waited for)
        char *h = nullptr;
        if (hipHostMalloc((void **)&h, n, hipHostMallocDefault) != hipSuccess) return WV_ENOMEM;
        (void)hipHostFree(u.h);
        u.h = h;
        u.cap = n;
    }
    memcpy(u.h + u.used, src, n);
    WV_HIP(hipMemcpyAsync(dst, u.h + u.used, n, hipMemcpyHostToDevice, st));
    u.used = (u.used + n + 255) & ~(size_t)255;
    return WV_OK;
}

int finish_empty(wv_server *s, Request *r) {
    r->state = REQ_DONE;
    r->t_done = now_s();
    s->completed++;
    s->lat_ms.push_back((r->t_done - r->t_submit) * 1e3);
    return WV_OK;
}

// Ends a request with an error: its pool slots (if any) are freed, it keeps no
// results, and wv_server_result reports `status`.  Failed requests do not
// enter the latency statistics.
void fail_request(wv_server *s, Request *r, int status) {
    pool_free(s, r->base, r->n);
    r->n = 0;
    r->results.clear();
    r->status = status;
    r->state = REQ_DONE;
    r->t_done = now_s();
    s->completed++;
    s->failed++;
}

// Plans a pending request into the pool (enqueued on st).  Sets *admitted
// false when there is no room yet (slots, or staging for its copies); an
// error return leaves no pool slot taken.
int admit(wv_server *s, Request *r, bool *admitted, hipStream_t st) {
    wv_ctx *c = s->c;
    *admitted = false;
    const uint64_t n = r->n_primes;   // submission checked n <= pool
    if (n == 0) {
        *admitted = true;
        r->t_admit = now_s();
        return finish_empty(s, r);
    }
    uint32_t base = 0;
    if (!pool_alloc(s, (uint32_t)n, &base)) return WV_OK;
    r->base = base;
    r->n = (uint32_t)n;
    uint64_t *dp = as<uint64_t>(s->plist) + base;
    int rc = WV_OK;
    if (r->is_range) {
        std::vector<SegDesc> d;
        window_descs(r->lo, r->hi, d);   // at most kMaxBatchSegs (checked at submission)
        rc = stage_upload(s, d.data(), d.size() * sizeof(SegDesc), s->sdesc.ptr, st);
        if (rc == WV_OK && (launch_seg_sieve(st, as<SegDesc>(s->sdesc), (unsigned)d.size(), as<uint32_t>(c->base_primes),
                                             c->n_base, as<uint32_t>(s->sbits), as<uint32_t>(s->scount)) != hipSuccess ||
                            launch_seg_offsets(st, as<uint32_t>(s->scount), (unsigned)d.size(), n, as<uint64_t>(s->soff),
                                               dp) != hipSuccess ||
                            launch_seg_compact(st, as<SegDesc>(s->sdesc), (unsigned)d.size(), as<uint32_t>(s->sbits),
                                               as<uint64_t>(s->soff), dp, n) != hipSuccess))
            rc = WV_EHIP;
    } else {
        rc = stage_upload(s, r->primes.data(), n * sizeof(uint64_t), dp, st);
    }
    if (rc == WV_OK) {
        const size_t first = (size_t)base * s->NS, nseg = (size_t)n * s->NS;
        if (launch_plan(st, dp, (uint32_t)n, s->tb, s->te, table_fallback(c, s->tb), table_fallback(c, s->te), s->nB,
                        s->nE, table_store(c), as<PrimeRec>(s->pr) + base, as<SegRec>(s->segs) + first,
                        as<uint64_t>(s->terms) + first, as<uint64_t>(s->coefs) + first,
                        as<uint64_t>(s->lhsmod) + 2 * (size_t)base, base) != hipSuccess ||
            launch_fill_pairs(st, as<Pair>(s->acc) + first, nseg, 1, 0) != hipSuccess)
            rc = WV_EHIP;
    }
    if (rc != WV_OK) {
        (void)hipGetLastError();
        pool_free(s, r->base, r->n);
        r->n = 0;
        return rc == WV_EBUSY ? WV_OK : rc;   // no staging room: stays pending
    }
    r->t_admit = now_s();
    r->next = 0;
    r->tpp = terms_per_prime(s, r->pmax);
    r->state = REQ_ACTIVE;
    s->active.push_back(r);
    *admitted = true;
    return WV_OK;
}

// Restart every active request from its plan (after a failed step; nothing is
// in flight on either stream).
int readmit_all(wv_server *s) {
    for (Request *r : s->active) {
        r->next = 0;
        WV_HIP(launch_fill_pairs(s->c->stream, as<Pair>(s->acc) + (size_t)r->base * s->NS, (size_t)r->n * s->NS, 1, 0));
        s->readmits++;
    }
    WV_HIP(hipStreamSynchronize(s->c->stream));
    return WV_OK;
}

// Chooses the next step's primes on the host (step_share: an even share of
// the budget for every active request with primes left, then what is left of
// the budget to the smallest remaining work first, at least one prime per
// step) and launches the step with buffer set k on its stream.  The
// requests' counters advance now.  *launched is false when no request has
// primes left.
int launch_step(wv_server *s, int sk, bool *launched) {
    StepSet &ss = s->set[sk];
    wv_ctx *c = s->c;
    *launched = false;
    std::vector<Request *> cand;
    for (Request *r : s->active)
        if (r->next < r->n) cand.push_back(r);
    if (cand.empty()) return WV_OK;
    std::stable_sort(cand.begin(), cand.end(), [](const Request *a, const Request *b) {
        return (a->n - a->next) * a->tpp < (b->n - b->next) * b->tpp;
    });
    std::vector<ShareReq> share(cand.size());
    for (size_t k = 0; k < cand.size(); k++) share[k] = ShareReq{(uint64_t)(cand[k]->n - cand[k]->next), cand[k]->tpp};
    std::vector<uint32_t> give(cand.size(), 0);
    const uint64_t nq = step_share(share.data(), share.size(), (double)s->step_terms, (uint64_t)s->NS, give.data());
    // spans in candidate order; requests whose last primes this step holds
    // are finalized at its end
    std::vector<StepSpan> spans;
    std::vector<FinReq> fins;
    ss.finishing.clear();
    ss.fin_out.clear();
    uint32_t q0 = 0, nres = 0;
    double t_est = 0;
    for (size_t k = 0; k < cand.size(); k++) {
        if (!give[k]) continue;
        Request *r = cand[k];
        spans.push_back(StepSpan{(uint64_t)r->base * s->NS, r->n, r->next, q0, give[k]});
        q0 += give[k];
        t_est += give[k] * r->tpp;
        if (r->next + give[k] == r->n) {
            fins.push_back(FinReq{r->base, r->n, nres, 0});
            ss.finishing.push_back(r);
            ss.fin_out.push_back(nres);
            nres += r->n;
        }
    }
    const uint64_t nt = nq * (uint64_t)s->NS, nbt = nq * (uint64_t)s->nB;
    // partial pairs: room for the estimated terms at the configured (or
    // adaptive) chunk and for every task's tail; the device picks a chunk
    // size that fits whatever the terms turn out to be
    // consecutive steps overlap on the two streams, so a step's ragged end
    // costs little: its chunks are sized as for a launch four times its work
    // (fewer chunk set-ups); a configured or tuned size is kept
    uint64_t chunk_cfg = c->chunk_cfg ? c->chunk_cfg : c->chunk_auto;
    if (!chunk_cfg)
        chunk_cfg = (adaptive_chunk((uint64_t)std::min(4.0 * t_est, 1.8e19), sum_lanes(c)) + 63) & ~63ull;
    const double chunk = (double)chunk_cfg;
    const uint64_t cap = std::max<uint64_t>(
        2 * nt, (uint64_t)std::min<double>(std::max<double>(t_est / chunk + 2.0 * nt, (double)kMinChunks),
                                           (double)kMaxChunks));
    WV_TRY(ensure(c, ss.spans, spans.size() * sizeof(StepSpan)));
    WV_TRY(ensure(c, ss.tasks, nt * sizeof(SegRec)));
    WV_TRY(ensure(c, ss.terms, nt * sizeof(uint64_t)));
    WV_TRY(ensure(c, ss.cnt, nt * sizeof(uint64_t)));
    WV_TRY(ensure(c, ss.off, (nt + 1) * sizeof(uint64_t)));
    WV_TRY(ensure(c, ss.tiles, ((nt + kScanTile - 1) / kScanTile + 1) * sizeof(uint64_t)));
    WV_TRY(ensure(c, ss.target, nt * sizeof(uint32_t)));
    WV_TRY(ensure(c, ss.tpairs, nt * sizeof(Pair)));
    WV_TRY(ensure(c, ss.tails, nt * sizeof(uint32_t)));
    WV_TRY(ensure(c, ss.hist, 2 * kTailClasses * sizeof(uint64_t)));
    WV_TRY(ensure(c, ss.partials, cap * sizeof(Pair)));
    WV_TRY(ensure(c, ss.fin, std::max<size_t>(fins.size(), 1) * sizeof(FinReq)));
    WV_TRY(ensure(c, ss.res, std::max<size_t>(nres, 1) * sizeof(wv_result)));
    WV_TRY(pinned_reserve(ss.spans_h, ss.spans_cap, spans.size()));
    WV_TRY(pinned_reserve(ss.fin_h, ss.fin_cap, std::max<size_t>(fins.size(), 1)));
    WV_TRY(pinned_reserve(ss.res_h, ss.res_cap, std::max<size_t>(nres, 1)));
    memcpy(ss.spans_h, spans.data(), spans.size() * sizeof(StepSpan));
    if (!fins.empty()) memcpy(ss.fin_h, fins.data(), fins.size() * sizeof(FinReq));

    hipStream_t st = stream_of(s, sk);
    uint64_t *scal = as<uint64_t>(ss.scal);
    uint64_t *off = as<uint64_t>(ss.off);
    // admissions enqueued on the other stream come first
    if (s->adm_pending[1 - sk]) {
        WV_HIP(hipStreamWaitEvent(st, s->ev_adm[1 - sk], 0));
        s->adm_pending[1 - sk] = false;
    }
    WV_HIP(hipEventRecord(ss.ev0, st));
    WV_HIP(hipMemcpyAsync(ss.spans.ptr, ss.spans_h, spans.size() * sizeof(StepSpan), hipMemcpyHostToDevice, st));
    if (!fins.empty())
        WV_HIP(hipMemcpyAsync(ss.fin.ptr, ss.fin_h, fins.size() * sizeof(FinReq), hipMemcpyHostToDevice, st));
    WV_HIP(launch_set_u64(st, scal, 8, 0));
    WV_HIP(launch_step_expand(st, as<StepSpan>(ss.spans), (uint32_t)spans.size(), (uint32_t)nq, s->nB, s->nE,
                              as<SegRec>(s->segs), as<SegRec>(ss.tasks), as<uint64_t>(ss.terms),
                              as<uint32_t>(ss.target)));
    WV_HIP(launch_scan(st, as<uint64_t>(ss.terms), nt, off, as<uint64_t>(ss.tiles)));
    WV_HIP(launch_pick_chunk(st, off + nt, nt, chunk_cfg, sum_lanes(c), cap, scal + kScalLayout));
    WV_HIP(launch_copy_u64(st, off + nt, scal + kScalTerms, 1));
    WV_HIP(launch_copy_u64(st, off + nbt, scal + kScalTermsB, 1));
    WV_HIP(launch_chunk_layout(st, as<uint64_t>(ss.terms), nt, nbt, scal + kScalLayout, as<uint64_t>(ss.cnt), off,
                               as<uint64_t>(ss.tiles), as<unsigned long long>(ss.hist), as<uint32_t>(ss.tails),
                               scal + kScalChunks));
    WV_HIP(hipEventRecord(ss.ev_sum0, st));
    const int v = c->variant;
    WV_HIP(launch_sum(st, v, (unsigned)c->sum_blocks[v], as<SegRec>(ss.tasks), off, (uint32_t)nt, as<PrimeRec>(s->pr),
                      scal + kScalLayout, as<uint32_t>(ss.tails), as<Pair>(ss.partials), as<Pair>(ss.tpairs),
                      (unsigned long long *)(scal + kScalCounter), UINT64_MAX,
                      (unsigned long long *)(scal + kScalErr)));
    WV_HIP(hipEventRecord(ss.ev_sum, st));
    WV_HIP(launch_reduce(st, as<SegRec>(ss.tasks), off, (uint32_t)nt, as<PrimeRec>(s->pr), as<Pair>(ss.partials),
                         scal + kScalLayout, as<Pair>(ss.tpairs)));
    WV_HIP(launch_fold(st, as<SegRec>(ss.tasks), as<uint32_t>(ss.target), as<Pair>(ss.tpairs), (uint32_t)nt,
                       as<PrimeRec>(s->pr), as<Pair>(s->acc)));
    WV_HIP(hipEventRecord(s->ev_fold[sk], st));
    s->fold_recorded[sk] = true;
    if (!fins.empty()) {
        // the finalized requests' earlier primes may have been folded by the
        // other stream's step
        if (s->fold_recorded[1 - sk]) WV_HIP(hipStreamWaitEvent(st, s->ev_fold[1 - sk], 0));
        WV_HIP(launch_finalize_multi(st, table_store(c), as<PrimeRec>(s->pr), as<Pair>(s->acc),
                                     as<uint64_t>(s->coefs), as<uint64_t>(s->lhsmod), as<FinReq>(ss.fin),
                                     (uint32_t)fins.size(), nres, s->nB, s->nE, as<wv_result>(ss.res),
                                     (const unsigned long long *)(scal + kScalErr)));
        WV_HIP(hipMemcpyAsync(ss.res_h, ss.res.ptr, (size_t)nres * sizeof(wv_result), hipMemcpyDeviceToHost, st));
    }
    WV_HIP(hipMemcpyAsync(ss.scal_h, scal, 8 * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    WV_HIP(hipEventRecord(ss.ev1, st));
    // the primes are handed out
    ss.id = ++s->launched;
    for (size_t k = 0; k < cand.size(); k++) cand[k]->next += give[k];
    ss.busy = true;
    *launched = true;
    return WV_OK;
}

// Waits for the step of buffer set `ss`; on success completes every request
// it finalized.
int complete_step(wv_server *s, StepSet &ss) {
    WV_HIP(hipEventSynchronize(ss.ev1));
    ss.busy = false;
    // device time: the union of the steps' intervals (consecutive steps on the
    // two streams overlap), measured from the reference event
    float a0 = 0.f, a1 = 0.f, b0 = 0.f, b1 = 0.f;
    (void)hipEventElapsedTime(&a0, s->ev_ref, ss.ev0);
    (void)hipEventElapsedTime(&a1, s->ev_ref, ss.ev1);
    (void)hipEventElapsedTime(&b0, s->ev_ref, ss.ev_sum0);
    (void)hipEventElapsedTime(&b1, s->ev_ref, ss.ev_sum);
    s->busy_s += std::max(0.0, a1 - std::max<double>(a0, s->busy_end_ms)) * 1e-3;
    s->busy_end_ms = std::max<double>(s->busy_end_ms, a1);
    s->sum_s += std::max(0.0, b1 - std::max<double>(b0, s->sum_end_ms)) * 1e-3;
    s->sum_end_ms = std::max<double>(s->sum_end_ms, b1);
    s->steps++;
    if (ss.scal_h[kScalErr]) return WV_EHIP;   // the term sums did not cover every chunk: discard the step
    if (s->fault_after >= 0 && (int64_t)s->steps > s->fault_after) {
        s->fault_after = -1;   // one forced failure: the step's work is discarded
        return WV_EHIP;
    }
    s->terms_done += ss.scal_h[kScalTerms];
    s->terms_done_b += ss.scal_h[kScalTermsB];
    s->fail_streak = 0;
    if (ss.finishing.empty()) return WV_OK;
    for (size_t k = 0; k < ss.finishing.size(); k++) {
        Request *r = ss.finishing[k];
        const wv_result *res = ss.res_h + ss.fin_out[k];
        bool bad = false;
        for (uint32_t i = 0; i < r->n; i++) bad |= res[i].flags == 0xFFFFFFFFu;
        if (bad) {
            // every prime of a request is valid (checked at submission, or
            // from the sieve): a rejected one means the admission went wrong
            fail_request(s, r, WV_EHIP);
            continue;
        }
        r->results.assign(res, res + r->n);
        pool_free(s, r->base, r->n);
        r->state = REQ_DONE;
        r->t_done = now_s();
        s->completed++;
        s->primes_done += r->n;
        s->lat_ms.push_back((r->t_done - r->t_submit) * 1e3);
    }
    std::vector<Request *> still;
    for (Request *r : s->active)
        if (r->state == REQ_ACTIVE) still.push_back(r);
    s->active.swap(still);
    ss.finishing.clear();
    return WV_OK;
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace

extern "C" {

int wv_server_create(wv_ctx *c, const wv_server_config *cfg, wv_server **out) {
    if (!c || !out) return WV_EINVAL;
    *out = nullptr;
    WV_TRY(check_device(c));
    wv_server *s = new (std::nothrow) wv_server();
    if (!s) return WV_ENOMEM;
    s->c = c;
    if (cfg && cfg->step_terms) s->step_terms = cfg->step_terms;
    s->tb = c->tb;
    s->te = c->te;
    s->nB = side_slots(c, c->tb);
    s->nE = side_slots(c, c->te);
    s->NS = s->nB + s->nE;
    // default pool: 65536 primes, fewer where the congruences have so many
    // sums that this would pass 2^30 slots (56 bytes of device state each)
    if (cfg && cfg->max_primes) s->pool = cfg->max_primes;
    else s->pool = (uint32_t)std::min<uint64_t>(s->pool, std::max<uint64_t>(1024, (1ull << 30) / s->NS));
    const size_t nseg = (size_t)s->pool * s->NS;
    if (nseg >= (1ull << 32)) {   // pool indices of the step tasks are 32-bit
        delete s;
        return WV_EINVAL;
    }
    int rc = WV_OK;
    if ((rc = ensure(c, s->pr, s->pool * sizeof(PrimeRec))) != WV_OK ||
        (rc = ensure(c, s->segs, nseg * sizeof(SegRec))) != WV_OK ||
        (rc = ensure(c, s->acc, nseg * sizeof(Pair))) != WV_OK ||
        (rc = ensure(c, s->terms, nseg * sizeof(uint64_t))) != WV_OK ||
        (rc = ensure(c, s->coefs, nseg * sizeof(uint64_t))) != WV_OK ||
        (rc = ensure(c, s->lhsmod, 2 * (size_t)s->pool * sizeof(uint64_t))) != WV_OK ||
        (rc = ensure(c, s->plist, s->pool * sizeof(uint64_t))) != WV_OK ||
        (rc = ensure(c, s->sdesc, kMaxBatchSegs * sizeof(SegDesc))) != WV_OK ||
        (rc = ensure(c, s->scount, kMaxBatchSegs * sizeof(uint32_t))) != WV_OK ||
        (rc = ensure(c, s->sbits, kMaxBatchSegs * kSegWords * sizeof(uint32_t))) != WV_OK ||
        (rc = ensure(c, s->soff, (kMaxBatchSegs + 1) * sizeof(uint64_t))) != WV_OK) {
        wv_server_destroy(s);
        return rc;
    }
    if (hipStreamCreateWithFlags(&s->own, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&s->ev_ref) != hipSuccess || hipEventRecord(s->ev_ref, c->stream) != hipSuccess)
        rc = WV_EHIP;
    for (int k = 0; k < 2 && rc == WV_OK; k++)
        if (hipEventCreateWithFlags(&s->ev_adm[k], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&s->ev_fold[k], hipEventDisableTiming) != hipSuccess)
            rc = WV_EHIP;
    for (int k = 0; k < 2 && rc == WV_OK; k++) {
        StepSet &ss = s->set[k];
        if ((rc = ensure(c, ss.scal, 8 * sizeof(uint64_t))) != WV_OK) break;
        if (hipHostMalloc((void **)&ss.scal_h, 8 * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess ||
            hipEventCreate(&ss.ev0) != hipSuccess || hipEventCreate(&ss.ev_sum0) != hipSuccess ||
            hipEventCreate(&ss.ev_sum) != hipSuccess || hipEventCreate(&ss.ev1) != hipSuccess)
            rc = WV_EHIP;
        else
            memset(ss.scal_h, 0, 8 * sizeof(uint64_t));
        Upload &u = s->up[k];
        if (rc == WV_OK && (hipHostMalloc((void **)&u.h, kUploadBytes, hipHostMallocDefault) != hipSuccess ||
                            hipEventCreate(&u.ev) != hipSuccess))
            rc = WV_EHIP;
        if (rc == WV_OK) u.cap = kUploadBytes;
    }
    if (rc != WV_OK) {
        wv_server_destroy(s);
        return rc;
    }
    s->free_ranges.push_back({0, s->pool});
    *out = s;
    return WV_OK;
}

int wv_server_inject_fault(wv_server *s, int after_steps) {
    if (!s) return WV_EINVAL;
    s->fault_after = after_steps < 0 ? -1 : (int64_t)(s->steps + after_steps);
    return WV_OK;
}

int wv_server_destroy(wv_server *s) {
    if (!s) return WV_OK;
    if (s->c) (void)hipStreamSynchronize(s->c->stream);
    if (s->own) (void)hipStreamSynchronize(s->own);
    DevBuf *bufs[] = {&s->pr, &s->segs, &s->acc, &s->terms, &s->coefs, &s->lhsmod, &s->plist,
                      &s->sdesc, &s->scount, &s->sbits, &s->soff};
    for (DevBuf *b : bufs)
        if (b->ptr) (void)hipFree(b->ptr);
    for (StepSet &ss : s->set) {
        DevBuf *sb[] = {&ss.spans, &ss.tasks, &ss.terms, &ss.cnt, &ss.off, &ss.tiles, &ss.target,
                        &ss.tpairs, &ss.partials, &ss.tails, &ss.hist, &ss.scal, &ss.fin, &ss.res};
        for (DevBuf *b : sb)
            if (b->ptr) (void)hipFree(b->ptr);
        void *hb[] = {ss.spans_h, ss.fin_h, ss.res_h, ss.scal_h};
        for (void *h : hb)
            if (h) (void)hipHostFree(h);
        hipEvent_t evs[] = {ss.ev0, ss.ev_sum0, ss.ev_sum, ss.ev1};
        for (hipEvent_t e : evs)
            if (e) (void)hipEventDestroy(e);
    }
    for (Upload &u : s->up) {
        if (u.h) (void)hipHostFree(u.h);
        if (u.ev) (void)hipEventDestroy(u.ev);
    }
    hipEvent_t sev[] = {s->ev_adm[0], s->ev_adm[1], s->ev_fold[0], s->ev_fold[1], s->ev_ref};
    for (hipEvent_t e : sev)
        if (e) (void)hipEventDestroy(e);
    if (s->own) (void)hipStreamDestroy(s->own);
    for (auto &kv : s->all) delete kv.second;
    delete s;
    return WV_OK;
}

int wv_server_submit_range(wv_server *s, uint64_t lo, uint64_t hi, uint64_t *id) {
    if (!s || !id || lo > hi) return WV_EINVAL;
    if (hi > WV_P_MAX) return WV_EDOMAIN;
    if (hi - (lo & ~1ull) > kMaxBatchSegs * kSegSpan) return WV_EINVAL;   // one batch of sieve segments
    // the prime count decides whether the request can ever fit in the pool
    const uint64_t n = count_primes_host(s->base_primes, s->base_limit, lo, hi);
    if (n > s->pool) return WV_EINVAL;
    Request *r = new (std::nothrow) Request();
    if (!r) return WV_ENOMEM;
    r->id = s->next_id++;
    r->is_range = true;
    r->lo = lo;
    r->hi = hi;
    r->n_primes = n;
    r->pmax = hi;
    r->t_submit = now_s();
    if (!s->submitted) s->t_first = r->t_submit;
    s->submitted++;
    s->all[r->id] = r;
    s->pending.push_back(r);
    *id = r->id;
    return WV_OK;
}

int wv_server_submit_primes(wv_server *s, const uint64_t *primes, size_t n, uint64_t *id) {
    if (!s || !id || (n && !primes)) return WV_EINVAL;
    if (n > s->pool) return WV_EINVAL;
    uint64_t pmax = 0;
    for (size_t i = 0; i < n; i++) {
        if (primes[i] < 5 || primes[i] >= WV_P_MAX) return WV_EDOMAIN;
        if (!is_prime_u64(primes[i])) return WV_ENOTPRIME;
        pmax = std::max(pmax, primes[i]);
    }
    Request *r = new (std::nothrow) Request();
    if (!r) return WV_ENOMEM;
    r->id = s->next_id++;
    r->primes.assign(primes, primes + n);
    r->n_primes = n;
    r->pmax = pmax;
    r->t_submit = now_s();
    if (!s->submitted) s->t_first = r->t_submit;
    s->submitted++;
    s->all[r->id] = r;
    s->pending.push_back(r);
    *id = r->id;
    return WV_OK;
}

// Sums planned into the pool per call at most, so that admitting a burst of
// large requests does not hold back the next step.
constexpr size_t kAdmitSums = 1u << 24;
// A request pending longer than this is admitted before smaller ones, in
// arrival order, so that a stream of small requests cannot starve it.
constexpr double kAdmitAgeS = 2.0;
// After this many consecutive failed steps the active requests end with the
// step's error instead of restarting again.
constexpr int kMaxFailedSteps = 3;

int wv_server_step(wv_server *s, uint32_t *n_active, uint32_t *n_pending) {
    if (!s) return WV_EINVAL;
    WV_TRY(check_device(s->c));
    // this call's upload staging: the copies its previous use enqueued have
    // run once the step launched after them completed (a call ago)
    Upload &u = s->up[s->up_cur];
    if (u.pending) WV_HIP(hipEventSynchronize(u.ev));
    u.pending = false;
    u.used = 0;
    // admit requests pending for kAdmitAgeS or more in arrival order, then the
    // smallest first (by number of primes), arrival order among equals,
    // within the per-call budget of sums; a request that does not fit in the
    // pool yet does not block those behind it
    const double t_old = now_s() - kAdmitAgeS;
    std::stable_sort(s->pending.begin(), s->pending.end(), [&](const Request *a, const Request *b) {
        const bool oa = a->t_submit <= t_old, ob = b->t_submit <= t_old;
        if (oa != ob) return oa;
        if (oa) return a->t_submit < b->t_submit;
        return a->n_primes < b->n_primes;
    });
    size_t admitted_sums = 0;
    std::deque<Request *> waiting;
    const hipStream_t ast = stream_of(s, s->next);   // the stream of the step launched next
    bool enqueued = false;
    // admissions share the sieve buffers: the other stream's come first
    if (!s->pending.empty() && s->adm_recorded[1 - s->next])
        WV_HIP(hipStreamWaitEvent(ast, s->ev_adm[1 - s->next], 0));
    while (!s->pending.empty()) {
        Request *r = s->pending.front();
        s->pending.pop_front();
        if (admitted_sums >= kAdmitSums) {
            waiting.push_back(r);
            continue;
        }
        bool ok = false;
        const int rc = admit(s, r, &ok, ast);
        if (rc != WV_OK) {
            // the request ends with this error (wv_server_result returns it)
            fail_request(s, r, rc);
            continue;
        }
        if (!ok) {
            waiting.push_back(r);
        } else {
            admitted_sums += (size_t)r->n * s->NS;
            enqueued |= r->n > 0;
        }
    }
    s->pending.swap(waiting);
    if (u.used) {
        WV_HIP(hipEventRecord(u.ev, ast));
        u.pending = true;
        s->up_cur ^= 1;
    }
    if (enqueued) {
        WV_HIP(hipEventRecord(s->ev_adm[s->next], ast));
        s->adm_pending[s->next] = true;
        s->adm_recorded[s->next] = true;
    }
    // launch the next step, then wait for the older step in flight (or, when
    // nothing new was launched, for the one still in flight)
    StepSet &nx = s->set[s->next];
    StepSet &older = s->set[1 - s->next];
    int rc = WV_OK;
    bool launched = false;
    if (!nx.busy) rc = launch_step(s, s->next, &launched);
    if (rc == WV_OK) {
        if (launched) s->next = 1 - s->next;
        if (older.busy) rc = complete_step(s, older);
        else if (!launched && nx.busy) rc = complete_step(s, nx);
    }
    if (rc != WV_OK) {
        (void)hipGetLastError();
        // every step in flight is discarded: the active requests restart from
        // their plans, or end with the error after repeated failures
        (void)hipStreamSynchronize(s->c->stream);
        (void)hipStreamSynchronize(s->own);
        for (StepSet &ss : s->set) {
            ss.busy = false;
            ss.finishing.clear();
        }
        if (++s->fail_streak >= kMaxFailedSteps) {
            for (Request *r : s->active) fail_request(s, r, rc);
            s->active.clear();
            s->fail_streak = 0;
        } else if (readmit_all(s) != WV_OK) {
            for (Request *r : s->active) fail_request(s, r, rc);
            s->active.clear();
        }
    }
    if (n_active) *n_active = (uint32_t)s->active.size();
    if (n_pending) *n_pending = (uint32_t)s->pending.size();
    return rc;
}

int wv_server_result(wv_server *s, uint64_t id, wv_result *out, size_t cap, size_t *n_out, double *latency_ms) {
    if (!s || !n_out) return WV_EINVAL;
    auto it = s->all.find(id);
    if (it == s->all.end()) return WV_EINVAL;
    Request *r = it->second;
    if (r->state != REQ_DONE) return WV_EBUSY;
    *n_out = r->results.size();
    if (latency_ms) *latency_ms = (r->t_done - r->t_submit) * 1e3;
    if (r->status != WV_OK) {
        // the request ended with an error: report it once, then forget it
        const int st = r->status;
        s->all.erase(it);
        delete r;
        return st;
    }
    if (r->results.size() > cap) return WV_ETRUNC;
    if (!r->results.empty()) {
        if (!out) return WV_EINVAL;
        memcpy(out, r->results.data(), r->results.size() * sizeof(wv_result));
    }
    s->all.erase(it);
    delete r;
    return WV_OK;
}

int wv_server_get_stats(const wv_server *s, wv_server_stats *out) {
    if (!s || !out) return WV_EINVAL;
    memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->failed = s->failed;
    out->pending = s->pending.size();
    out->active = s->active.size();
    out->primes_done = s->primes_done;
    out->terms_done = s->terms_done;
    out->terms_done_b = s->terms_done_b;
    out->sum_s = s->sum_s;
    out->block_k_b = (uint32_t)sum_variant_kb(s->c->variant);
    out->block_k_e = (uint32_t)sum_variant_ke(s->c->variant);
    out->steps = s->steps;
    out->readmits = s->readmits;
    out->p50_ms = percentile(s->lat_ms, 0.50);
    out->p99_ms = percentile(s->lat_ms, 0.99);
    double sum = 0, mx = 0;
    for (double v : s->lat_ms) {
        sum += v;
        mx = std::max(mx, v);
    }
    out->mean_ms = s->lat_ms.empty() ? 0.0 : sum / s->lat_ms.size();
    out->max_ms = mx;
    out->busy_s = s->busy_s;
    out->wall_s = s->submitted ? now_s() - s->t_first : 0.0;
    return WV_OK;
}

}  // extern "C"
