// wv_server.hip -- request server with continuous batching at chunk
// granularity (the serving loop of the residue search).
//
// Requests (a prime list, or every prime of an interval) are admitted into a
// device pool of prime slots when a contiguous range of slots is free: their
// primes are planned into the pool (PrimeRec, one SegRec per (prime, sum)) and
// each sum gets an accumulator pair (c0, c1) = (1, 0) on the device.  Every
// step then cuts a budget of terms into tasks -- contiguous ranges of one sum
// -- shared fairly among the active requests, runs them through the same
// term-sum and reduction kernels as a batch, and folds each task's pair into
// its sum's accumulator with eqnCombinePairs (Section 3).  A request whose
// sums are all complete is finalized (Sections 3 and 5 congruences), its
// results copied out and its slots freed.  New requests join at the next
// step, so short requests overtake long ones instead of queueing behind them.
//
// Steps are pipelined two deep: a call of wv_server_step plans and launches
// the next step (the host advances the requests' cursors when it plans, so the
// plan never waits for the device) and then waits for the step launched by the
// previous call.  The host's work between steps -- planning, the caller's own
// loop -- overlaps the device's work.  Admission (sieve, plan into the pool)
// and finalization run on a second stream: they touch pool slots that no step
// in flight uses.
//
// Because the pair product is associative and commutative and all arithmetic
// is exact, a request's residues do not depend on how its work was cut into
// tasks or interleaved with other requests.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

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
    uint32_t n = 0;            // primes in the pool
    uint32_t base = 0;         // first pool slot
    std::vector<uint64_t> seg_lo, seg_len, cursor;   // cursor: terms handed to launched steps
    size_t first_open = 0;     // first sum with terms not yet handed out
    uint64_t remaining = 0;    // terms not yet handed to a launched step
    uint64_t last_step = 0;    // the last launched step holding terms of this request (0: none)
    std::vector<wv_result> results;
};

struct Task {
    Request *r;
    size_t k;        // sum index within the request
    uint64_t t;      // terms
};

// One step's device buffers, the host staging its copies read from (kept
// until the step completes), its events and its error word.
struct StepSet {
    DevBuf tasks, target, toff, tpairs, partials, tails, scal;
    std::vector<SegRec> recs;
    std::vector<uint32_t> tgt, tails_h;
    std::vector<uint64_t> off;
    uint64_t layout[5] = {};
    uint64_t *err_host = nullptr;   // pinned: the step's term-sum error word
    hipEvent_t ev0 = nullptr, ev_sum = nullptr, ev1 = nullptr;
    bool busy = false;              // launched and not yet completed
    uint64_t id = 0;                // step number (1, 2, ...)
    uint64_t terms = 0, terms_b = 0;
};

}  // namespace

struct wv_server {
    wv_ctx *c = nullptr;
    uint64_t step_terms = 1ull << 38;
    uint32_t pool = 1u << 16;
    int tb = 0, te = 0;        // congruences fixed at creation (the pool layout depends on them)
    int nB = 0, nE = 0, NS = 0;
    DevBuf pr, segs, acc, terms, tmp, res, coefs, lhsmod;
    StepSet set[2];
    int next = 0;              // the set the next launch uses
    uint64_t launched = 0;     // steps launched
    hipStream_t aux = nullptr; // admission and finalization
    std::vector<std::pair<uint32_t, uint32_t>> free_ranges;   // (first slot, count), sorted
    std::deque<Request *> pending;
    std::vector<Request *> active;
    std::map<uint64_t, Request *> all;
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

// Finalize a request whose steps have all completed: residues from its sums'
// accumulators (on the auxiliary stream; no step in flight uses its slots),
// copied out; its slots are freed.
int finish_request(wv_server *s, Request *r) {
    wv_ctx *c = s->c;
    if (r->n) {
        WV_HIP(launch_finalize(s->aux, table_store(c), as<PrimeRec>(s->pr) + r->base,
                               as<Pair>(s->acc) + (size_t)r->base * s->NS,
                               as<uint64_t>(s->coefs) + (size_t)r->base * s->NS,
                               as<uint64_t>(s->lhsmod) + 2 * (size_t)r->base, r->n, s->nB, s->nE,
                               as<wv_result>(s->res), nullptr));
        r->results.resize(r->n);
        WV_HIP(hipMemcpyAsync(r->results.data(), s->res.ptr, r->n * sizeof(wv_result), hipMemcpyDeviceToHost,
                              s->aux));
        WV_HIP(hipStreamSynchronize(s->aux));
    }
    pool_free(s, r->base, r->n);
    r->state = REQ_DONE;
    r->t_done = now_s();
    s->completed++;
    s->primes_done += r->n;
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

// Plans the n primes at d_primes into the pool slots [r->base, r->base + n)
// and reads the per-sum records back (auxiliary stream).  The caller frees the
// slots on error.
int plan_request(wv_server *s, Request *r, const uint64_t *d_primes, uint32_t n) {
    wv_ctx *c = s->c;
    const size_t first = (size_t)r->base * s->NS, nseg = (size_t)n * s->NS;
    WV_HIP(launch_plan(s->aux, d_primes, n, s->tb, s->te, table_fallback(c, s->tb), table_fallback(c, s->te), s->nB,
                       s->nE, table_store(c), as<PrimeRec>(s->pr) + r->base, as<SegRec>(s->segs) + first,
                       as<uint64_t>(s->terms) + first, as<uint64_t>(s->coefs) + first,
                       as<uint64_t>(s->lhsmod) + 2 * (size_t)r->base, r->base));
    WV_HIP(launch_fill_pairs(s->aux, as<Pair>(s->acc) + first, nseg, 1, 0));
    std::vector<SegRec> recs(nseg);
    WV_HIP(hipMemcpyAsync(recs.data(), as<SegRec>(s->segs) + first, nseg * sizeof(SegRec), hipMemcpyDeviceToHost,
                          s->aux));
    WV_HIP(hipStreamSynchronize(s->aux));
    r->seg_lo.resize(nseg);
    r->seg_len.resize(nseg);
    r->cursor.assign(nseg, 0);
    r->remaining = 0;
    for (size_t k = 0; k < nseg; k++) {
        r->seg_lo[k] = recs[k].lo;
        r->seg_len[k] = recs[k].len;
        r->remaining += recs[k].len;
    }
    r->first_open = 0;
    r->last_step = 0;
    return WV_OK;
}

// Plans a pending request into the pool.  Returns WV_OK with *admitted false
// when there is no room yet; an error return leaves no pool slot taken.
int admit(wv_server *s, Request *r, bool *admitted) {
    wv_ctx *c = s->c;
    *admitted = false;
    // submission checked that the request fits in an empty pool
    const uint64_t n = r->n_primes;
    if (n > s->pool) return WV_EINVAL;
    uint32_t base = 0;
    if (n > 0 && !pool_alloc(s, (uint32_t)n, &base)) return WV_OK;
    r->base = base;
    r->n = (uint32_t)n;
    int rc = WV_OK;
    const uint64_t *d_primes = nullptr;
    if (n > 0 && r->is_range) {
        std::vector<SegDesc> d;
        window_descs(r->lo, r->hi, d);
        std::vector<uint32_t> counts(d.size());
        uint64_t got = 0;
        rc = sieve_count(c, d.data(), d.size(), true, counts.data(), s->aux);
        if (rc == WV_OK) rc = compact(c, d.data(), d.size(), counts.data(), &got, s->aux);
        if (rc == WV_OK && got != n) rc = WV_EHIP;   // the sieve is deterministic
        d_primes = as<uint64_t>(c->primes);
    } else if (n > 0) {
        rc = ensure(c, s->tmp, n * sizeof(uint64_t));
        if (rc == WV_OK && hipMemcpyAsync(s->tmp.ptr, r->primes.data(), n * sizeof(uint64_t), hipMemcpyHostToDevice,
                                          s->aux) != hipSuccess)
            rc = WV_EHIP;
        d_primes = as<uint64_t>(s->tmp);
    }
    if (rc == WV_OK && n > 0) rc = plan_request(s, r, d_primes, (uint32_t)n);
    if (rc != WV_OK) {
        (void)hipGetLastError();
        pool_free(s, r->base, r->n);
        r->n = 0;
        return rc;
    }
    r->t_admit = now_s();
    *admitted = true;
    if (n == 0 || r->remaining == 0) return finish_request(s, r);
    r->state = REQ_ACTIVE;
    s->active.push_back(r);
    return WV_OK;
}

// Restart every active request from scratch (after a failed step; no step is
// in flight).
int readmit_all(wv_server *s) {
    for (Request *r : s->active) {
        std::fill(r->cursor.begin(), r->cursor.end(), 0);
        r->first_open = 0;
        r->remaining = 0;
        r->last_step = 0;
        for (uint64_t l : r->seg_len) r->remaining += l;
        WV_HIP(launch_fill_pairs(s->c->stream, as<Pair>(s->acc) + (size_t)r->base * s->NS, (size_t)r->n * s->NS,
                                 1, 0));
        s->readmits++;
    }
    WV_HIP(hipStreamSynchronize(s->c->stream));
    return WV_OK;
}

// Plans the next step on the host -- a fair share of the budget per active
// request with terms not yet handed out, cut into tasks of whole chunks -- and
// launches it on the context stream with buffer set `ss`.  The requests'
// cursors advance now.  *launched is false when no request has terms left.
int launch_step(wv_server *s, StepSet &ss, bool *launched) {
    wv_ctx *c = s->c;
    *launched = false;
    const uint64_t C = c->chunk_cfg   ? c->chunk_cfg
                       : c->chunk_auto ? c->chunk_auto
                                       : (adaptive_chunk(s->step_terms, sum_lanes(c)) + 63) & ~63ull;
    // fair share of the step budget, leftovers to whoever still has work
    std::vector<uint64_t> allow(s->active.size(), 0);
    uint64_t budget = s->step_terms;
    for (int pass = 0; pass < 2 && budget > 0; pass++) {
        size_t want = 0;
        for (size_t i = 0; i < s->active.size(); i++)
            if (s->active[i]->remaining > allow[i]) want++;
        if (!want) break;
        const uint64_t share = std::max<uint64_t>(C, budget / want);
        for (size_t i = 0; i < s->active.size() && budget > 0; i++) {
            const uint64_t left = s->active[i]->remaining - allow[i];
            if (!left) continue;
            const uint64_t g = std::min(std::min(left, share), budget);
            allow[i] += g;
            budget -= g;
        }
    }
    std::vector<Task> tasks;
    for (size_t i = 0; i < s->active.size(); i++) {
        Request *r = s->active[i];
        uint64_t a = allow[i];
        for (size_t k = r->first_open; k < r->seg_len.size() && a > 0; k++) {
            const uint64_t left = r->seg_len[k] - r->cursor[k];
            if (!left) continue;
            uint64_t t = std::min(left, ((a + C - 1) / C) * C);
            tasks.push_back(Task{r, k, t});
            a -= std::min(a, t);
        }
    }
    if (tasks.empty()) return WV_OK;
    const size_t nt = tasks.size();
    ss.recs.resize(nt);
    ss.tgt.resize(nt);
    ss.off.assign(nt + 1, 0);
    uint64_t terms = 0, terms_b = 0;
    for (size_t j = 0; j < nt; j++) {
        const Task &t = tasks[j];
        const size_t k = t.k;
        // slot k of the request: Bernoulli slots (i*nB + j) first, then Euler
        const bool bern = k < (size_t)t.r->n * s->nB;
        const uint32_t prime = bern ? (uint32_t)(k / s->nB) : (uint32_t)((k - (size_t)t.r->n * s->nB) / s->nE);
        ss.recs[j] = SegRec{t.r->seg_lo[k] + t.r->cursor[k], t.t, t.r->base + prime, bern ? 3u : 2u};
        ss.tgt[j] = (uint32_t)((size_t)t.r->base * s->NS + k);
        ss.off[j + 1] = ss.off[j] + t.t / C;   // full chunks
        terms += t.t;
        if (bern) terms_b += t.t;
    }
    // tail chunks (tasks whose length C does not divide) by length class,
    // longest first, each class's s^-3 tasks before its s^-2 ones (counting
    // sort, as the batch plan does on the device)
    std::vector<uint32_t> cls(nt, kTailClasses);
    uint64_t first[kTailClasses + 1] = {};
    for (size_t j = 0; j < nt; j++)
        if (const uint64_t rem = tasks[j].t % C) first[(cls[j] = tail_class(rem, C, ss.recs[j].deg)) + 1]++;
    for (int b = 0; b < kTailClasses; b++) first[b + 1] += first[b];
    ss.tails_h.resize(first[kTailClasses]);
    for (size_t j = 0; j < nt; j++)
        if (cls[j] < (uint32_t)kTailClasses) ss.tails_h[first[cls[j]]++] = (uint32_t)j;
    const uint64_t chunks = ss.off[nt];
    WV_TRY(ensure(c, ss.tasks, nt * sizeof(SegRec)));
    WV_TRY(ensure(c, ss.target, nt * sizeof(uint32_t)));
    WV_TRY(ensure(c, ss.toff, (nt + 1) * sizeof(uint64_t)));
    WV_TRY(ensure(c, ss.tpairs, nt * sizeof(Pair)));
    WV_TRY(ensure(c, ss.partials, std::max<uint64_t>(chunks, 1) * sizeof(Pair)));
    WV_TRY(ensure(c, ss.tails, std::max<size_t>(ss.tails_h.size(), 1) * sizeof(uint32_t)));
    hipStream_t st = c->stream;
    WV_HIP(hipMemcpyAsync(ss.tasks.ptr, ss.recs.data(), nt * sizeof(SegRec), hipMemcpyHostToDevice, st));
    WV_HIP(hipMemcpyAsync(ss.target.ptr, ss.tgt.data(), nt * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    WV_HIP(hipMemcpyAsync(ss.toff.ptr, ss.off.data(), (nt + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    if (!ss.tails_h.empty())
        WV_HIP(hipMemcpyAsync(ss.tails.ptr, ss.tails_h.data(), ss.tails_h.size() * sizeof(uint32_t),
                              hipMemcpyHostToDevice, st));
    // chunk layout, the chunk counter, the term-sum error word
    ss.layout[0] = C;
    ss.layout[1] = chunks;
    ss.layout[2] = ss.tails_h.size();
    ss.layout[3] = 0;
    ss.layout[4] = 0;
    uint64_t *scal = as<uint64_t>(ss.scal);
    WV_HIP(hipMemcpyAsync(scal, ss.layout, sizeof(ss.layout), hipMemcpyHostToDevice, st));
    WV_HIP(hipEventRecord(ss.ev0, st));
    const int v = c->variant;
    WV_HIP(launch_sum(st, v, (unsigned)c->sum_blocks[v], as<SegRec>(ss.tasks), as<uint64_t>(ss.toff), (uint32_t)nt,
                      as<PrimeRec>(s->pr), scal, as<uint32_t>(ss.tails), as<Pair>(ss.partials), as<Pair>(ss.tpairs),
                      (unsigned long long *)(scal + 3), UINT64_MAX, (unsigned long long *)(scal + 4)));
    WV_HIP(hipEventRecord(ss.ev_sum, st));
    WV_HIP(launch_reduce(st, as<SegRec>(ss.tasks), as<uint64_t>(ss.toff), (uint32_t)nt, as<PrimeRec>(s->pr),
                         as<Pair>(ss.partials), scal, as<Pair>(ss.tpairs)));
    WV_HIP(launch_fold(st, as<SegRec>(ss.tasks), as<uint32_t>(ss.target), as<Pair>(ss.tpairs), (uint32_t)nt,
                       as<PrimeRec>(s->pr), as<Pair>(s->acc)));
    WV_HIP(hipMemcpyAsync(ss.err_host, scal + 4, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    WV_HIP(hipEventRecord(ss.ev1, st));
    // the terms are handed out: advance the cursors
    ss.id = ++s->launched;
    for (const Task &t : tasks) {
        t.r->cursor[t.k] += t.t;
        t.r->remaining -= t.t;
        t.r->last_step = ss.id;
    }
    for (Request *r : s->active)
        while (r->first_open < r->seg_len.size() && r->cursor[r->first_open] == r->seg_len[r->first_open])
            r->first_open++;
    ss.terms = terms;
    ss.terms_b = terms_b;
    ss.busy = true;
    *launched = true;
    return WV_OK;
}

// Waits for the step of buffer set `ss`; on success finalizes every request
// whose last step it was.
int complete_step(wv_server *s, StepSet &ss) {
    WV_HIP(hipEventSynchronize(ss.ev1));
    ss.busy = false;
    float ms = 0.f, ms_sum = 0.f;
    (void)hipEventElapsedTime(&ms, ss.ev0, ss.ev1);
    (void)hipEventElapsedTime(&ms_sum, ss.ev0, ss.ev_sum);
    s->busy_s += ms * 1e-3;
    s->sum_s += ms_sum * 1e-3;
    s->steps++;
    if (*ss.err_host) return WV_EHIP;   // the term sums did not cover every chunk: discard the step
    if (s->fault_after >= 0 && (int64_t)s->steps > s->fault_after) {
        s->fault_after = -1;   // one forced failure: the step's work is discarded
        return WV_EHIP;
    }
    s->terms_done += ss.terms;
    s->terms_done_b += ss.terms_b;
    s->fail_streak = 0;
    // finished requests leave the active list one by one, so that an error in
    // a later finalize leaves only unfinished requests active
    std::vector<Request *> still;
    int rc = WV_OK;
    size_t i = 0;
    for (; i < s->active.size() && rc == WV_OK; i++) {
        Request *r = s->active[i];
        if (r->remaining == 0 && r->last_step <= ss.id) {
            rc = finish_request(s, r);
            if (rc != WV_OK) still.push_back(r);   // not finished: its sums restart with the others
        } else {
            still.push_back(r);
        }
    }
    for (; i < s->active.size(); i++) still.push_back(s->active[i]);
    s->active.swap(still);
    return rc;
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
    if (cfg && cfg->max_primes) s->pool = cfg->max_primes;
    s->tb = c->tb;
    s->te = c->te;
    s->nB = side_slots(c, c->tb);
    s->nE = side_slots(c, c->te);
    s->NS = s->nB + s->nE;
    const size_t nseg = (size_t)s->pool * s->NS;
    int rc = WV_OK;
    if ((rc = ensure(c, s->pr, s->pool * sizeof(PrimeRec))) != WV_OK ||
        (rc = ensure(c, s->segs, nseg * sizeof(SegRec))) != WV_OK ||
        (rc = ensure(c, s->acc, nseg * sizeof(Pair))) != WV_OK ||
        (rc = ensure(c, s->terms, nseg * sizeof(uint64_t))) != WV_OK ||
        (rc = ensure(c, s->coefs, nseg * sizeof(uint64_t))) != WV_OK ||
        (rc = ensure(c, s->lhsmod, 2 * (size_t)s->pool * sizeof(uint64_t))) != WV_OK ||
        (rc = ensure(c, s->res, s->pool * sizeof(wv_result))) != WV_OK) {
        wv_server_destroy(s);
        return rc;
    }
    if (hipStreamCreateWithFlags(&s->aux, hipStreamNonBlocking) != hipSuccess) rc = WV_EHIP;
    for (int k = 0; k < 2 && rc == WV_OK; k++) {
        StepSet &ss = s->set[k];
        if ((rc = ensure(c, ss.scal, 8 * sizeof(uint64_t))) != WV_OK) break;
        if (hipHostMalloc((void **)&ss.err_host, sizeof(uint64_t), hipHostMallocDefault) != hipSuccess ||
            hipEventCreate(&ss.ev0) != hipSuccess || hipEventCreate(&ss.ev_sum) != hipSuccess ||
            hipEventCreate(&ss.ev1) != hipSuccess)
            rc = WV_EHIP;
        else
            *ss.err_host = 0;
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
    if (s->aux) (void)hipStreamSynchronize(s->aux);
    DevBuf *bufs[] = {&s->pr, &s->segs, &s->acc, &s->terms, &s->tmp, &s->res, &s->coefs, &s->lhsmod};
    for (DevBuf *b : bufs)
        if (b->ptr) (void)hipFree(b->ptr);
    for (StepSet &ss : s->set) {
        DevBuf *sb[] = {&ss.tasks, &ss.target, &ss.toff, &ss.tpairs, &ss.partials, &ss.tails, &ss.scal};
        for (DevBuf *b : sb)
            if (b->ptr) (void)hipFree(b->ptr);
        if (ss.err_host) (void)hipHostFree(ss.err_host);
        hipEvent_t evs[] = {ss.ev0, ss.ev_sum, ss.ev1};
        for (hipEvent_t e : evs)
            if (e) (void)hipEventDestroy(e);
    }
    if (s->aux) (void)hipStreamDestroy(s->aux);
    for (auto &kv : s->all) delete kv.second;
    delete s;
    return WV_OK;
}

int wv_server_submit_range(wv_server *s, uint64_t lo, uint64_t hi, uint64_t *id) {
    if (!s || !id || lo > hi) return WV_EINVAL;
    if (hi > WV_P_MAX) return WV_EDOMAIN;
    if (hi - (lo & ~1ull) > kMaxBatchSegs * kSegSpan) return WV_EINVAL;   // one batch of sieve segments
    WV_TRY(check_device(s->c));
    // the prime count decides whether the request can ever fit in the pool
    std::vector<SegDesc> d;
    window_descs(lo, hi, d);
    std::vector<uint32_t> counts(d.size());
    if (!d.empty()) WV_TRY(sieve_count(s->c, d.data(), d.size(), false, counts.data(), s->aux));
    uint64_t n = 0;
    for (uint32_t k : counts) n += k;
    if (n > s->pool) return WV_EINVAL;
    Request *r = new (std::nothrow) Request();
    if (!r) return WV_ENOMEM;
    r->id = s->next_id++;
    r->is_range = true;
    r->lo = lo;
    r->hi = hi;
    r->n_primes = n;
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
    for (size_t i = 0; i < n; i++) {
        if (primes[i] < 5 || primes[i] >= WV_P_MAX) return WV_EDOMAIN;
        if (!is_prime_u64(primes[i])) return WV_ENOTPRIME;
    }
    Request *r = new (std::nothrow) Request();
    if (!r) return WV_ENOMEM;
    r->id = s->next_id++;
    r->primes.assign(primes, primes + n);
    r->n_primes = n;
    r->t_submit = now_s();
    if (!s->submitted) s->t_first = r->t_submit;
    s->submitted++;
    s->all[r->id] = r;
    s->pending.push_back(r);
    *id = r->id;
    return WV_OK;
}

// Sums planned into the pool per step at most (planning copies each sum's
// record to the host), so that admitting a burst of large requests does not
// hold back the next step.
constexpr size_t kAdmitSums = 1u << 22;
// A request pending longer than this is admitted before smaller ones, in
// arrival order, so that a stream of small requests cannot starve it.
constexpr double kAdmitAgeS = 2.0;
// After this many consecutive failed steps the active requests end with the
// step's error instead of restarting again.
constexpr int kMaxFailedSteps = 3;

int wv_server_step(wv_server *s, uint32_t *n_active, uint32_t *n_pending) {
    if (!s) return WV_EINVAL;
    WV_TRY(check_device(s->c));
    // admit requests pending for kAdmitAgeS or more in arrival order, then the
    // smallest first (by number of primes), arrival order among equals,
    // within the per-step budget of sums; a request that does not fit in the
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
    while (!s->pending.empty()) {
        Request *r = s->pending.front();
        s->pending.pop_front();
        if (admitted_sums >= kAdmitSums) {
            waiting.push_back(r);
            continue;
        }
        bool ok = false;
        const int rc = admit(s, r, &ok);
        if (rc != WV_OK) {
            // the request ends with this error (wv_server_result returns it)
            fail_request(s, r, rc);
            continue;
        }
        if (!ok) waiting.push_back(r);
        else admitted_sums += (size_t)r->n * s->NS;
    }
    s->pending.swap(waiting);
    // launch the next step, then wait for the older step in flight (or, when
    // nothing new was launched, for the one still in flight)
    StepSet &nx = s->set[s->next];
    StepSet &older = s->set[1 - s->next];
    int rc = WV_OK;
    bool launched = false;
    if (!nx.busy) rc = launch_step(s, nx, &launched);
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
        s->set[0].busy = s->set[1].busy = false;
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
