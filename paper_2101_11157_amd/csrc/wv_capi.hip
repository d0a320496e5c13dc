// wv_capi.hip -- context, pipeline orchestration and the C ABI of
// libwvprime.so.  Every computational step runs in the kernels of
// wv_kernels.hip; this file sizes buffers, orders launches on the context's
// stream, and moves inputs and results across the boundary.
//
// Method: Booker, Hathi, Mossinghoff, Trudgian, "Wolstenholme and Vandiver
// primes" (arXiv:2101.11157) -- see wv_kernels.hip for the step-by-step map.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "wv_ctx.hpp"

using namespace wv;

// ==========================================================================
// helpers
// ==========================================================================

namespace wv {

int ensure(wv_ctx *c, DevBuf &b, size_t bytes) {
    if (b.cap >= bytes && b.ptr) return WV_OK;
    const size_t old = b.cap;
    if (b.ptr) {
        WV_HIP(hipFree(b.ptr));
        b.ptr = nullptr;
        b.cap = 0;
    }
    const size_t need = std::max(bytes, (size_t)256);
    // a buffer that grows again gets half as much again (at most twice the
    // request), so that calls of slowly growing sizes do not reallocate each time
    size_t want = old ? std::max(need, std::min(old + old / 2, 2 * need)) : need;
    want = (want + 65535) & ~(size_t)65535;
    if (hipMalloc(&b.ptr, want) != hipSuccess) {
        (void)hipGetLastError();
        b.ptr = nullptr;
        want = need;
        WV_HIP(hipMalloc(&b.ptr, want));
    }
    b.cap = want;
    c->gen++;   // captured graphs hold the old address
    return WV_OK;
}

static uint64_t mulmod_h(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((unsigned __int128)a * b % m); }

static uint64_t powmod_h(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod_h(r, a, m);
        a = mulmod_h(a, a, m);
        e >>= 1;
    }
    return r;
}

// Deterministic Miller-Rabin for n < 2^64 (first twelve prime bases).
bool is_prime_u64(uint64_t n) {
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return false;
    for (uint64_t b : bases) {
        if (n == b) return true;
        if (n % b == 0) return false;
    }
    uint64_t d = n - 1;
    int s = 0;
    while (!(d & 1)) {
        d >>= 1;
        s++;
    }
    for (uint64_t a : bases) {
        uint64_t x = powmod_h(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s; r++) {
            x = mulmod_h(x, x, n);
            if (x == n - 1) {
                comp = false;
                break;
            }
        }
        if (comp) return false;
    }
    return true;
}

static float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
    return ms;
}

int check_device(wv_ctx *c) {
    WV_HIP(hipSetDevice(c->device));
    return WV_OK;
}

// ==========================================================================
// one batch of primes on the device: plan -> sums -> reduce -> finalize
// ==========================================================================

int batch_shape(const wv_ctx *c, uint32_t n, uint64_t pmax, BatchShape *sh) {
    sh->tb = batch_table(c, c->tb, pmax);
    sh->te = batch_table(c, c->te, pmax);
    sh->n = n;
    sh->nB = side_slots(c, sh->tb);
    sh->nE = side_slots(c, sh->te);
    sh->nseg = (uint64_t)n * (sh->nB + sh->nE);
    // partial pairs: the plan picks chunk >= total_terms / (cap - nseg), so
    // cap > nseg always; with room for total_terms / chunk_cfg + nseg chunks
    // the configured chunk size is kept.  total_terms <= n (pmax cost + sums).
    const uint64_t chunk_cfg = c->chunk_cfg ? c->chunk_cfg : c->chunk_auto;
    const double cost = side_cost(c, sh->tb) + side_cost(c, sh->te);
    const double t_max = (double)n * ((double)pmax * cost + sh->nB + sh->nE);
    // the adaptive chunk grows with T, so T / chunk is largest at the bound
    const double chunk = chunk_cfg ? (double)chunk_cfg
                                   : (double)adaptive_chunk((uint64_t)std::min(t_max, 1.8e19), sum_lanes(c));
    const double want = t_max / chunk + 2.0 * sh->nseg;
    sh->cap = (uint64_t)std::min<double>(std::max<double>(want, (double)kMinChunks), (double)kMaxChunks);
    sh->cap = std::max<uint64_t>(sh->cap, 2 * sh->nseg);
    return WV_OK;
}

int prepare(wv_ctx *c, const BatchShape &sh) {
    const uint64_t n = sh.n, nseg = sh.nseg;
    WV_TRY(ensure(c, c->pr, n * sizeof(PrimeRec)));
    WV_TRY(ensure(c, c->segs, nseg * sizeof(SegRec)));
    WV_TRY(ensure(c, c->terms, nseg * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->cnt, nseg * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->off, (nseg + 1) * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->tiles, ((nseg + kScanTile - 1) / kScanTile + 1) * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->scal, 8 * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->partials, sh.cap * sizeof(Pair)));
    WV_TRY(ensure(c, c->seg_pairs, nseg * sizeof(Pair)));
    WV_TRY(ensure(c, c->coefs, nseg * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->lhsmod, 2 * n * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->tails, nseg * sizeof(uint32_t)));
    WV_TRY(ensure(c, c->tail_hist, 2 * kTailClasses * sizeof(uint64_t)));
    return WV_OK;
}

BatchBufs ctx_bufs(wv_ctx *c) {
    BatchBufs b;
    b.pr = as<PrimeRec>(c->pr);
    b.segs = as<SegRec>(c->segs);
    b.terms = as<uint64_t>(c->terms);
    b.cnt = as<uint64_t>(c->cnt);
    b.off = as<uint64_t>(c->off);
    b.tiles = as<uint64_t>(c->tiles);
    b.scal = as<uint64_t>(c->scal);
    b.partials = as<Pair>(c->partials);
    b.seg_pairs = as<Pair>(c->seg_pairs);
    b.coefs = as<uint64_t>(c->coefs);
    b.lhsmod = as<uint64_t>(c->lhsmod);
    b.tails = as<uint32_t>(c->tails);
    b.tail_hist = as<unsigned long long>(c->tail_hist);
    return b;
}

int enqueue_plan(wv_ctx *c, const BatchBufs &b, const uint64_t *d_primes, const BatchShape &sh, hipStream_t st) {
    uint64_t *scal = b.scal;
    uint64_t *toff = b.off;   // prefix of terms, then of full chunks
    const uint64_t chunk_cfg = c->chunk_cfg ? c->chunk_cfg : c->chunk_auto;
    WV_HIP(launch_set_u64(st, scal, 8, 0));
    WV_HIP(launch_plan(st, d_primes, sh.n, sh.tb, sh.te, table_fallback(c, sh.tb), table_fallback(c, sh.te), sh.nB,
                       sh.nE, table_store(c), b.pr, b.segs, b.terms, b.coefs, b.lhsmod, 0));
    WV_HIP(launch_scan(st, b.terms, sh.nseg, toff, b.tiles));
    WV_HIP(launch_pick_chunk(st, toff + sh.nseg, sh.nseg, chunk_cfg, sum_lanes(c), sh.cap, scal + kScalLayout));
    WV_HIP(launch_copy_u64(st, toff + sh.nseg, scal + kScalTerms, 1));
    WV_HIP(launch_copy_u64(st, toff + (uint64_t)sh.n * sh.nB, scal + kScalTermsB, 1));
    WV_HIP(launch_chunk_layout(st, b.terms, sh.nseg, (uint64_t)sh.n * sh.nB, scal + kScalLayout, b.cnt, toff, b.tiles,
                               b.tail_hist, b.tails, scal + kScalChunks));
    return WV_OK;
}

int enqueue_sum(wv_ctx *c, const BatchBufs &b, const BatchShape &sh, hipStream_t st, uint64_t begin, uint64_t end) {
    uint64_t *scal = b.scal;
    const int v = c->variant;
    WV_HIP(launch_set_u64(st, scal + kScalCounter, 1, begin));
    WV_HIP(launch_sum(st, v, (unsigned)c->sum_blocks[v], b.segs, b.off, (uint32_t)sh.nseg, b.pr, scal + kScalLayout,
                      b.tails, b.partials, b.seg_pairs, (unsigned long long *)(scal + kScalCounter), end,
                      (unsigned long long *)(scal + kScalErr)));
    return WV_OK;
}

int enqueue_finish(wv_ctx *c, const BatchBufs &b, const BatchShape &sh, hipStream_t st, wv_result *d_out) {
    WV_HIP(launch_reduce(st, b.segs, b.off, (uint32_t)sh.nseg, b.pr, b.partials, b.scal + kScalLayout, b.seg_pairs));
    WV_HIP(launch_finalize(st, table_store(c), b.pr, b.seg_pairs, b.coefs, b.lhsmod, sh.n, sh.nB, sh.nE, d_out,
                           (const unsigned long long *)(b.scal + kScalErr)));
    return WV_OK;
}

// Synchronous batch on the context stream with timing.  When a progress
// callback is set, the term sums run as several launches over consecutive
// chunk ranges of about `launch_terms` terms each, with the callback between
// them; the partial pairs of all ranges are reduced together afterwards, so
// the result does not depend on the split.
int run_batch_sync(wv_ctx *c, const uint64_t *d_primes, uint32_t n, uint64_t pmax, wv_result *d_out) {
    hipStream_t st = c->stream;
    BatchShape sh;
    WV_TRY(batch_shape(c, n, pmax, &sh));
    WV_TRY(prepare(c, sh));
    const BatchBufs bufs = ctx_bufs(c);
    WV_HIP(hipEventRecord(c->ev[EV_PLAN0], st));
    WV_TRY(enqueue_plan(c, bufs, d_primes, sh, st));
    WV_HIP(hipEventRecord(c->ev[EV_PLAN], st));
    double ms_sum = 0.0;
    if (!c->progress) {
        // one launch; its time is read after the batch's single wait below
        WV_TRY(enqueue_sum(c, bufs, sh, st, 0, UINT64_MAX));
        WV_HIP(hipEventRecord(c->ev[EV_SUM], st));
    } else {
        uint64_t host[8];
        WV_HIP(hipMemcpyAsync(host, c->scal.ptr, sizeof(host), hipMemcpyDeviceToHost, st));
        WV_HIP(hipStreamSynchronize(st));
        const uint64_t total = host[kScalChunks], chunk = host[kScalLayout];
        const uint64_t per = std::max<uint64_t>(64, (c->launch_terms / std::max<uint64_t>(chunk, 1)) & ~63ull);
        for (uint64_t b = 0; b < total; b += per) {
            const uint64_t e = b + per >= total ? UINT64_MAX : b + per;   // ranges stay 64-aligned
            WV_HIP(hipEventRecord(c->ev[EV_SUM0], st));
            WV_TRY(enqueue_sum(c, bufs, sh, st, b, e));
            WV_HIP(hipEventRecord(c->ev[EV_SUM], st));
            WV_HIP(hipEventSynchronize(c->ev[EV_SUM]));
            ms_sum += elapsed(c->ev[EV_SUM0], c->ev[EV_SUM]);
            c->progress(c->progress_user, std::min(total, b + per), total);
        }
    }
    WV_HIP(launch_reduce(st, as<SegRec>(c->segs), as<uint64_t>(c->off), (uint32_t)sh.nseg, as<PrimeRec>(c->pr),
                         as<Pair>(c->partials), as<uint64_t>(c->scal) + kScalLayout, as<Pair>(c->seg_pairs)));
    WV_HIP(hipEventRecord(c->ev[EV_RED], st));
    WV_HIP(launch_finalize(st, table_store(c), as<PrimeRec>(c->pr), as<Pair>(c->seg_pairs), as<uint64_t>(c->coefs),
                           as<uint64_t>(c->lhsmod), sh.n, sh.nB, sh.nE, d_out,
                           (const unsigned long long *)(as<uint64_t>(c->scal) + kScalErr)));
    WV_HIP(hipEventRecord(c->ev[EV_FINAL], st));
    // statistics (the batch's one wait)
    uint64_t host[8];
    WV_HIP(hipMemcpyAsync(host, c->scal.ptr, sizeof(host), hipMemcpyDeviceToHost, st));
    WV_HIP(hipStreamSynchronize(st));
    if (host[kScalErr]) return WV_EHIP;   // the term sums did not cover every chunk
    if (!c->progress) ms_sum = elapsed(c->ev[EV_PLAN], c->ev[EV_SUM]);
    wv_stats &s = c->stats;
    s.ms_plan += elapsed(c->ev[EV_PLAN0], c->ev[EV_PLAN]);
    s.ms_sum += ms_sum;
    s.ms_reduce += elapsed(c->ev[EV_SUM], c->ev[EV_RED]);
    s.ms_finalize += elapsed(c->ev[EV_RED], c->ev[EV_FINAL]);
    s.ms_total += elapsed(c->ev[EV_PLAN0], c->ev[EV_FINAL]);
    s.n_primes += n;
    s.n_sums += sh.nseg;
    s.n_chunks += host[kScalChunks];
    s.n_terms += host[kScalTerms];
    s.n_terms_b += host[kScalTermsB];
    s.chunk_terms = host[kScalLayout];
    s.block_k_b = (uint32_t)sum_variant_kb(c->variant);
    s.block_k_e = (uint32_t)sum_variant_ke(c->variant);
    s.grid = (uint32_t)c->sum_blocks[c->variant];
    return WV_OK;
}

// ==========================================================================
// sieve over segment descriptors
// ==========================================================================

void window_descs(uint64_t lo, uint64_t hi, std::vector<SegDesc> &d, uint64_t piece) {
    if (hi <= lo || hi <= 5) return;
    piece = std::max<uint64_t>(piece, 1);
    for (uint64_t L = lo & ~1ull; L < hi; L += kSegSpan) {
        if (piece >= kSegSpan) {
            d.push_back(SegDesc{L, lo, hi});
            continue;
        }
        // the segment's integers in pieces: each piece sieves the whole
        // segment and keeps the primes of its own sub-range
        const uint64_t a = std::max(L, lo), b = std::min(L + kSegSpan, hi);
        for (uint64_t x = a; x < b; x += piece) d.push_back(SegDesc{L, x, std::min(b, x + piece)});
    }
}

uint64_t window_piece(const wv_ctx *c, uint64_t hi) {
    // integers holding about kMaxBatchTerms / 2 terms of work at primes near hi
    const double cost = side_cost(c, c->tb) + side_cost(c, c->te);
    const double per_prime = std::max(1.0, (double)hi * cost);
    const double w = kMaxBatchTerms / 2 / per_prime * std::log(std::max<double>((double)hi, 3.0));
    return (uint64_t)std::min<double>(std::max(w, 4096.0), (double)kSegSpan);
}

// Prime counts of descs[0..ns) into counts; with keep_bits the prime bitmaps
// stay in c->seg_bits for a following compaction (ns <= kMaxBatchSegs).
int sieve_count(wv_ctx *c, const SegDesc *descs, size_t ns, bool keep_bits, uint32_t *counts, hipStream_t st) {
    if (!st) st = c->stream;
    WV_TRY(ensure(c, c->seg_desc, std::min<size_t>(ns, kSieveLaunch) * sizeof(SegDesc)));
    WV_TRY(ensure(c, c->seg_counts, std::min<size_t>(ns, kSieveLaunch) * sizeof(uint32_t)));
    if (keep_bits) WV_TRY(ensure(c, c->seg_bits, ns * kSegWords * sizeof(uint32_t)));
    for (size_t b = 0; b < ns; b += kSieveLaunch) {
        const size_t k = std::min<size_t>(kSieveLaunch, ns - b);
        WV_HIP(hipMemcpyAsync(c->seg_desc.ptr, descs + b, k * sizeof(SegDesc), hipMemcpyHostToDevice, st));
        WV_HIP(launch_seg_sieve(st, as<SegDesc>(c->seg_desc), (unsigned)k, as<uint32_t>(c->base_primes), c->n_base,
                                keep_bits ? as<uint32_t>(c->seg_bits) : nullptr, as<uint32_t>(c->seg_counts)));
        WV_HIP(hipMemcpyAsync(counts + b, c->seg_counts.ptr, k * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        WV_HIP(hipStreamSynchronize(st));
    }
    return WV_OK;
}

// Primes of descs[0..ns) (bitmaps already in c->seg_bits) into c->primes.
int compact(wv_ctx *c, const SegDesc *descs, size_t ns, const uint32_t *counts, uint64_t *np_out, hipStream_t st,
            bool descs_ready) {
    if (!st) st = c->stream;
    std::vector<uint64_t> offs(ns + 1, 0);
    for (size_t i = 0; i < ns; i++) offs[i + 1] = offs[i] + counts[i];
    *np_out = offs[ns];
    if (offs[ns] == 0) return WV_OK;
    WV_TRY(ensure(c, c->seg_off, (ns + 1) * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->primes, offs[ns] * sizeof(uint64_t)));
    if (!descs_ready)
        WV_HIP(hipMemcpyAsync(c->seg_desc.ptr, descs, ns * sizeof(SegDesc), hipMemcpyHostToDevice, st));
    WV_HIP(hipMemcpyAsync(c->seg_off.ptr, offs.data(), (ns + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    WV_HIP(launch_seg_compact(st, as<SegDesc>(c->seg_desc), (unsigned)ns, as<uint32_t>(c->seg_bits),
                              as<uint64_t>(c->seg_off), as<uint64_t>(c->primes), offs[ns]));
    return WV_OK;
}

int pin_res_reserve(wv_ctx *c, size_t n) {
    if (n <= c->pin_res_cap) return WV_OK;
    const size_t want = std::max(n, c->pin_res_cap + c->pin_res_cap / 2);
    wv_result *h = nullptr;
    if (hipHostMalloc((void **)&h, want * sizeof(wv_result), hipHostMallocDefault) != hipSuccess) return WV_ENOMEM;
    if (c->pin_res) (void)hipHostFree(c->pin_res);
    c->pin_res = h;
    c->pin_res_cap = want;
    return WV_OK;
}

int results_to_host(wv_ctx *c, const wv_result *d, size_t n, wv_result *out) {
    if (n == 0) return WV_OK;
    WV_TRY(pin_res_reserve(c, n));
    WV_HIP(hipMemcpyAsync(c->pin_res, d, n * sizeof(wv_result), hipMemcpyDeviceToHost, c->stream));
    WV_HIP(hipStreamSynchronize(c->stream));
    std::memcpy(out, c->pin_res, n * sizeof(wv_result));
    return WV_OK;
}

// All primes of the descriptor list (in order) and their residues into out.
// Descriptors are grouped into batches of at most kMaxBatchSegs segments and
// about kMaxBatchPrimes primes; each batch is one plan and one persistent
// term-sum launch (or one split launch sequence under a progress callback).
int search_descs(wv_ctx *c, const std::vector<SegDesc> &descs, const std::vector<uint32_t> &counts, wv_result *out,
                 StatsSink *sink, const uint64_t *dest, bool bits_ready) {
    std::vector<wv_result> staging;
    hipStream_t st = c->stream;
    size_t i = 0, written = 0;
    while (i < descs.size()) {
        // a batch ends at kMaxBatchSegs segments, kMaxBatchPrimes primes or
        // about kMaxBatchTerms terms (bounded by count * largest p * cost):
        // with the partial pairs capped, a bigger batch would force chunks
        // longer than its sums
        // (slots per prime: those of the tables a batch up to its largest
        // prime can pick; work: each piece at the cost of the table serving
        // its top)
        size_t j = i;
        uint64_t np = 0, pm = 0;
        double est = 0.0;
        while (j < descs.size() && j - i < kMaxBatchSegs) {
            const uint64_t top = std::min(descs[j].hi, descs[j].L + kSegSpan);
            const uint64_t pm_j = std::max(pm, top);
            const uint64_t per = (uint64_t)side_slots(c, batch_table(c, c->tb, pm_j)) +
                                 side_slots(c, batch_table(c, c->te, pm_j));
            const uint64_t max_np = std::min<uint64_t>(kMaxBatchPrimes, kMaxBatchSlots / per);
            const double e = (double)counts[j] * (double)top * (prime_cost(c, c->tb, top) + prime_cost(c, c->te, top));
            if (np > 0 && (np + counts[j] > max_np || est + e > kMaxBatchTerms)) break;
            np += counts[j++];
            est += e;
            pm = pm_j;
        }
        if (np == 0) {
            i = j;
            continue;
        }
        WV_HIP(hipEventRecord(c->ev[EV_START], st));
        const bool whole = bits_ready && i == 0 && j == descs.size();
        if (!whole) {
            // the bitmaps of this batch's segments (the counting pass kept none)
            std::vector<uint32_t> again(j - i);
            WV_TRY(sieve_count(c, descs.data() + i, j - i, true, again.data()));
            for (size_t k = 0; k < again.size(); k++)
                if (again[k] != counts[i + k]) return WV_EHIP;   // the sieve is deterministic
        }
        uint64_t got = 0;
        // the counting pass (or the re-sieve just above) left these
        // descriptors in c->seg_desc when they fit one launch
        WV_TRY(compact(c, descs.data() + i, j - i, counts.data() + i, &got, nullptr, j - i <= kSieveLaunch));
        WV_HIP(hipEventRecord(c->ev[EV_SIEVE], st));
        WV_TRY(ensure(c, c->results, got * sizeof(wv_result)));
        uint64_t pmax = 0;
        for (size_t k = i; k < j; k++) pmax = std::max(pmax, std::min(descs[k].hi, descs[k].L + kSegSpan));
        WV_TRY(run_batch_sync(c, as<uint64_t>(c->primes), (uint32_t)got, pmax, as<wv_result>(c->results)));
        c->stats.ms_sieve += elapsed(c->ev[EV_START], c->ev[EV_SIEVE]);   // both recorded before its wait
        if (out && !dest) WV_TRY(results_to_host(c, as<wv_result>(c->results), got, out + written));
        if (out && dest) {
            staging.resize(got);
            WV_TRY(results_to_host(c, as<wv_result>(c->results), got, staging.data()));
            uint64_t o = 0;
            for (size_t k = i; k < j; k++) {
                std::memcpy(out + dest[k], staging.data() + o, counts[k] * sizeof(wv_result));
                o += counts[k];
            }
        }
        if (sink) {
            // near-miss slots: a counter, then room for two entries per prime
            WV_TRY(ensure(c, c->stats_near, 64 + 2 * got * sizeof(wv_near)));
            auto *cnt = as<unsigned long long>(c->stats_near);
            auto *near = reinterpret_cast<wv_near *>(as<char>(c->stats_near) + 64);
            WV_HIP(launch_set_u64(st, reinterpret_cast<uint64_t *>(cnt), 1, 0));
            WV_HIP(launch_stats(st, as<wv_result>(c->results), (uint32_t)got, sink->bins, sink->bound,
                                as<unsigned long long>(c->stats_hist), near, cnt));
            unsigned long long nn = 0;
            WV_HIP(hipMemcpyAsync(&nn, cnt, sizeof(nn), hipMemcpyDeviceToHost, st));
            WV_HIP(hipStreamSynchronize(st));
            if (nn > 2 * got) return WV_EHIP;   // cannot happen: two residues per prime
            const size_t base = sink->near.size();
            sink->near.resize(base + nn);
            if (nn)
                WV_HIP(hipMemcpyAsync(sink->near.data() + base, near, nn * sizeof(wv_near), hipMemcpyDeviceToHost,
                                      st));
        }
        WV_HIP(hipStreamSynchronize(st));
        written += got;
        i = j;
    }
    return WV_OK;
}

// ---- congruence registry ---------------------------------------------------

static std::vector<uint32_t> limbs_of(uint64_t v) {
    std::vector<uint32_t> l;
    while (v) {
        l.push_back((uint32_t)v);
        v >>= 32;
    }
    return l;
}

// Decimal string (optional leading '-') -> magnitude limbs and sign.
static bool parse_int(const char *str, std::vector<uint32_t> *mag, bool *neg) {
    if (!str) return false;
    mag->clear();
    *neg = false;
    const char *q = str;
    if (*q == '-' || *q == '+') *neg = *q++ == '-';
    if (!*q || std::strlen(q) > 20000) return false;
    for (; *q; q++) {
        if (*q < '0' || *q > '9') return false;
        uint64_t carry = (uint64_t)(*q - '0');
        for (uint32_t &w : *mag) {
            const uint64_t t = (uint64_t)w * 10 + carry;
            w = (uint32_t)t;
            carry = t >> 32;
        }
        if (carry) mag->push_back((uint32_t)carry);
    }
    if (mag->empty()) *neg = false;   // zero
    return true;
}

static int upload_tables(wv_ctx *c) {
    WV_TRY(ensure(c, c->tbl_head, c->t_head.size() * sizeof(TableHead)));
    WV_TRY(ensure(c, c->tbl_term, c->t_term.size() * sizeof(TableTerm)));
    WV_TRY(ensure(c, c->tbl_limb, std::max<size_t>(1, c->t_limb.size()) * sizeof(uint32_t)));
    WV_HIP(hipMemcpyAsync(c->tbl_head.ptr, c->t_head.data(), c->t_head.size() * sizeof(TableHead),
                          hipMemcpyHostToDevice, c->stream));
    WV_HIP(hipMemcpyAsync(c->tbl_term.ptr, c->t_term.data(), c->t_term.size() * sizeof(TableTerm),
                          hipMemcpyHostToDevice, c->stream));
    if (!c->t_limb.empty())
        WV_HIP(hipMemcpyAsync(c->tbl_limb.ptr, c->t_limb.data(), c->t_limb.size() * sizeof(uint32_t),
                              hipMemcpyHostToDevice, c->stream));
    WV_HIP(hipStreamSynchronize(c->stream));
    return WV_OK;
}

int table_add(wv_ctx *c, int deg, const std::vector<uint32_t> &lhs_mag, bool lhs_neg,
              const std::vector<std::vector<uint32_t>> &coef_mag, const std::vector<bool> &coef_neg,
              const uint64_t *xa, const uint64_t *xb, const uint64_t *ya, const uint64_t *yb, uint64_t min_p,
              int *id) {
    TableHead h{};
    h.deg = deg;
    h.n = (int32_t)coef_mag.size();
    h.term_off = (uint32_t)c->t_term.size();
    h.lhs_off = (uint32_t)c->t_limb.size();
    h.lhs_nlimb = (uint16_t)lhs_mag.size();
    h.lhs_neg = lhs_neg ? 1 : 0;
    h.min_p = min_p;
    // compiled tables serve every prime; a defined one hands the others to the
    // printed table of its degree until wv_set_table_below says otherwise
    h.below = c->t_head.size() < (size_t)WV_TABLE_COUNT ? -1 : (deg == 3 ? WV_TABLE_BB30 : WV_TABLE_EE33);
    c->t_limb.insert(c->t_limb.end(), lhs_mag.begin(), lhs_mag.end());
    double cost = 0.0;
    for (size_t i = 0; i < coef_mag.size(); i++) {
        TableTerm t{};
        t.xa = xa[i];
        t.xb = xb[i];
        t.ya = ya[i];
        t.yb = yb[i];
        t.limb_off = (uint32_t)c->t_limb.size();
        t.nlimb = (uint16_t)coef_mag[i].size();
        t.neg = coef_neg[i] ? 1 : 0;
        c->t_limb.insert(c->t_limb.end(), coef_mag[i].begin(), coef_mag[i].end());
        c->t_term.push_back(t);
        cost += (double)ya[i] / (double)yb[i] - (double)xa[i] / (double)xb[i];
    }
    c->t_head.push_back(h);
    c->t_cost.push_back(cost);
    const int rc = upload_tables(c);
    if (rc != WV_OK) {
        // leave the registry as it was (the next upload rewrites the device copy)
        c->t_head.pop_back();
        c->t_cost.pop_back();
        c->t_term.resize(h.term_off);
        c->t_limb.resize(h.lhs_off);
        return rc;
    }
    *id = (int)c->t_head.size() - 1;
    return WV_OK;
}

// The compiled tables, from wv_tables.hpp, become registry entries 0..WV_TABLE_COUNT-1.
int tables_init(wv_ctx *c) {
    c->t_head.clear();
    c->t_term.clear();
    c->t_limb.clear();
    c->t_cost.clear();
    for (int i = 0; i < kNumTables; i++) {
        const TableDef &d = kTables[i];
        std::vector<std::vector<uint32_t>> mag(d.n);
        std::vector<bool> neg(d.n);
        std::vector<uint64_t> xa(d.n), xb(d.n), ya(d.n), yb(d.n);
        for (int j = 0; j < d.n; j++) {
            const TermDef &t = d.t[j];
            mag[j] = limbs_of(t.coef < 0 ? (uint64_t)(-t.coef) : (uint64_t)t.coef);
            neg[j] = t.coef < 0;
            xa[j] = t.xa;
            xb[j] = t.xb;
            ya[j] = t.ya;
            yb[j] = t.yb;
        }
        int id = 0;
        WV_TRY(table_add(c, d.deg, limbs_of(d.lhs < 0 ? (uint64_t)(-d.lhs) : (uint64_t)d.lhs), d.lhs < 0, mag, neg,
                         xa.data(), xb.data(), ya.data(), yb.data(), 5, &id));
        if (id != i) return WV_EHIP;
    }
    return WV_OK;
}

TableStore table_store(wv_ctx *c) {
    return TableStore{as<TableHead>(c->tbl_head), as<TableTerm>(c->tbl_term), as<uint32_t>(c->tbl_limb)};
}

int table_fallback(const wv_ctx *c, int id) {
    if (id < WV_TABLE_COUNT) return id;
    return c->t_head[id].deg == 3 ? WV_TABLE_BB30 : WV_TABLE_EE33;
}

// The table a batch whose largest prime is pmax starts from: defined tables
// whose min_p no prime of the batch reaches hand over to the one below.
int batch_table(const wv_ctx *c, int id, uint64_t pmax) {
    while (id >= WV_TABLE_COUNT && pmax <= c->t_head[id].min_p) id = c->t_head[id].below;
    return id;
}

// Sums per prime and cost per unit p a batch must allow for: the largest over
// the tables the plan can pick from id down (the chain and its end).
int side_slots(const wv_ctx *c, int id) {
    int n = std::max(c->t_head[table_fallback(c, id)].n, 1);
    for (int t = id;; t = c->t_head[t].below) {
        n = std::max(n, c->t_head[t].n);
        if (t < WV_TABLE_COUNT) break;
    }
    return n;
}

// Terms per unit p of the table that serves a prime of size p (the chain's
// min_p only; an estimate of work, not a choice of table).
double prime_cost(const wv_ctx *c, int id, uint64_t p) {
    while (id >= WV_TABLE_COUNT && p < c->t_head[id].min_p) id = c->t_head[id].below;
    return c->t_cost[id];
}

double side_cost(const wv_ctx *c, int id) {
    double v = c->t_cost[table_fallback(c, id)];
    for (int t = id;; t = c->t_head[t].below) {
        v = std::max(v, c->t_cost[t]);
        if (t < WV_TABLE_COUNT) break;
    }
    return v;
}

void pick_tuned(wv_ctx *c, uint64_t pmax) {
    if (c->shape_forced || pmax < 2) return;
    int b = 63 - __builtin_clzll(pmax);
    for (const TuneEntry &t : c->tune)
        if (t.log2p == b) {
            c->variant = t.variant;
            c->chunk_auto = t.chunk;
            return;
        }
}

// An upper bound on the primes p with max(lo, 5) <= p < hi: the odd numbers
// there, pi(x) < 1.25506 x / log x (Rosser and Schoenfeld) below hi, and
// pi(x + y) - pi(x) <= 2 y / log y (Montgomery and Vaughan) for y > 1.
uint64_t prime_count_bound(uint64_t lo, uint64_t hi) {
    if (hi <= lo) return 0;
    const uint64_t y = hi - lo;
    uint64_t b = y / 2 + 2;
    if (hi > 17) b = std::min<uint64_t>(b, (uint64_t)(1.25506 * (double)hi / std::log((double)hi)) + 2);
    if (y > 1) b = std::min<uint64_t>(b, (uint64_t)(2.0 * (double)y / std::log((double)y)) + 2);
    return b;
}

// A single-batch search replayed from one captured graph: sieve -> segment
// offsets -> compaction -> plan -> term sums -> reduce -> finalize, sized by
// an upper bound on the prime count (rounded up to a multiple of 1024; the
// padding slots hold 0, which the plan rejects and which cost no term work).
// The device counts the primes; the count, the batch's scalars and the
// results come back after the call's one wait.  d: the segments (at most
// kMaxBatchSegs), in ascending order, so the compacted primes ascend.
int search_graph(wv_ctx *c, const std::vector<SegDesc> &d, uint64_t n_bound, uint64_t pmax, wv_result *out,
                 size_t *n_out) {
    hipStream_t st = c->stream;
    const uint64_t ns = d.size();
    const uint64_t n_pad = (n_bound + 1023) & ~1023ull;
    BatchShape sh;
    WV_TRY(batch_shape(c, (uint32_t)n_pad, pmax, &sh));
    if (sh.nseg > kMaxBatchSlots) return kGraphNotTaken;   // more than one batch: the counted path
    WV_TRY(prepare(c, sh));
    WV_TRY(ensure(c, c->seg_desc, ns * sizeof(SegDesc)));
    WV_TRY(ensure(c, c->seg_counts, ns * sizeof(uint32_t)));
    WV_TRY(ensure(c, c->seg_bits, ns * kSegWords * sizeof(uint32_t)));
    WV_TRY(ensure(c, c->seg_off, (ns + 1) * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->pad_primes, n_pad * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->results, n_pad * sizeof(wv_result)));
    WV_TRY(pin_res_reserve(c, n_pad));
    const uint64_t chunk = c->chunk_cfg ? c->chunk_cfg : c->chunk_auto;
    hipGraphExec_t exec = nullptr;
    for (GraphEntry &g : c->graphs)
        if (g.ns == ns && g.n_pad == n_pad && g.gen == c->gen && g.variant == c->variant && g.tb == c->tb &&
            g.te == c->te && g.chunk == chunk && g.tbl_b == sh.tb && g.tbl_e == sh.te)
            exec = g.exec;
    if (!exec) {
        WV_HIP(hipStreamSynchronize(st));   // the capture stream must be idle
        hipGraph_t graph = nullptr;
        WV_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        const BatchBufs bufs = ctx_bufs(c);
        uint64_t *primes = as<uint64_t>(c->pad_primes);
        int rc = WV_OK;
        if (launch_seg_sieve(st, as<SegDesc>(c->seg_desc), (unsigned)ns, as<uint32_t>(c->base_primes), c->n_base,
                             as<uint32_t>(c->seg_bits), as<uint32_t>(c->seg_counts)) != hipSuccess ||
            launch_copy_pad(st, primes, 0, primes, n_pad) != hipSuccess ||   // every slot 0 (padding)
            launch_seg_offsets(st, as<uint32_t>(c->seg_counts), (unsigned)ns, UINT64_MAX, as<uint64_t>(c->seg_off),
                               primes) != hipSuccess ||
            launch_seg_compact(st, as<SegDesc>(c->seg_desc), (unsigned)ns, as<uint32_t>(c->seg_bits),
                               as<uint64_t>(c->seg_off), primes, n_pad) != hipSuccess)
            rc = WV_EHIP;
        if (rc == WV_OK) rc = enqueue_plan(c, bufs, primes, sh, st);
        if (rc == WV_OK) rc = enqueue_sum(c, bufs, sh, st, 0, UINT64_MAX);
        if (rc == WV_OK) rc = enqueue_finish(c, bufs, sh, st, as<wv_result>(c->results));
        hipError_t e = hipStreamEndCapture(st, &graph);
        if (rc != WV_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        WV_HIP(e);
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        WV_HIP(e);
        GraphEntry g{n_pad, c->gen, c->variant, c->tb, c->te, chunk, exec};
        g.ns = ns;
        g.tbl_b = sh.tb;
        g.tbl_e = sh.te;
        c->graphs.push_back(g);
    }
    WV_HIP(hipMemcpyAsync(c->seg_desc.ptr, d.data(), ns * sizeof(SegDesc), hipMemcpyHostToDevice, st));
    WV_HIP(hipEventRecord(c->ev[EV_PLAN0], st));
    WV_HIP(hipGraphLaunch(exec, st));
    WV_HIP(hipEventRecord(c->ev[EV_FINAL], st));
    uint64_t host[9];
    WV_HIP(hipMemcpyAsync(c->pin_res, c->results.ptr, n_pad * sizeof(wv_result), hipMemcpyDeviceToHost, st));
    WV_HIP(hipMemcpyAsync(host, c->scal.ptr, 8 * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    WV_HIP(hipMemcpyAsync(host + 8, as<uint64_t>(c->seg_off) + ns, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    WV_HIP(hipStreamSynchronize(st));
    if (host[kScalErr]) return WV_EHIP;   // the term sums did not cover every chunk
    const uint64_t n = host[8];
    if (n > n_pad) return WV_EHIP;        // cannot happen: the bound holds
    std::memcpy(out, c->pin_res, n * sizeof(wv_result));
    *n_out = (size_t)n;
    wv_stats &s = c->stats;
    const double ms = elapsed(c->ev[EV_PLAN0], c->ev[EV_FINAL]);
    s.ms_total += ms;
    s.ms_sum += ms;   // one graph: the phases are not timed apart
    s.n_primes += n;
    s.n_sums += n * (sh.nB + sh.nE);
    s.n_chunks += host[kScalChunks];
    s.n_terms += host[kScalTerms];
    s.n_terms_b += host[kScalTermsB];
    s.chunk_terms = host[kScalLayout];
    s.block_k_b = (uint32_t)sum_variant_kb(c->variant);
    s.block_k_e = (uint32_t)sum_variant_ke(c->variant);
    s.grid = (uint32_t)c->sum_blocks[c->variant];
    return WV_OK;
}

}  // namespace wv

// ==========================================================================
// C ABI
// ==========================================================================

extern "C" {

const char *wv_strerror(int status) {
    switch (status) {
    case WV_OK: return "ok";
    case WV_EINVAL: return "invalid argument";
    case WV_EDOMAIN: return "prime outside [5, 2^40)";
    case WV_ENOTPRIME: return "input is not prime";
    case WV_ETRUNC: return "output buffer too small";
    case WV_ENOMEM: return "device out of memory";
    case WV_EHIP: return "HIP runtime error";
    case WV_EBUSY: return "request not finished";
    default: return "unknown status";
    }
}

int wv_table_info(int id, int *n_sums, int64_t *lhs, uint64_t *cost_num, uint64_t *cost_den) {
    if (id < 0 || id >= kNumTables) return WV_EINVAL;
    if (n_sums) *n_sums = kTables[id].n;
    if (lhs) *lhs = kTables[id].lhs;
    if (cost_num) *cost_num = kTables[id].cost_num;
    if (cost_den) *cost_den = kTables[id].cost_den;
    return WV_OK;
}

int wv_table_term(int id, int i, int64_t *coef, uint32_t *xa, uint32_t *xb, uint32_t *ya, uint32_t *yb) {
    if (id < 0 || id >= kNumTables || i < 0 || i >= kTables[id].n) return WV_EINVAL;
    const TermDef &t = kTables[id].t[i];
    if (coef) *coef = t.coef;
    if (xa) *xa = t.xa;
    if (xb) *xb = t.xb;
    if (ya) *ya = t.ya;
    if (yb) *yb = t.yb;
    return WV_OK;
}

int wv_create(int hip_device, wv_ctx **out) {
    if (!out) return WV_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) return WV_EINVAL;
    wv_ctx *c = new (std::nothrow) wv_ctx();
    if (!c) return WV_ENOMEM;
    c->device = hip_device;
    int rc = WV_OK;
    do {
        if (hipSetDevice(hip_device) != hipSuccess) { rc = WV_EHIP; break; }
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) { rc = WV_EHIP; break; }
        for (int i = 0; i < EV_COUNT; i++)
            if (hipEventCreate(&c->ev[i]) != hipSuccess) { rc = WV_EHIP; break; }
        if (rc) break;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) { rc = WV_EHIP; break; }
        c->num_cus = prop.multiProcessorCount;
        snprintf(c->arch, sizeof(c->arch), "%s", prop.gcnArchName);
        for (int v = 0; v < num_sum_variants(); v++) {
            int per_cu = 0;
            if (sum_variant_occupancy(v, &per_cu) != hipSuccess || per_cu < 1) per_cu = 1;
            c->sum_blocks[v] = c->num_cus * per_cu;
        }
        if ((rc = tables_init(c)) != WV_OK) break;
        if ((rc = ensure(c, c->base_primes, kBaseLimit / 2 * sizeof(uint32_t))) != WV_OK) break;
        if ((rc = ensure(c, c->scal, 8 * sizeof(uint64_t))) != WV_OK) break;
        if (launch_base_sieve(c->stream, as<uint32_t>(c->base_primes), as<uint32_t>(c->scal)) != hipSuccess) {
            rc = WV_EHIP;
            break;
        }
        uint32_t nb = 0;
        if (hipMemcpyAsync(&nb, c->scal.ptr, sizeof(nb), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) { rc = WV_EHIP; break; }
        c->n_base = nb;
        // the allocation-free entry point's scratch array on this device; a
        // failed lookup leaves that one entry point returning WV_EHIP
        if (static_scratch_setup(hip_device, &c->scratch) != WV_OK) {
            (void)hipGetLastError();
            c->scratch = nullptr;
        }
    } while (0);
    if (rc != WV_OK) {
        wv_destroy(c);
        return rc;
    }
    *out = c;
    return WV_OK;
}

int wv_destroy(wv_ctx *c) {
    if (!c) return WV_OK;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (GraphEntry &g : c->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    DevBuf *bufs[] = {&c->base_primes, &c->primes, &c->pr, &c->segs, &c->terms, &c->cnt, &c->off, &c->tiles,
                      &c->scal, &c->partials, &c->seg_pairs, &c->results, &c->seg_counts, &c->seg_bits,
                      &c->seg_off, &c->seg_desc, &c->pad_primes, &c->stats_hist, &c->stats_near, &c->coefs,
                      &c->lhsmod, &c->tbl_head, &c->tbl_term, &c->tbl_limb, &c->tails, &c->tail_hist,
                      &c->irr_tasks, &c->irr_units, &c->irr_primes, &c->irr_roff, &c->irr_v, &c->irr_fix,
                      &c->irr_counts, &c->irr_pairs, &c->irr_b, &c->irr_e};
    for (DevBuf *b : bufs)
        if (b->ptr) (void)hipFree(b->ptr);
    for (int i = 0; i < EV_COUNT; i++)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    if (c->pin_res) (void)hipHostFree(c->pin_res);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return WV_OK;
}

int wv_define_table(wv_ctx *c, int deg, const char *lhs, size_t n, const char *const *coef, const uint64_t *xa,
                    const uint64_t *xb, const uint64_t *ya, const uint64_t *yb, uint64_t min_p, int *id) {
    if (!c || !id || (deg != 2 && deg != 3) || n == 0 || n > kMaxTableTerms || !coef || !xa || !xb || !ya || !yb)
        return WV_EINVAL;
    if (min_p < 11 || min_p > WV_P_MAX) return WV_EINVAL;
    if ((int)c->t_head.size() >= WV_TABLE_COUNT + kMaxDefinedTables) return WV_EINVAL;
    std::vector<uint32_t> lmag;
    bool lneg = false;
    if (!parse_int(lhs, &lmag, &lneg) || lmag.empty() || lmag.size() > 0xFFFF) return WV_EINVAL;
    std::vector<std::vector<uint32_t>> mag(n);
    std::vector<bool> neg(n);
    for (size_t i = 0; i < n; i++) {
        bool ng = false;
        if (!parse_int(coef[i], &mag[i], &ng) || mag[i].size() > 0xFFFF) return WV_EINVAL;
        neg[i] = ng;
        // 0 <= x < y <= 1, denominators below 2^63
        if (xb[i] == 0 || yb[i] == 0 || xb[i] >> 63 || yb[i] >> 63) return WV_EINVAL;
        if (xa[i] > xb[i] || ya[i] > yb[i]) return WV_EINVAL;
        if ((unsigned __int128)xa[i] * yb[i] >= (unsigned __int128)ya[i] * xb[i]) return WV_EINVAL;
    }
    WV_TRY(check_device(c));
    WV_TRY(table_add(c, deg, lmag, lneg, mag, neg, xa, xb, ya, yb, min_p, id));
    c->gen++;   // captured graphs hold the old table ids' shapes
    return WV_OK;
}

int wv_set_table_below(wv_ctx *c, int id, int below) {
    if (!c) return WV_EINVAL;
    const int nt = (int)c->t_head.size();
    if (id < WV_TABLE_COUNT || id >= nt || below < 0 || below >= nt) return WV_EINVAL;
    if (c->t_head[below].deg != c->t_head[id].deg) return WV_EINVAL;
    if (below == WV_TABLE_V12 || below == WV_TABLE_E1) return WV_EINVAL;
    // a defined table below must start lower, so every chain ends at a compiled table
    if (below >= WV_TABLE_COUNT && c->t_head[below].min_p >= c->t_head[id].min_p) return WV_EINVAL;
    WV_TRY(check_device(c));
    const int32_t old = c->t_head[id].below;
    c->t_head[id].below = below;
    const int rc = upload_tables(c);
    if (rc != WV_OK) {
        c->t_head[id].below = old;   // the device copy may be partial: the next upload restores it
        return rc;
    }
    c->gen++;   // captured graphs were sized for the old chain
    return WV_OK;
}

int wv_set_tables(wv_ctx *c, int b_table, int e_table) {
    if (!c) return WV_EINVAL;
    const int nt = (int)c->t_head.size();
    if (b_table < 0 || b_table >= nt || e_table < 0 || e_table >= nt) return WV_EINVAL;
    if (c->t_head[b_table].deg != 3 || c->t_head[e_table].deg != 2) return WV_EINVAL;
    // the root forms eqnV12 / eqnE1 serve p = 5, 7 only
    if (b_table == WV_TABLE_V12 || e_table == WV_TABLE_E1) return WV_EINVAL;
    c->tb = b_table;
    c->te = e_table;
    return WV_OK;
}

int wv_set_chunk_terms(wv_ctx *c, uint64_t chunk_terms) {
    if (!c || (chunk_terms % 64) != 0) return WV_EINVAL;
    c->chunk_cfg = chunk_terms;
    return WV_OK;
}

int wv_set_block(wv_ctx *c, int kb, int ke) {
    if (!c) return WV_EINVAL;
    if (kb == 0 && ke == 0) {
        c->shape_forced = false;
        c->variant = kDefaultVariant;
        return WV_OK;
    }
    for (int v = 0; v < num_sum_variants(); v++) {
        if (sum_variant_kb(v) == kb && sum_variant_ke(v) == ke) {
            c->variant = v;
            c->shape_forced = true;
            return WV_OK;
        }
    }
    return WV_EINVAL;
}

int wv_set_progress(wv_ctx *c, wv_progress_fn fn, void *user, uint64_t terms_per_launch) {
    if (!c) return WV_EINVAL;
    c->progress = fn;
    c->progress_user = user;
    c->launch_terms = terms_per_launch ? terms_per_launch : (1ull << 44);
    return WV_OK;
}

int wv_get_stats(const wv_ctx *c, wv_stats *out) {
    if (!c || !out) return WV_EINVAL;
    *out = c->stats;
    return WV_OK;
}

int wv_count_primes(wv_ctx *c, uint64_t lo, uint64_t hi, uint64_t *n) {
    if (!c || !n || lo > hi) return WV_EINVAL;
    if (hi > WV_P_MAX) return WV_EDOMAIN;
    WV_TRY(check_device(c));
    *n = 0;
    std::vector<SegDesc> d;
    window_descs(lo, hi, d);
    if (d.empty()) return WV_OK;
    std::vector<uint32_t> counts(d.size());
    WV_TRY(sieve_count(c, d.data(), d.size(), false, counts.data()));
    uint64_t t = 0;
    for (uint32_t k : counts) t += k;
    *n = t;
    return WV_OK;
}

int wv_search_windows(wv_ctx *c, const uint64_t *lo, const uint64_t *hi, size_t nwin, wv_result *out, size_t cap,
                      size_t *n_out, size_t *win_off) {
    if (!c || !n_out || (nwin && (!lo || !hi))) return WV_EINVAL;
    for (size_t w = 0; w < nwin; w++) {
        if (lo[w] > hi[w]) return WV_EINVAL;
        if (hi[w] > WV_P_MAX) return WV_EDOMAIN;
    }
    WV_TRY(check_device(c));
    std::vector<SegDesc> d;
    std::vector<size_t> first(nwin + 1, 0);
    uint64_t pmax = 0;
    for (size_t w = 0; w < nwin; w++) {
        first[w] = d.size();
        window_descs(lo[w], hi[w], d, window_piece(c, hi[w]));
        if (hi[w] > lo[w]) pmax = std::max(pmax, hi[w] - 1);
    }
    first[nwin] = d.size();
    // a small single-window search: one graph, sized by the prime-count bound
    if (nwin == 1 && out && !d.empty() && d.size() <= kMaxBatchSegs && !c->progress) {
        const uint64_t bound = prime_count_bound(std::max<uint64_t>(lo[0], 5), hi[0]);
        const double work = (double)bound * (double)pmax * (side_cost(c, c->tb) + side_cost(c, c->te));
        if (bound <= cap && bound <= kMaxBatchPrimes && work <= kGraphSearchTerms) {
            c->stats = wv_stats{};
            pick_tuned(c, pmax);
            size_t n = 0;
            const int rc = search_graph(c, d, bound, pmax + 1, out, &n);
            if (rc != kGraphNotTaken) {
                if (rc != WV_OK) return rc;
                *n_out = n;
                if (win_off) {
                    win_off[0] = 0;
                    win_off[1] = n;
                }
                return WV_OK;
            }
        }
    }
    std::vector<uint32_t> counts(d.size());
    // a single batch's worth of segments keeps its bitmaps from this count
    const bool keep = d.size() <= kMaxBatchSegs;
    if (!d.empty()) WV_TRY(sieve_count(c, d.data(), d.size(), keep, counts.data()));
    uint64_t total = 0;
    for (size_t w = 0; w < nwin; w++) {
        if (win_off) win_off[w] = (size_t)total;
        for (size_t k = first[w]; k < first[w + 1]; k++) total += counts[k];
    }
    if (win_off) win_off[nwin] = (size_t)total;
    *n_out = (size_t)total;
    if (total > cap) return WV_ETRUNC;
    if (total > 0 && !out) return WV_EINVAL;
    c->stats = wv_stats{};
    if (total == 0) return WV_OK;
    pick_tuned(c, pmax);
    // Batch the segments in ascending position, so that a batch holds primes of
    // one size (chunk sizes then fit every sum of the batch), and place each
    // segment's primes at its window's offset.
    std::vector<uint64_t> dest(d.size());
    uint64_t o = 0;
    for (size_t k = 0; k < d.size(); k++) {
        dest[k] = o;
        o += counts[k];
    }
    std::vector<size_t> ord(d.size());
    for (size_t k = 0; k < ord.size(); k++) ord[k] = k;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return d[a].L < d[b].L; });
    std::vector<SegDesc> ds(d.size());
    std::vector<uint32_t> cs(d.size());
    std::vector<uint64_t> dst(d.size());
    bool same_order = true;
    for (size_t k = 0; k < ord.size(); k++) {
        ds[k] = d[ord[k]];
        cs[k] = counts[ord[k]];
        dst[k] = dest[ord[k]];
        same_order &= ord[k] == k;
    }
    return search_descs(c, ds, cs, out, nullptr, dst.data(), keep && same_order);
}

int wv_range_stats(wv_ctx *c, uint64_t lo, uint64_t hi, uint32_t bins, uint64_t near_bound, uint64_t *hist_b,
                   uint64_t *hist_e, wv_near *near, size_t near_cap, size_t *n_near, uint64_t *n_primes) {
    if (!c || lo > hi || bins == 0 || bins > WV_MAX_BINS || !hist_b || !hist_e || !n_near || (near_cap && !near))
        return WV_EINVAL;
    if (hi > WV_P_MAX) return WV_EDOMAIN;
    WV_TRY(check_device(c));
    std::vector<SegDesc> d;
    window_descs(lo, hi, d, window_piece(c, hi));
    std::vector<uint32_t> counts(d.size());
    if (!d.empty()) WV_TRY(sieve_count(c, d.data(), d.size(), false, counts.data()));
    uint64_t total = 0;
    for (uint32_t k : counts) total += k;
    c->stats = wv_stats{};
    StatsSink sink{bins, near_bound, {}};
    WV_TRY(ensure(c, c->stats_hist, 2 * (size_t)bins * sizeof(uint64_t)));
    WV_HIP(launch_fill_pairs(c->stream, as<Pair>(c->stats_hist), bins, 0, 0));   // 2 * bins zero words
    if (total > 0) {
        pick_tuned(c, hi - 1);
        WV_TRY(search_descs(c, d, counts, nullptr, &sink));
    }
    WV_HIP(hipMemcpyAsync(hist_b, c->stats_hist.ptr, bins * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
    WV_HIP(hipMemcpyAsync(hist_e, as<uint64_t>(c->stats_hist) + bins, bins * sizeof(uint64_t),
                          hipMemcpyDeviceToHost, c->stream));
    WV_HIP(hipStreamSynchronize(c->stream));
    std::sort(sink.near.begin(), sink.near.end(), [](const wv_near &a, const wv_near &b) {
        return a.p != b.p ? a.p < b.p : a.which < b.which;
    });
    *n_near = sink.near.size();
    if (n_primes) *n_primes = total;
    const size_t nw = std::min(near_cap, sink.near.size());
    if (nw) std::copy(sink.near.begin(), sink.near.begin() + nw, near);
    return sink.near.size() > near_cap ? WV_ETRUNC : WV_OK;
}

int wv_search_range(wv_ctx *c, uint64_t lo, uint64_t hi, wv_result *out, size_t cap, size_t *n_out,
                    uint64_t *hits, size_t hit_cap, size_t *n_hits) {
    if (!c || !n_out || lo > hi || (hit_cap && !hits)) return WV_EINVAL;
    if (n_hits) *n_hits = 0;
    WV_TRY(wv_search_windows(c, &lo, &hi, 1, out, cap, n_out, nullptr));
    size_t nh = 0;
    for (size_t i = 0; i < *n_out; i++) {
        if (out[i].flags) {
            if (nh < hit_cap) hits[nh] = out[i].p;
            nh++;
        }
    }
    if (n_hits) *n_hits = nh;
    return WV_OK;
}

int wv_eval_primes(wv_ctx *c, const uint64_t *primes, size_t n, wv_result *out) {
    if (!c) return WV_EINVAL;
    if (n == 0) return WV_OK;
    if (!primes || !out) return WV_EINVAL;
    if (n > 0xFFFFFFFFull) return WV_EINVAL;
    uint64_t pmax = 0;
    for (size_t i = 0; i < n; i++) {
        if (primes[i] < 5 || primes[i] >= WV_P_MAX) return WV_EDOMAIN;
        if (!is_prime_u64(primes[i])) return WV_ENOTPRIME;
        pmax = std::max(pmax, primes[i]);
    }
    WV_TRY(check_device(c));
    c->stats = wv_stats{};
    pick_tuned(c, pmax);
    WV_TRY(ensure(c, c->primes, n * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->results, n * sizeof(wv_result)));
    WV_HIP(hipMemcpyAsync(c->primes.ptr, primes, n * sizeof(uint64_t), hipMemcpyHostToDevice, c->stream));
    // batches of at most kMaxBatchSlots (prime, sum) slots, in input order
    const uint64_t per = (uint64_t)side_slots(c, c->tb) + side_slots(c, c->te);
    const size_t step = (size_t)std::max<uint64_t>(1, kMaxBatchSlots / per);
    for (size_t b = 0; b < n; b += step) {
        const size_t k = std::min(step, n - b);
        WV_TRY(run_batch_sync(c, as<uint64_t>(c->primes) + b, (uint32_t)k, pmax + 1, as<wv_result>(c->results) + b));
    }
    return results_to_host(c, as<wv_result>(c->results), n, out);
}

int wv_eval_sums(wv_ctx *c, const uint64_t *primes, size_t n, uint64_t *out_b, uint64_t *out_e) {
    if (!c) return WV_EINVAL;
    if (n == 0) return WV_OK;
    if (!primes || !out_b || !out_e || n > 0xFFFFFFFFull) return WV_EINVAL;
    uint64_t pmax = 0;
    for (size_t i = 0; i < n; i++) {
        if (primes[i] < 5 || primes[i] >= WV_P_MAX) return WV_EDOMAIN;
        if (!is_prime_u64(primes[i])) return WV_ENOTPRIME;
        pmax = std::max(pmax, primes[i]);
    }
    WV_TRY(check_device(c));
    c->stats = wv_stats{};
    BatchShape sh;
    WV_TRY(batch_shape(c, (uint32_t)n, pmax + 1, &sh));
    if (sh.nseg > kMaxBatchSlots) return WV_EINVAL;   // one batch only
    WV_TRY(ensure(c, c->primes, n * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->results, std::max(n * sizeof(wv_result), (size_t)sh.nseg * sizeof(uint64_t))));
    WV_HIP(hipMemcpyAsync(c->primes.ptr, primes, n * sizeof(uint64_t), hipMemcpyHostToDevice, c->stream));
    WV_TRY(run_batch_sync(c, as<uint64_t>(c->primes), (uint32_t)n, pmax + 1, as<wv_result>(c->results)));
    // the results buffer is free again once finalize has run: reuse it for the sums
    uint64_t *d_sums = as<uint64_t>(c->results);
    WV_HIP(launch_sum_values(c->stream, as<SegRec>(c->segs), as<PrimeRec>(c->pr), as<Pair>(c->seg_pairs), sh.nseg,
                             d_sums));
    WV_HIP(hipMemcpyAsync(out_b, d_sums, (size_t)n * sh.nB * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
    WV_HIP(hipMemcpyAsync(out_e, d_sums + (size_t)n * sh.nB, (size_t)n * sh.nE * sizeof(uint64_t),
                          hipMemcpyDeviceToHost, c->stream));
    WV_HIP(hipStreamSynchronize(c->stream));
    return WV_OK;
}

// Device-pointer entry point: pads the batch to a power of two (padding slots
// hold 0, which the plan rejects and which cost no term work), and replays a
// captured graph of the whole plan -> finalize sequence for that size.
int wv_eval_primes_async(wv_ctx *c, const uint64_t *d_primes, size_t n, wv_result *d_out, void *hip_stream) {
    if (!c) return WV_EINVAL;
    if (n == 0) return WV_OK;
    if (!d_primes || !d_out || n > 0x7FFFFFFFull) return WV_EINVAL;
    WV_TRY(check_device(c));
    hipStream_t st = (hipStream_t)hip_stream;
    uint64_t n_pad = 64;
    while (n_pad < n) n_pad <<= 1;
    BatchShape sh;
    WV_TRY(batch_shape(c, (uint32_t)n_pad, WV_P_MAX, &sh));   // the primes are not seen on the host
    if (sh.nseg > kMaxBatchSlots) return WV_EINVAL;            // one captured batch
    WV_TRY(prepare(c, sh));
    WV_TRY(ensure(c, c->pad_primes, n_pad * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->results, n_pad * sizeof(wv_result)));
    hipGraphExec_t exec = nullptr;
    const uint64_t chunk = c->chunk_cfg ? c->chunk_cfg : c->chunk_auto;
    for (GraphEntry &g : c->graphs)
        if (g.ns == 0 && g.n_pad == n_pad && g.gen == c->gen && g.variant == c->variant && g.tb == c->tb &&
            g.te == c->te && g.chunk == chunk)
            exec = g.exec;
    if (!exec) {
        // the capture stream must be idle: earlier work on it may still run
        WV_HIP(hipStreamSynchronize(c->stream));
        hipGraph_t graph = nullptr;
        WV_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        const BatchBufs bufs = ctx_bufs(c);
        int rc = enqueue_plan(c, bufs, as<uint64_t>(c->pad_primes), sh, c->stream);
        if (rc == WV_OK) rc = enqueue_sum(c, bufs, sh, c->stream, 0, UINT64_MAX);
        if (rc == WV_OK) rc = enqueue_finish(c, bufs, sh, c->stream, as<wv_result>(c->results));
        hipError_t e = hipStreamEndCapture(c->stream, &graph);
        if (rc != WV_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        WV_HIP(e);
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        WV_HIP(e);
        c->graphs.push_back(GraphEntry{n_pad, c->gen, c->variant, c->tb, c->te, chunk, exec});
    }
    WV_HIP(launch_copy_pad(st, d_primes, n, as<uint64_t>(c->pad_primes), n_pad));
    WV_HIP(hipGraphLaunch(exec, st));
    WV_HIP(launch_copy_results(st, as<wv_result>(c->results), n, d_out));
    return WV_OK;
}

}  // extern "C"
