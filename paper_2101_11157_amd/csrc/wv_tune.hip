// wv_tune.hip -- autotuner of the term-sum launch shape.
//
// The block shape (terms per block on the s^3 and s^2 sides) and the chunk
// size (terms per lane) decide the term-sum kernel's speed: larger blocks cut
// the Montgomery products per term but raise register use and occupancy
// drops; larger chunks amortise the difference tables but coarsen the load
// balance.  The tuner times every compiled shape with three chunk sizes on
// sample primes of the target size and keeps the fastest per power of two.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "wv_ctx.hpp"

using namespace wv;

extern "C" {

int wv_autotune(wv_ctx *c, uint64_t p_hint, int n_sample, int *kb, int *ke, uint64_t *chunk_terms, double *rates) {
    if (!c || p_hint < 11 || p_hint >= WV_P_MAX) return p_hint >= WV_P_MAX ? WV_EDOMAIN : WV_EINVAL;
    WV_TRY(check_device(c));
    if (n_sample <= 0) n_sample = 16;
    // sample: the first n_sample primes at or above p_hint
    std::vector<SegDesc> d;
    std::vector<uint32_t> counts;
    uint64_t width = 1 << 12, np = 0;
    for (;;) {
        d.clear();
        const uint64_t hi = std::min<uint64_t>(WV_P_MAX, p_hint + width);
        window_descs(p_hint, hi, d);
        counts.assign(d.size(), 0);
        WV_TRY(sieve_count(c, d.data(), d.size(), d.size() <= kMaxBatchSegs, counts.data()));
        np = 0;
        for (uint32_t k : counts) np += k;
        if (np >= (uint64_t)n_sample || hi == WV_P_MAX || d.size() > kMaxBatchSegs / 2) break;
        width <<= 1;
    }
    if (np == 0 || d.size() > kMaxBatchSegs) return WV_EINVAL;
    const uint64_t sample_hi = std::min<uint64_t>(WV_P_MAX, p_hint + width);
    uint64_t got = 0;
    WV_TRY(compact(c, d.data(), d.size(), counts.data(), &got));
    const uint32_t n = (uint32_t)std::min<uint64_t>(got, (uint64_t)n_sample);
    WV_TRY(ensure(c, c->results, n * sizeof(wv_result)));
    // keep the sample apart: search buffers are reused by every call
    DevBuf sample;
    WV_HIP(hipMalloc(&sample.ptr, n * sizeof(uint64_t)));
    WV_HIP(hipMemcpyAsync(sample.ptr, c->primes.ptr, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, c->stream));

    const int saved_variant = c->variant;
    const bool saved_forced = c->shape_forced;
    const uint64_t saved_chunk = c->chunk_cfg;
    const uint64_t chunks[3] = {1ull << 16, 1ull << 18, 0};   // 0: adaptive per batch
    int best_v = kDefaultVariant;
    uint64_t best_c = kDefaultChunk;
    double best = -1.0;
    int rc = WV_OK;
    const uint64_t saved_auto = c->chunk_auto;
    c->chunk_auto = 0;
    c->variant = kDefaultVariant;
    c->chunk_cfg = kDefaultChunk;
    c->stats = wv_stats{};
    rc = run_batch_sync(c, as<uint64_t>(sample), n, sample_hi, as<wv_result>(c->results));   // warm-up
    for (int v = 0; v < num_sum_variants() && rc == WV_OK; v++) {
        for (int j = 0; j < 3 && rc == WV_OK; j++) {
            c->variant = v;
            c->chunk_cfg = chunks[j];
            c->stats = wv_stats{};
            rc = run_batch_sync(c, as<uint64_t>(sample), n, sample_hi, as<wv_result>(c->results));
            if (rc != WV_OK) break;
            const double r = c->stats.ms_sum > 0 ? (double)c->stats.n_terms / (c->stats.ms_sum * 1e-3) : 0.0;
            if (rates) rates[v * 3 + j] = r;
            if (r > best) {
                best = r;
                best_v = v;
                best_c = chunks[j];
            }
        }
    }
    c->variant = saved_forced ? saved_variant : best_v;
    c->shape_forced = saved_forced;
    c->chunk_cfg = saved_chunk;
    c->chunk_auto = saved_auto;
    (void)hipFree(sample.ptr);
    if (rc != WV_OK) return rc;
    const int lg = 63 - __builtin_clzll(p_hint);
    TuneEntry e{lg, best_v, best_c, best};
    bool replaced = false;
    for (TuneEntry &t : c->tune)
        if (t.log2p == lg) {
            t = e;
            replaced = true;
        }
    if (!replaced) c->tune.push_back(e);
    if (!saved_forced) c->chunk_auto = best_c;
    if (kb) *kb = sum_variant_kb(best_v);
    if (ke) *ke = sum_variant_ke(best_v);
    if (chunk_terms) *chunk_terms = best_c;
    return WV_OK;
}

int wv_tune_save(const wv_ctx *c, const char *path) {
    if (!c || !path) return WV_EINVAL;
    FILE *f = fopen(path, "w");
    if (!f) return WV_EINVAL;
    for (const TuneEntry &t : c->tune)
        fprintf(f, "%s %d %d %d %llu %.6e\n", c->arch, t.log2p, sum_variant_kb(t.variant), sum_variant_ke(t.variant),
                (unsigned long long)t.chunk, t.terms_per_s);
    fclose(f);
    return WV_OK;
}

// Entries for another architecture or an uncompiled shape are skipped.
int wv_tune_load(wv_ctx *c, const char *path) {
    if (!c || !path) return WV_EINVAL;
    FILE *f = fopen(path, "r");
    if (!f) return WV_EINVAL;
    char arch[64];
    int lg, kb, ke;
    unsigned long long chunk;
    double rate;
    while (fscanf(f, "%63s %d %d %d %llu %lf", arch, &lg, &kb, &ke, &chunk, &rate) == 6) {
        if (strcmp(arch, c->arch) != 0 || lg < 0 || lg > 40 || chunk % 64 != 0) continue;   // 0: adaptive
        int v = -1;
        for (int k = 0; k < num_sum_variants(); k++)
            if (sum_variant_kb(k) == kb && sum_variant_ke(k) == ke) v = k;
        if (v < 0) continue;
        TuneEntry e{lg, v, (uint64_t)chunk, rate};
        bool replaced = false;
        for (TuneEntry &t : c->tune)
            if (t.log2p == lg) {
                t = e;
                replaced = true;
            }
        if (!replaced) c->tune.push_back(e);
    }
    fclose(f);
    return WV_OK;
}

}  // extern "C"
