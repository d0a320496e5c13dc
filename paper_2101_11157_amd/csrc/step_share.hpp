// How the request server composes a step (host code only, no HIP): the whole
// primes that each active request hands to the next step.
#pragma once
#include <algorithm>
#include <cstddef>
#include <cstdint>

namespace wv {

// Tasks per step at most (whole primes of nB + nE sums each): with the
// derived ladders' 61,597 sums per prime near 1e11, 136 primes, so that the
// configured step_terms (2^38 by default, about 88 such primes) sets the
// step, not this cap (at 2^22 it did: 68 primes, 2 % less throughput on the
// serving trace for a third less median latency).  Half of it while a
// request with little work left is active.
constexpr uint64_t kMaxStepTasks = 1ull << 23;

// One active request as the step planner sees it.
struct ShareReq {
    uint64_t left;  // primes not yet handed to a step (> 0)
    double tpp;     // estimated terms per prime (> 0)
};

// Primes per step at most for candidates sorted by remaining work: the task
// cap over the sums per prime, the cap halved while the least candidate has
// at most an eighth of step_terms left (a single prime, a short interval),
// so that it completes in a short step; at least one.
inline uint64_t step_max_primes(const ShareReq &least, double step_terms, uint64_t sums_per_prime) {
    const bool small_left = (double)least.left * least.tpp * 8.0 <= step_terms;
    const uint64_t cap = small_left ? kMaxStepTasks / 2 : kMaxStepTasks;
    return std::max<uint64_t>(1, cap / std::max<uint64_t>(1, sums_per_prime));
}

// Fills give[0..n) for n > 0 candidates sorted by remaining work (left * tpp)
// ascending and returns the step's primes: first an even share of
// step_terms to every candidate, then what is left of the budget to the
// smallest remaining work first, the first prime regardless of the budget,
// never more than step_max_primes in all.
inline uint64_t step_share(const ShareReq *c, size_t n, double step_terms, uint64_t sums_per_prime, uint32_t *give) {
    const uint64_t max_q = step_max_primes(c[0], step_terms, sums_per_prime);
    double budget = step_terms;
    uint64_t nq = 0;
    const double even = budget / (double)n;
    for (size_t k = 0; k < n; k++) {
        const uint64_t g = std::min<uint64_t>({c[k].left, (uint64_t)(even / c[k].tpp), max_q - nq});
        give[k] = (uint32_t)g;
        nq += g;
        budget -= (double)g * c[k].tpp;
    }
    for (size_t k = 0; k < n && nq < max_q; k++) {
        const uint64_t left = c[k].left - give[k];
        if (!left) continue;
        if (budget < c[k].tpp && nq > 0) break;
        const uint64_t g = std::min<uint64_t>({left, std::max<uint64_t>(1, (uint64_t)(budget / c[k].tpp)), max_q - nq});
        give[k] += (uint32_t)g;
        nq += g;
        budget -= (double)g * c[k].tpp;
    }
    return nq;
}

}  // namespace wv
