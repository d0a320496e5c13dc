// sum_core.hpp -- the per-lane hot loop of the term-sum kernel and the
// chunk-to-sum lookup, written so that a plain C++ build can unit-test them.
#pragma once
#include <cstdint>
#include "mont.hpp"

namespace wv {

// (c0, c1) of prod_{s = s0}^{s0+n-1} (z + s^DEG) mod p (eqnComputeS), with
// u = s^DEG R mod p stepped by forward differences.  c0, c1 enter as (1, 0)
// and leave lazy (c0 < 2p, c1 < 4p); u and its differences stay in [0, p).
template <int DEG>
__device__ __forceinline__ void run_chunk(uint64_t s0, uint64_t n, const Mont &m, uint64_t r2, uint64_t one,
                                          uint64_t &c0, uint64_t &c1) {
    const uint64_t p = m.p;
    const uint64_t sR = to_mont(s0, r2, m);
    const uint64_t s2R = red1(mmul(sR, sR, m), p);
    uint64_t u, d1, d2 = 0, d3 = 0;
    if (DEG == 3) {
        // s^3, 3s^2+3s+1, 6s+6, 6
        u = red1(mmul(s2R, sR, m), p);
        const uint64_t t3s = addm(addm(sR, sR, p), sR, p);
        d1 = addm(addm(addm(addm(s2R, s2R, p), s2R, p), t3s, p), one, p);
        const uint64_t six = addm(addm(addm(one, one, p), addm(one, one, p), p), addm(one, one, p), p);
        d2 = addm(addm(t3s, t3s, p), six, p);
        d3 = six;
    } else {
        // s^2, 2s+1, 2
        u = s2R;
        d1 = addm(addm(sR, sR, p), one, p);
        d2 = addm(one, one, p);
    }
    uint64_t a0 = 1, a1 = 0;
    for (uint64_t k = 0; k < n; k++) {
        a1 = mmul(a1, u, m) + a0;
        a0 = mmul(a0, u, m);
        u = addm(u, d1, p);
        d1 = addm(d1, d2, p);
        if (DEG == 3) d2 = addm(d2, d3, p);
    }
    c0 = a0;
    c1 = a1;
}

__device__ __forceinline__ uint32_t find_seg(const uint64_t *__restrict__ off, uint32_t nseg, uint64_t chunk) {
    // largest j in [0, nseg) with off[j] <= chunk
    uint32_t lo = 0, hi = nseg;   // invariant: off[lo] <= chunk < off[hi] (off[nseg] = total)
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= chunk) lo = mid;
        else hi = mid;
    }
    return lo;
}

}  // namespace wv
