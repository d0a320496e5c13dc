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

// x < 4p -> x mod p
__host__ __device__ __forceinline__ uint64_t canon4(uint64_t x, uint64_t p) {
    x = x >= 2 * p ? x - 2 * p : x;
    return x >= p ? x - p : x;
}

// a, b in [0, p), negp = 2^64 - p: a + b mod p as two 64-bit adds, an
// arithmetic shift of the high word of s - p into a mask, and two bitfield
// selects.  No carry or condition flags, so consecutive additions interleave
// freely.  (The selects are written as instructions: the compiler otherwise
// rebuilds a compare-and-select chain through the condition register.)
__host__ __device__ __forceinline__ uint64_t addm_n(uint64_t a, uint64_t b, uint64_t negp) {
    const uint64_t s = a + b;
    const uint64_t t = s + negp;                   // s - p, negative when s < p
    const uint32_t sl = (uint32_t)s, sh = (uint32_t)(s >> 32);
    const uint32_t tl = (uint32_t)t, th = (uint32_t)(t >> 32);
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t mask, rl, rh;
    asm("v_ashrrev_i32 %0, 31, %1" : "=v"(mask) : "v"(th));
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(rl) : "v"(mask), "v"(sl), "v"(tl));
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(rh) : "v"(mask), "v"(sh), "v"(th));
#else
    const uint32_t mask = (uint32_t)((int32_t)th >> 31);
    const uint32_t rl = (sl & mask) | (tl & ~mask);
    const uint32_t rh = (sh & mask) | (th & ~mask);
#endif
    return ((uint64_t)rh << 32) | rl;
}

// u = s^DEG R mod p for one s < p (canonical).
template <int DEG>
__host__ __device__ __forceinline__ uint64_t pow_mont(uint64_t s, const Mont &m, uint64_t r2) {
    const uint64_t sR = to_mont(s, r2, m);
    uint64_t u = red1(mmul(sR, sR, m), m.p);
    if (DEG == 3) u = red1(mmul(u, sR, m), m.p);
    return u;
}

// Blocked form of eqnComputeS.  For a block of K consecutive s starting at x,
//   prod_{j<K} (z + (x+j)^DEG) = P(x) + Q(x) z + O(z^2),
//   P(x) = prod_j (x+j)^DEG,   Q(x) = sum_j prod_{i != j} (x+i)^DEG,
// and P, Q are polynomials in x of degrees DEG*K and DEG*(K-1).  Along the
// blocks x = s0, s0+K, s0+2K, ... they are stepped by forward differences and
// each block is folded into the running pair with the pair product of
// eqnCombinePairs:
//   (c0, c1) <- (c0 P, c0 Q + c1 P)      (three Montgomery products per block).
// The difference tables start from P, Q evaluated directly at the first
// DEG*K + 1 block points, in [0, p).  Between reductions the differences are
// stepped as plain 64-bit sums: n steps from entries below 2p leave every entry
// below 2p * 2^n (entry i becomes sum_j C(n, j) D_{i+j}), and the Montgomery
// product accepts such a second operand for n <= 20 (mont.hpp).  So the tables
// are brought back below 2p only every kRenorm blocks, by reduce_f64.  Each
// sum passes through opaque(): the compiler otherwise recognises the chain of
// additions as a polynomial recurrence and rewrites the values after the loop
// as closed forms with binomial coefficients, which costs hundreds of
// registers.  Terms
// beyond the last full block are folded one by one.  The result is the same
// (c0, c1) as run_chunk up to rounding order, which exact arithmetic does not
// have: bit-identical residues.
// x < p * 2^24, p < 2^40 -> r == x (mod p), r in [0, 2p).  The quotient is
// estimated in double precision: xd * pinv carries a relative error below
// 2^-51 on a value below 2^24, so y = x/p - 1/2 is known to within 2^-26 and
// its truncation is floor(x/p) or one less (0 when y < 0).  The remainder is
// formed modulo 2^64 as x + q (2^64 - p).
__host__ __device__ __forceinline__ uint64_t reduce_f64(uint64_t x, uint64_t negp, double pinv) {
    const double y = (double)x * pinv - 0.5;
    const uint32_t q = y > 0.0 ? (uint32_t)y : 0u;
    return x + mul32w(q, (uint32_t)negp) + ((uint64_t)(q * (uint32_t)(negp >> 32)) << 32);
}

constexpr int kRenorm = 20;

// x unchanged, but hidden from the optimiser's recurrence analysis
__host__ __device__ __forceinline__ uint64_t opaque(uint64_t x) {
#if defined(__HIP_DEVICE_COMPILE__)
    asm("" : "+v"(x));
#endif
    return x;
}

template <int DEG, int K>
__host__ __device__ __forceinline__ void run_chunk_blocked(uint64_t s0, uint64_t n, const Mont &m, uint64_t r2,
                                                           uint64_t one, uint64_t &c0, uint64_t &c1) {
    constexpr int DP = DEG * K;
    constexpr int DQ = DEG * (K - 1);
    const uint64_t p = m.p;
    const uint64_t nb = n / K;
    uint64_t a0 = 1, a1 = 0;
    if (nb > 0) {
        uint64_t Pd[DP + 1] = {}, Qd[DQ + 1] = {};
        // direct values at x = s0 + b K, b = 0..DP, with u = s^DEG R stepped
        // over consecutive s by forward differences
        const uint64_t sR = to_mont(s0, r2, m);
        const uint64_t s2R = red1(mmul(sR, sR, m), p);
        uint64_t u, d1, d2 = 0, d3 = 0;
        if (DEG == 3) {
            u = red1(mmul(s2R, sR, m), p);
            const uint64_t t3s = addm(addm(sR, sR, p), sR, p);
            d1 = addm(addm(addm(addm(s2R, s2R, p), s2R, p), t3s, p), one, p);
            const uint64_t six = addm(addm(addm(one, one, p), addm(one, one, p), p), addm(one, one, p), p);
            d2 = addm(addm(t3s, t3s, p), six, p);
            d3 = six;
        } else {
            u = s2R;
            d1 = addm(addm(sR, sR, p), one, p);
            d2 = addm(one, one, p);
        }
WV_UNROLL
        for (int b = 0; b <= DP; b++) {
            uint64_t P = one, Q = 0;
            for (int j = 0; j < K; j++) {
                Q = mmul(Q, u, m) + P;
                P = mmul(P, u, m);
                u = addm(u, d1, p);
                d1 = addm(d1, d2, p);
                if (DEG == 3) d2 = addm(d2, d3, p);
            }
            Pd[b] = canon4(P, p);
            if (b <= DQ) Qd[b] = canon4(Q, p);
        }
        // forward differences at b = 0: entry i becomes Delta^i
WV_UNROLL
        for (int lev = 1; lev <= DP; lev++) {
WV_UNROLL
            for (int i = DP; i >= lev; i--) Pd[i] = subm(Pd[i], Pd[i - 1], p);
        }
WV_UNROLL
        for (int lev = 1; lev <= DQ; lev++) {
WV_UNROLL
            for (int i = DQ; i >= lev; i--) Qd[i] = subm(Qd[i], Qd[i - 1], p);
        }
        const uint64_t negp = 0 - p;
        const double pinv = 1.0 / (double)p;
        uint64_t b = 0;
        for (;;) {
            const uint64_t steps = nb - b < (uint64_t)kRenorm ? nb - b : (uint64_t)kRenorm;
            for (uint64_t k = 0; k < steps; k++) {
                a1 = mmul(a0, Qd[0], m) + mmul(a1, Pd[0], m);
                a0 = mmul(a0, Pd[0], m);
WV_UNROLL
                for (int i = 0; i < DP; i++) Pd[i] = opaque(Pd[i] + Pd[i + 1]);
WV_UNROLL
                for (int i = 0; i < DQ; i++) Qd[i] = opaque(Qd[i] + Qd[i + 1]);
            }
            b += steps;
            if (b >= nb) break;
WV_UNROLL
            for (int i = 0; i < DP; i++) Pd[i] = reduce_f64(Pd[i], negp, pinv);
WV_UNROLL
            for (int i = 0; i < DQ; i++) Qd[i] = reduce_f64(Qd[i], negp, pinv);
        }
    }
    for (uint64_t t = nb * K; t < n; t++) {
        const uint64_t u = pow_mont<DEG>(s0 + t, m, r2);
        a1 = mmul(a1, u, m) + a0;
        a0 = mmul(a0, u, m);
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
