// sum_core.hpp -- the per-lane hot loop of the term-sum kernel and the
// chunk-to-sum lookup, written so that a plain C++ build can unit-test them.
#pragma once
#include <cmath>
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

__host__ __device__ __forceinline__ double opaque_f(double x) {
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

// ---- the blocked loop in double precision ------------------------------------
//
// Residues held as integer-valued doubles, signed and lazily reduced, for p <
// 2^40.  One modular product of integers a, b is six full-rate f64 operations:
//   h = ab rounded;  l = fma(a, b, -h) = ab - h exactly (an error-free product);
//   q = the integer nearest h * (1/p) (fma with 1.5 * 2^52, then subtract it);
//   r = fma(-q, p, h) + l.
// With |ab| <= 300 p^2 (the loop's bounds below): h/p < 2^49, so the rounding
// trick applies; |q - h/p| <= 1/2 + h 2^-53 / p, so h - qp is an integer below
// p in magnitude and the fma computes it exactly; l is an integer with
// |l| <= h 2^-53; hence r = ab - qp exactly, r == ab (mod p), and
// |r| <= p/2 + 2 h 2^-53 <= p/2 + 600 p 2^-13 <= 0.574 p.
struct Fmod {
    double p, pinv;   // p, round(1/p)
};

constexpr double kRound = 6755399441055744.0;   // 1.5 * 2^52: x + kRound - kRound rounds |x| < 2^51

__host__ __device__ __forceinline__ double f_mulmod(double a, double b, const Fmod &f) {
    const double h = a * b;
    const double l = fma(a, b, -h);
    const double q = fma(h, f.pinv, kRound) - kRound;
    return fma(-q, f.p, h) + l;
}

// x an integer, |x| <= 2^53 -> r == x (mod p), |r| <= p/2 + 2 |x| 2^-53 / p (< 0.51p), exactly.
__host__ __device__ __forceinline__ double f_reduce(double x, const Fmod &f) {
    const double q = fma(x, f.pinv, kRound) - kRound;
    return fma(-q, f.p, x);
}

// an integer below 2^50 in magnitude -> its canonical residue in [0, p)
__host__ __device__ __forceinline__ uint64_t f_canon(double x, const Fmod &f) {
    const double r = f_reduce(x, f);
    return (uint64_t)(r < 0.0 ? r + f.p : r);
}

// Same fold as run_chunk_blocked (P(x), Q(x) of each block of K terms stepped
// by finite differences; (c0, c1) <- (c0 P, c0 Q + c1 P)), in the double
// representation above.  The direct values at the first DEG*K + 1 block points
// are products of s^DEG mod p, their difference table is reduced to
// (-0.51p, 0.51p), and after n steps every entry is below 0.51p 2^n; the tables
// are reduced every kRenormF = 10 blocks, so entries stay below 522p < 2^50
// (exact) and the P, Q entering a product below 261p.  The running pair then
// stays below (0.574p, 1.148p): |a| |b| <= 1.148 * 261 p^2 < 300 p^2.  Returns
// plain residues in [0, p): the same ratio c1/c0 as run_chunk.
constexpr int kRenormF = 10;

template <int DEG>
__host__ __device__ __forceinline__ double f_pow(double s, const Fmod &f) {
    const double s2 = f_mulmod(s, s, f);
    return DEG == 3 ? f_mulmod(s2, s, f) : s2;
}

template <int DEG, int K>
__host__ __device__ __forceinline__ void run_chunk_blocked_f64(uint64_t s0, uint64_t n, uint64_t p, uint64_t &c0,
                                                               uint64_t &c1) {
    constexpr int DP = DEG * K;
    constexpr int DQ = DEG * (K - 1);
    Fmod f;
    f.p = (double)p;
    f.pinv = 1.0 / f.p;
    const uint64_t nb = n / K;
    double a0 = 1.0, a1 = 0.0;
    if (nb > 0) {
        double Pd[DP + 1], Qd[DQ + 1];
        // direct values P, Q at x = s0 + b K, b = 0..DP
WV_UNROLL
        for (int b = 0; b <= DP; b++) {
            double P = 1.0, Q = 0.0;
            for (int j = 0; j < K; j++) {
                const double u = f_pow<DEG>((double)(s0 + (uint64_t)b * K + j), f);
                Q = f_reduce(f_mulmod(Q, u, f) + P, f);
                P = f_mulmod(P, u, f);
            }
            Pd[b] = P;
            if (b <= DQ) Qd[b] = Q;
        }
        // forward differences at b = 0: entry i becomes Delta^i, reduced
WV_UNROLL
        for (int lev = 1; lev <= DP; lev++) {
WV_UNROLL
            for (int i = DP; i >= lev; i--) Pd[i] = f_reduce(Pd[i] - Pd[i - 1], f);
        }
WV_UNROLL
        for (int lev = 1; lev <= DQ; lev++) {
WV_UNROLL
            for (int i = DQ; i >= lev; i--) Qd[i] = f_reduce(Qd[i] - Qd[i - 1], f);
        }
        uint64_t b = 0;
        for (;;) {
            const uint64_t steps = nb - b < (uint64_t)kRenormF ? nb - b : (uint64_t)kRenormF;
            for (uint64_t k = 0; k < steps; k++) {
                const double n1 = f_mulmod(a0, Qd[0], f) + f_mulmod(a1, Pd[0], f);
                a0 = f_mulmod(a0, Pd[0], f);
                a1 = n1;
WV_UNROLL
                for (int i = 0; i < DP; i++) Pd[i] = opaque_f(Pd[i] + Pd[i + 1]);
WV_UNROLL
                for (int i = 0; i < DQ; i++) Qd[i] = opaque_f(Qd[i] + Qd[i + 1]);
            }
            b += steps;
            if (b >= nb) break;
WV_UNROLL
            for (int i = 0; i < DP; i++) Pd[i] = f_reduce(Pd[i], f);
WV_UNROLL
            for (int i = 0; i < DQ; i++) Qd[i] = f_reduce(Qd[i], f);
        }
    }
    for (uint64_t t = nb * K; t < n; t++) {
        const double u = f_pow<DEG>((double)(s0 + t), f);
        a1 = f_mulmod(a1, u, f) + a0;
        a0 = f_mulmod(a0, u, f);
        a1 = f_reduce(a1, f);
    }
    c0 = f_canon(a0, f);
    c1 = f_canon(a1, f);
}

// ---- blocked loop through the Taylor coefficients of F ------------------------
//
// With F(x) = prod_{j<K} (x + j) and g_k(x) = F^(k)(x) / k! (the coefficients
// of F(x + h) = sum_k g_k h^k), the block factor of run_chunk_blocked is
//   P = F^d,  Q = P sum_j (x + j)^-d,
// and the logarithmic derivatives of F give, as polynomial identities,
//   d = 2:  sum_j (x+j)^-2 = (F'^2 - F F'') / F^2,             Q = g1^2 - 2 g0 g2,
//   d = 3:  sum_j (x+j)^-3 = (F''' F^2 - 3 F F' F'' + 2 F'^3) / (2 F^3),
//           Q = 3 g3 g0^2 - 3 g0 g1 g2 + g1^3.
// So only g_0..g_d (degrees K..K-d in x) are stepped by finite differences
// with step K: (d+1)K - d(d+1)/2 additions per block instead of d(2K-1), for
// a few more products per block.  The g_k entering the products are reduced
// first (|g| < 0.51p), so every product stays within f_mulmod's bounds
// (|Q| < 4.1p, |a0 Q| < 2.4 p^2).  The tables themselves only need to stay
// exact integers: every entry is below 0.574p after a reduction and at most
// doubles per block, so for p < 2^b they are reduced every 53 - b blocks
// (0.574 2^53 < 2^53; 13 blocks at p < 2^40, 16 at p < 2^37).  Returns plain
// residues in [0, p) with the same ratio c1/c0 as run_chunk.

template <int DEG, int K>
__host__ __device__ __forceinline__ void run_chunk_logd(uint64_t s0, uint64_t n, uint64_t p, uint64_t &c0,
                                                        uint64_t &c1) {
    // table k holds g_k: K - k + 1 entries from offset k (K + 1) - k (k - 1) / 2
    static_assert(K >= DEG, "g_DEG must have degree >= 0");
    constexpr int NT = DEG + 1;
    constexpr int SZ = NT * (K + 1) - NT * (NT - 1) / 2;
    Fmod f;
    f.p = (double)p;
    f.pinv = 1.0 / f.p;
    const uint64_t nb = n / K;
    const uint64_t period = (uint64_t)(53 - (64 - __builtin_clzll(p)));   // blocks between reductions
    double a0 = 1.0, a1 = 0.0;
    if (nb > 0) {
        double G[SZ];
        // direct values g_k(x) at x = s0 + b K for b = 0..K - k, built in place:
        // prod_j (x + j + h) mod h^NT, one factor (all points at once) per j.
        // Table k only needs points the lower tables also hold (b <= K - k <
        // K - k + 2), so the update g_k <- a g_k + g_{k-1} runs from the top
        // table down.
WV_UNROLL
        for (int i = 0; i < SZ; i++) G[i] = 0.0;
WV_UNROLL
        for (int b = 0; b <= K; b++) G[b] = 1.0;
WV_NO_UNROLL
        for (int j = 0; j < K; j++) {
            const double xj = (double)(s0 + (uint64_t)j);
WV_UNROLL
            for (int k = NT - 1; k >= 0; k--) {
                const int off = k * (K + 1) - k * (k - 1) / 2;
                const int offl = (k - 1) * (K + 1) - (k - 1) * (k - 2) / 2;
                double a = xj;   // x + j at point b, stepped (no table of constants)
WV_UNROLL
                for (int b = 0; b <= K - k; b++) {
                    const double t = f_mulmod(a, G[off + b], f);
                    G[off + b] = k == 0 ? t : f_reduce(t + G[(k > 0 ? offl : 0) + b], f);
                    a = opaque_f(a + (double)K);
                }
            }
        }
        // forward differences of each table (entry i becomes Delta^i), reduced
WV_UNROLL
        for (int k = 0; k < NT; k++) {
            const int off = k * (K + 1) - k * (k - 1) / 2;
            const int deg = K - k;
WV_UNROLL
            for (int lev = 1; lev <= deg; lev++) {
WV_UNROLL
                for (int i = deg; i >= lev; i--) G[off + i] = f_reduce(G[off + i] - G[off + i - 1], f);
            }
        }
        uint64_t b = 0;
        for (;;) {
            const uint64_t steps = nb - b < period ? nb - b : period;
            for (uint64_t t = 0; t < steps; t++) {
                const double r0 = f_reduce(G[0], f);
                const double r1 = f_reduce(G[K + 1], f);
                const double r2 = f_reduce(G[2 * K + 1], f);
                double P, Q;
                if (DEG == 2) {
                    P = f_mulmod(r0, r0, f);
                    const double u = f_mulmod(r0, r2, f);
                    Q = f_mulmod(r1, r1, f) - (u + u);
                } else {
                    const double r3 = f_reduce(G[3 * K], f);
                    const double sq = f_mulmod(r0, r0, f);
                    P = f_mulmod(sq, r0, f);
                    const double A = f_mulmod(r3, sq, f);
                    const double C = f_mulmod(f_mulmod(r0, r1, f), r2, f);
                    const double E = f_mulmod(f_mulmod(r1, r1, f), r1, f);
                    const double D = A - C;
                    Q = (D + D + D) + E;
                }
                const double n1 = f_mulmod(a0, Q, f) + f_mulmod(a1, P, f);
                a0 = f_mulmod(a0, P, f);
                a1 = n1;
WV_UNROLL
                for (int k = 0; k < NT; k++) {
                    const int off = k * (K + 1) - k * (k - 1) / 2;
WV_UNROLL
                    for (int i = 0; i < K - k; i++) G[off + i] = opaque_f(G[off + i] + G[off + i + 1]);
                }
            }
            b += steps;
            if (b >= nb) break;
WV_UNROLL
            for (int i = 0; i < SZ; i++) G[i] = f_reduce(G[i], f);
        }
    }
    for (uint64_t t = nb * K; t < n; t++) {
        const double u = f_pow<DEG>((double)(s0 + t), f);
        a1 = f_mulmod(a1, u, f) + a0;
        a0 = f_mulmod(a0, u, f);
        a1 = f_reduce(a1, f);
    }
    c0 = f_canon(a0, f);
    c1 = f_canon(a1, f);
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
