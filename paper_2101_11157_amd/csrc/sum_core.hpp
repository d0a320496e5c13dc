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

// x unchanged, but hidden from the optimiser's recurrence analysis: the chain
// of difference-table additions is otherwise recognised as a polynomial
// recurrence and the values after the loop rewritten as closed forms with
// binomial coefficients, which costs hundreds of registers.
__host__ __device__ __forceinline__ double opaque_f(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    asm("" : "+v"(x));
#endif
    return x;
}

// ---- the blocked loop in double precision ------------------------------------
//
// Residues held as integer-valued doubles, signed and lazily reduced, for p <
// 2^40.  One modular product of integers a, b is six full-rate f64 operations:
//   h = ab rounded;  l = fma(a, b, -h) = ab - h exactly (an error-free product);
//   q = the integer nearest h * (1/p) (fma with 1.5 * 2^52, then subtract it);
//   r = fma(-q, p, h) + l.
// With |ab| < 2^51 p: |h / p| < 2^51, so the rounding trick applies;
// |q - h/p| <= 1/2 + |h| 2^-53 / p, so h - qp is an integer of magnitude at
// most p/2 + |h| 2^-53 < p and the fma computes it exactly; l is an integer with
// |l| <= |h| 2^-53; hence r = ab - qp exactly, r == ab (mod p), and
// |r| <= p/2 + |ab| 2^-52.  For residues (|ab| <= 300 p^2, p < 2^40) that is
// below p/2 + 600 p 2^-13 <= 0.574 p.
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

// a b + e for integers a, b, e with |ab| < 2^51 p and |e| < 2^50: r == ab + e
// (mod p), |r| < 0.51p, exactly, in eight operations.  As f_mulmod, with e
// added to the rounded product before the quotient is taken and to the
// exact remainder after: h - qp is an integer below 2^51 (the fma is exact),
// and r = ab + e - qp with |r| <= p/2 + 2^-52 (|h| + |h + e|) < 0.51p.
__host__ __device__ __forceinline__ double f_mulmod_add(double a, double b, double e, const Fmod &f) {
    const double h = a * b;
    const double l = fma(a, b, -h);
    const double q = fma(h + e, f.pinv, kRound) - kRound;
    return (fma(-q, f.p, h) + l) + e;
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

// s^DEG mod p for one s in [0, 2p): the terms after the last full block
template <int DEG>
__host__ __device__ __forceinline__ double f_pow(double s, const Fmod &f) {
    const double s2 = f_mulmod(s, s, f);
    return DEG == 3 ? f_mulmod(s2, s, f) : s2;
}

// ---- blocked loop through the Taylor coefficients of F ------------------------
//
// Blocked form of eqnComputeS.  For a block of K consecutive s starting at x,
//   prod_{j<K} (z + (x+j)^d) = P + Q z + O(z^2),
//   P = prod_j (x+j)^d,   Q = P sum_j (x+j)^-d,
// and each block is folded into the running pair with the pair product of
// eqnCombinePairs: (c0, c1) <- (c0 P, c0 Q + c1 P).  With F(x) = prod_{j<K}
// (x + j) and g_k(x) = F^(k)(x) / k! (the coefficients of F(x + h) =
// sum_k g_k h^k), P = g0^d, and the logarithmic derivatives of F give Q as
// polynomial identities:
//   d = 2:  sum_j (x+j)^-2 = (F'^2 - F F'') / F^2,             Q = g1^2 - 2 g0 g2,
//   d = 3:  sum_j (x+j)^-3 = (F''' F^2 - 3 F F' F'' + 2 F'^3) / (2 F^3),
//           Q = 3 g3 g0^2 - 3 g0 g1 g2 + g1^3 = 3 g0^2 g3 + g1 (g1^2 - 3 g0 g2).
// So only g_0..g_d (degrees K..K-d in x) are stepped by finite differences
// along x = s0, s0 + K, ...: (d+1)K - d(d+1)/2 additions per block, where
// stepping P and Q themselves (degrees dK and d(K-1)) would take d(2K-1), for
// a few more products per block.
//
// Bounds.  After a reduction (and in fresh tables) every table entry is
// below 0.51p, and after t blocks entry i is sum_m C(t, m) D_{i+m} < 0.51p
// 2^t < 0.574p 2^t.  For p < 2^b (b <= 40) the
// tables are reduced every 53 - b >= 13 blocks (16 at p < 2^37), so they stay
// exact integers (0.574 2^53 < 2^53), and a value entry used in a product (at
// most 52 - b blocks after a reduction) is below 0.574 2^52.  g0 and g1 are
// reduced first (|r| < 0.51p); g2 and g3 enter unreduced, each times a reduced
// operand or a product of two (|x| < 0.574p), so |ab| < 0.33 p 2^52 = 2^50.4 p,
// inside f_mulmod's exact range (|ab| < 2^51 p), with |result| < 0.83p.  For
// d = 3, g1^2 - 3 g0 g2 is an exact integer below 3.1p, times g1 below 1.6p^2;
// then |Q| < 3.0p (d = 3) or 2.3p (d = 2) (the multiply-adds are exact), and
// |a0 Q| < 1.8 p^2.  Returns plain residues in [0, p) with the same ratio
// c1/c0 as run_chunk.
//
// nb_shared, period_shared: a block count and a reduction period that every
// lane of the calling wave shares, at most this lane's n / K and 53 - b (the
// caller's minima over the wave).  The first nb_shared blocks then run under
// wave-uniform loop control; the result does not depend on them.

template <int DEG, int K>
__host__ __device__ __forceinline__ void run_chunk_logd(uint64_t s0, uint64_t n, uint64_t p, uint64_t nb_shared,
                                                        uint64_t period_shared, uint64_t &c0, uint64_t &c1) {
    // table k holds g_k: K - k + 1 entries from offset k (K + 1) - k (k - 1) / 2
    static_assert(K >= DEG, "g_DEG must have degree >= 0");
    constexpr int NT = DEG + 1;
    constexpr int SZ = NT * (K + 1) - NT * (NT - 1) / 2;
    Fmod f;
    f.p = (double)p;
    f.pinv = 1.0 / f.p;
    const uint64_t nb = n / K;
    const uint64_t period = (uint64_t)(53 - (64 - __builtin_clzll(p)));   // blocks between reductions
    // The terms after the last full block go first (the pair product
    // commutes), so that s0 and n are dead while the tables are live.
    double a0 = 1.0, a1 = 0.0;
    for (uint64_t t = nb * K; t < n; t++) {
        const double u = f_pow<DEG>((double)(s0 + t), f);
        a1 = f_mulmod(a1, u, f) + a0;
        a0 = f_mulmod(a0, u, f);
        a1 = f_reduce(a1, f);
    }
    if (nb > 0) {
        double G[SZ];
        // The difference tables straight from the product.  With x = s0 + K t,
        //   F(x + h) = prod_{j<K} (a_j + K t + h),  a_j = s0 + j,
        // written as sum_{m,k} c_{m,k} C(t, m) h^k (k <= DEG, binomial
        // coefficients of t) has c_{m,k} = Delta^m g_k(s0) (Newton's forward
        // formula, step 1 in t): entry m of table k.  One more factor uses
        // (a + K t) C(t, m) = (a + K m) C(t, m) + K (m + 1) C(t, m + 1), so
        //   c_{m,k} <- (a + K m) c_{m,k} + K m c_{m-1,k} + c_{m,k-1}.
        // Tables from the top down and entries from the highest down read
        // only old values.  After J factors c_{m,k} = 0 for m > J - k, so
        // each factor updates only the blocks of four entries that can be
        // nonzero (a wave-uniform test).  Every entry stays reduced: the
        // other terms, K m (c_{m,k} + c_{m-1,k}) + c_{m,k-1}, are an exact
        // integer below 2^10 p < 2^50, added into the modular product a_j c
        // (|a_j c| < 2^41 p) by f_mulmod_add, which leaves it below 0.51 p.
        // About (DEG + 1) K^2 / 2 updates of 10 operations, against (DEG + 1)
        // K^2 products for the values at K + 1 points and the differencing
        // after them.
WV_UNROLL
        for (int i = 0; i < SZ; i++) G[i] = 0.0;
        G[0] = 1.0;
WV_NO_UNROLL
        for (int j = 0; j < K; j++) {
            const double aj = (double)(s0 + (uint64_t)j);
WV_UNROLL
            for (int k = NT - 1; k >= 0; k--) {
                const int off = k * (K + 1) - k * (k - 1) / 2;
                const int offl = (k - 1) * (K + 1) - (k - 1) * (k - 2) / 2;
WV_UNROLL
                for (int mb = (K - k) / 4; mb >= 0; mb--) {
                    if (4 * mb > j + 1 - k) continue;   // entries still zero
WV_UNROLL
                    for (int m = (4 * mb + 3 < K - k ? 4 * mb + 3 : K - k); m >= 4 * mb; m--) {
                        // (a_j + K m) c as a_j c (one product) plus K m c (exact):
                        // a single per-lane multiplier instead of one per m
                        const double km = (double)(K * m);
                        double e = k > 0 ? G[(k > 0 ? offl : 0) + m] : 0.0;
                        if (m > 0) e = fma(G[off + m - 1], km, fma(G[off + m], km, e));
                        G[off + m] = f_mulmod_add(G[off + m], aj, e, f);
                    }
                }
            }
        }
        // one block: fold P, Q into the running pair, step every table once
        auto step = [&]() {
            // g0 and g1 are squared, so they are reduced; g2 and g3 only meet
            // reduced partners and enter unreduced
            const double r0 = f_reduce(G[0], f);
            const double r1 = f_reduce(G[K + 1], f);
            const double r2 = G[2 * K + 1];
            double P, Q;
            if (DEG == 2) {
                // Q = g1^2 - 2 g0 g2 (as two additions: measured faster here
                // than one exact multiply-add)
                P = f_mulmod(r0, r0, f);
                const double u = f_mulmod(r0, r2, f);
                Q = f_mulmod(r1, r1, f) - (u + u);
            } else {
                // Q = 3 g0^2 g3 + g1 (g1^2 - 3 g0 g2): six products for P and Q
                const double r3 = G[3 * K];
                const double sq = f_mulmod(r0, r0, f);
                P = f_mulmod(sq, r0, f);
                const double A = f_mulmod(r3, sq, f);
                const double t = f_mulmod(r0, r2, f);
                const double u = fma(t, -3.0, f_mulmod(r1, r1, f));
                Q = fma(A, 3.0, f_mulmod(r1, u, f));
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
        };
        auto renorm = [&]() {
WV_UNROLL
            for (int i = 0; i < SZ; i++) G[i] = f_reduce(G[i], f);
        };
        // the first nb_shared blocks, reduced every period_shared blocks: the
        // same trip counts for every lane of a wave
        const uint64_t nbs = period_shared > 0 ? nb_shared : 0;
        const uint64_t ps = period_shared;
        uint64_t b = 0;
        while (b < nbs) {
            const uint64_t steps = nbs - b < ps ? nbs - b : ps;
            for (uint64_t t = 0; t < steps; t++) step();
            b += steps;
            renorm();
        }
        // this lane's remaining blocks
        while (b < nb) {
            const uint64_t steps = nb - b < period ? nb - b : period;
            for (uint64_t t = 0; t < steps; t++) step();
            b += steps;
            if (b >= nb) break;
            renorm();
        }
    }
    c0 = f_canon(a0, f);
    c1 = f_canon(a1, f);
}

// floor(len / C) for len < 2^53 and 1 <= C < 2^53, given invC = 1/C rounded
// to double: len and len * invC carry relative errors of at most 2^-53 each,
// so the product is within len/C * 2^-52 < 2 of len/C and its integer part is
// off by at most one, which the two comparisons correct.
__host__ __device__ __forceinline__ uint64_t full_chunks(uint64_t len, uint64_t C, double invC) {
    uint64_t q = (uint64_t)((double)len * invC);
    if (q * C > len) q--;
    else if ((q + 1) * C <= len) q++;
    return q;
}

// floor(x / b) for b >= 1 and a quotient below 2^52, from `est`, a double
// within a few units of x / b: two exact 128-bit comparisons move it onto the
// quotient (software 128-bit division is a long call on the GPU; these are a
// few multiplies).
__host__ __device__ __forceinline__ uint64_t quot_from_estimate(unsigned __int128 x, uint64_t b, double est) {
    uint64_t q = est > 0.0 ? (uint64_t)est : 0;
    while ((unsigned __int128)q * b > x) q--;
    while ((unsigned __int128)(q + 1) * b <= x) q++;
    return q;
}

// floor(a p / b) for a, b < 2^63 and a p / b < 2^52 (the endpoints of the
// open intervals of eqnDefnS): the double estimate a * p / b carries a
// relative error of at most 5 * 2^-53, under one unit.
__host__ __device__ __forceinline__ uint64_t floor_mul_div(uint64_t a, uint64_t p, uint64_t b) {
    return quot_from_estimate((unsigned __int128)a * p, b, (double)a * (double)p / (double)b);
}

// floor((a p - 1) / b) for a >= 1, as floor_mul_div.
__host__ __device__ __forceinline__ uint64_t floor_mul_minus1_div(uint64_t a, uint64_t p, uint64_t b) {
    return quot_from_estimate((unsigned __int128)a * p - 1, b, (double)a * (double)p / (double)b);
}

// (r 2^32 + limb) mod p for r < p < 2^40: one step of reducing an integer
// given as base-2^32 limbs, most significant first.  The quotient is below
// 2^32 and its double estimate is within one unit.
__host__ __device__ __forceinline__ uint64_t shift_in_limb(uint64_t r, uint32_t limb, uint64_t p) {
    const unsigned __int128 x = ((unsigned __int128)r << 32) | limb;
    const uint64_t q = quot_from_estimate(x, p, ((double)r * 4294967296.0 + (double)limb) / (double)p);
    return (uint64_t)(x - (unsigned __int128)q * p);
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
