// mont.hpp -- 64-bit Montgomery arithmetic mod an odd p < 2^40 for gfx950,
// built from 32x32->64 multiplies (v_mad_u64_u32 / v_mul_lo_u32 chains).
//
// Radix R = 2^64, reduced in two 32-bit word rounds (coarsely integrated
// operand scanning).  Values are kept "lazy": multiplication inputs may be
// < 4p, outputs are < 2p, and only the additive forward-difference state is
// kept canonical in [0, p).  The sums of the paper only ever need the ratio
// c1/c0 of a pair (Section 3, eqnComputeS), so a common power of R on both
// members of a pair is harmless; constants that enter a single residue are
// converted explicitly.
#pragma once
#include <cstdint>
#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define WV_UNROLL _Pragma("unroll")
#define WV_NO_UNROLL _Pragma("unroll 1")
#else
// Plain C++ build of the same arithmetic, for host-side unit tests.
#define __host__
#define __device__
#define __forceinline__ inline
#define WV_UNROLL
#define WV_NO_UNROLL
#endif

namespace wv {

struct Mont {
    uint64_t p;
    uint32_t p0, p1;   // 32-bit limbs of p; p1 < 2^8 because p < 2^40
    uint32_t ninv;     // -p^{-1} mod 2^32
};

__host__ __device__ __forceinline__ uint64_t mul32w(uint32_t a, uint32_t b) {
    return (uint64_t)a * (uint64_t)b;
}

// a * b * 2^-64 mod p (Montgomery product), output in [0, 2p).
// Preconditions (p < 2^40 odd): a < 4p, so a1 = a >> 32 < 2^10; b < 2^62; and
// a * b < p * 2^64.  Then the round-0 value is < 2^43, the round-1 value
// T1 = T0 + a0*b1 < 2^63, a1*b1 enters after the second division, and the
// result (ab + Mp)/2^64 < p + ab/2^64 < 2p.  With b < 4p as well this is the
// plain lazy Montgomery product; b may also be a value up to p * 2^21 that is
// only known modulo p (a finite-difference accumulator between reductions).
__host__ __device__ __forceinline__ uint64_t mmul(uint64_t a, uint64_t b, const Mont &m) {
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    // round 0: T = a*b0, q = T*ninv mod 2^32, T = (T + q p) / 2^32
    uint64_t t = mul32w(a0, b0);
    uint32_t q = (uint32_t)t * m.ninv;
    uint64_t x = mul32w(q, m.p0) + (uint32_t)t;          // == 0 mod 2^32, < 2^64
    uint64_t T = (t >> 32) + (x >> 32) + mul32w(a1, b0) + mul32w(q, m.p1);
    // round 1: the a0*b1 part shares the low word; a1*b1 sits one word higher
    // and is added after the division
    T += mul32w(a0, b1);
    q = (uint32_t)T * m.ninv;
    x = mul32w(q, m.p0) + (uint32_t)T;
    return (T >> 32) + (x >> 32) + mul32w(q, m.p1) + mul32w(a1, b1);
}

// x < 2p -> x mod p
__host__ __device__ __forceinline__ uint64_t red1(uint64_t x, uint64_t p) {
    return x >= p ? x - p : x;
}

// a, b in [0, p) -> a + b mod p in [0, p)
__host__ __device__ __forceinline__ uint64_t addm(uint64_t a, uint64_t b, uint64_t p) {
    uint64_t s = a + b;
    uint64_t t = s - p;
    return (int64_t)t < 0 ? s : t;
}

// a, b in [0, p) -> a - b mod p in [0, p)
__host__ __device__ __forceinline__ uint64_t subm(uint64_t a, uint64_t b, uint64_t p) {
    uint64_t d = a - b;
    return (int64_t)d < 0 ? d + p : d;
}

// -p^{-1} mod 2^32 by Newton iteration (p odd).
__host__ __device__ __forceinline__ uint32_t neg_inv32(uint32_t p0) {
    uint32_t inv = p0;                 // correct to 3 bits: p*p == 1 mod 8
    for (int i = 0; i < 5; i++) inv *= 2u - p0 * inv;
    return 0u - inv;
}

__host__ __device__ __forceinline__ Mont make_mont(uint64_t p) {
    Mont m;
    m.p = p;
    m.p0 = (uint32_t)p;
    m.p1 = (uint32_t)(p >> 32);
    m.ninv = neg_inv32(m.p0);
    return m;
}

// R mod p = 2^64 mod p
__host__ __device__ __forceinline__ uint64_t r_mod(uint64_t p) { return (0 - p) % p; }

// R^2 mod p from R mod p by 64 modular doublings.
__host__ __device__ __forceinline__ uint64_t r2_mod(uint64_t p) {
    uint64_t x = r_mod(p);
    for (int i = 0; i < 64; i++) x = addm(x, x, p);
    return x;
}

// Canonical Montgomery form x R mod p of x < p.
__host__ __device__ __forceinline__ uint64_t to_mont(uint64_t x, uint64_t r2, const Mont &m) {
    return red1(mmul(x, r2, m), m.p);
}

// Canonical x from a lazy Montgomery value xR (< 4p).
__host__ __device__ __forceinline__ uint64_t from_mont(uint64_t xr, const Mont &m) {
    return red1(mmul(xr, 1, m), m.p);
}

// Montgomery power: from aR (< 4p) and one = R mod p, returns a^e R (lazy, < 2p).
__host__ __device__ __forceinline__ uint64_t mpow(uint64_t ar, uint64_t e, uint64_t one, const Mont &m) {
    uint64_t r = one;
    for (int i = 63; i >= 0; i--) {
        r = mmul(r, r, m);
        if ((e >> i) & 1) r = mmul(r, ar, m);
    }
    return r;
}

// Pair product in F_p[z]/(z^2) (Section 3, eqnCombinePairs) on Montgomery
// values: (c0 + c1 z)(d0 + d1 z) = c0 d0 + (c0 d1 + c1 d0) z, each member
// scaled by R^-1.  Inputs c0, d0 < 2p and c1, d1 < 4p; outputs keep those bounds.
__host__ __device__ __forceinline__ void pair_mul(uint64_t &c0, uint64_t &c1, uint64_t d0, uint64_t d1,
                                                  const Mont &m) {
    uint64_t n1 = mmul(c0, d1, m) + mmul(c1, d0, m);
    c0 = mmul(c0, d0, m);
    c1 = n1;
}

}  // namespace wv
