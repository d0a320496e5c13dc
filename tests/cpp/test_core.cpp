// Host-side unit test of the device arithmetic (mont.hpp) and of the per-lane
// hot loop (sum_core.hpp) against unsigned __int128 products and %.
// Prints "OK <checks>" or the first failure.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>
#include "mont.hpp"
#include "step_share.hpp"
#include "sum_core.hpp"

using u128 = unsigned __int128;
using namespace wv;

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)((u128)a * b % p); }
static uint64_t powmod(uint64_t a, uint64_t e, uint64_t p) {
    uint64_t r = 1;
    a %= p;
    while (e) { if (e & 1) r = mulmod(r, a, p); a = mulmod(a, a, p); e >>= 1; }
    return r;
}

int main() {
    std::mt19937_64 rng(12345);
    // odd moduli (primality is not needed for the Montgomery identities)
    std::vector<uint64_t> ps = {11, 13, 101, 65537, 1000003, 998244353, 4294967291ull, 4294967311ull,
                                99999999977ull, 100000000003ull, (1ull << 40) - 87, (1ull << 40) - 1,
                                (1ull << 39) + 1, (1ull << 32) + 15, (1ull << 20) + 7, (1ull << 19) + 21};
    for (int i = 0; i < 40; i++) ps.push_back((rng() % ((1ull << 40) - 11)) | 1ull);
    long checks = 0;
    for (uint64_t p : ps) {
        if (p < 11) continue;
        Mont m = make_mont(p);
        if ((uint32_t)(m.ninv * (uint32_t)p) != 0xFFFFFFFFu) { printf("FAIL ninv p=%llu\n", (unsigned long long)p); return 1; }
        const uint64_t Rm = (uint64_t)(((u128)1 << 64) % p);
        const uint64_t R2 = mulmod(Rm, Rm, p);
        if (r_mod(p) != Rm || r2_mod(p) != R2) { printf("FAIL R p=%llu\n", (unsigned long long)p); return 1; }
        // R^-1 mod p via the extended identity: mmul(x, 1) == x R^-1
        auto check = [&](uint64_t a, uint64_t b) {
            // lazy inputs up to 4p
            uint64_t r = mmul(a, b, m);
            // r * R == a * b (mod p) and r < 2p
            uint64_t lhs = mulmod(r % p, Rm, p), rhs = mulmod(a % p, b % p, p);
            if (lhs != rhs || r >= 2 * p) {
                printf("FAIL mmul p=%llu a=%llu b=%llu r=%llu\n", (unsigned long long)p, (unsigned long long)a,
                       (unsigned long long)b, (unsigned long long)r);
                return false;
            }
            checks++;
            return true;
        };
        const uint64_t edge[] = {0, 1, 2, p - 1, p, p + 1, 2 * p - 1, 2 * p, 3 * p, 4 * p - 1, Rm, R2};
        for (uint64_t a : edge)
            for (uint64_t b : edge)
                if (!check(a, b)) return 1;
        for (int k = 0; k < 20000; k++) {
            uint64_t a = rng() % (4 * p), b = rng() % (4 * p);
            if (!check(a, b)) return 1;
        }
        // second operand up to p * 2^21 (unreduced difference accumulators)
        const uint64_t big = p << 21;
        const uint64_t bigs[] = {big - 1, big - p, (p << 15) + 12345, p << 8};
        for (uint64_t b : bigs)
            for (uint64_t a : edge)
                if (!check(a, b)) return 1;
        for (int k = 0; k < 20000; k++) {
            uint64_t a = rng() % (4 * p), b = rng() % big;
            if (!check(a, b)) return 1;
        }
        // addm / subm / to_mont / from_mont / mpow
        for (int k = 0; k < 2000; k++) {
            uint64_t a = rng() % p, b = rng() % p;
            if (addm(a, b, p) != (uint64_t)(((u128)a + b) % p)) { printf("FAIL addm\n"); return 1; }
            if (subm(a, b, p) != (uint64_t)(((u128)a + p - b) % p)) { printf("FAIL subm\n"); return 1; }
            uint64_t aR = to_mont(a, R2, m);
            if (aR != mulmod(a, Rm, p)) { printf("FAIL to_mont\n"); return 1; }
            if (from_mont(aR, m) != a) { printf("FAIL from_mont\n"); return 1; }
            uint64_t e = rng() % p;
            uint64_t pw = mpow(aR, e, Rm, m) % p;
            if (pw != mulmod(powmod(a, e, p), Rm, p)) { printf("FAIL mpow\n"); return 1; }
            checks += 5;
        }
        // pair product: ratio c1/c0 of a product equals the sum of the ratios
        for (int k = 0; k < 500; k++) {
            uint64_t c0 = 1 + rng() % (p - 1), c1 = rng() % (4 * p), d0 = 1 + rng() % (p - 1), d1 = rng() % (4 * p);
            uint64_t e0 = c0, e1 = c1;
            pair_mul(e0, e1, d0, d1, m);
            // e0 R == c0 d0, e1 R == c0 d1 + c1 d0
            if (mulmod(e0 % p, Rm, p) != mulmod(c0, d0, p) ||
                mulmod(e1 % p, Rm, p) != (mulmod(c0, d1 % p, p) + mulmod(c1 % p, d0, p)) % p ||
                e0 >= 2 * p || e1 >= 4 * p) {
                printf("FAIL pair_mul p=%llu\n", (unsigned long long)p);
                return 1;
            }
            checks++;
        }
    }
    // the hot loop: (c0, c1) of prod (z + s^deg) over s0 .. s0+n-1, written out
    for (uint64_t p : ps) {
        if (p < 11) continue;
        Mont m = make_mont(p);
        const uint64_t R2 = r2_mod(p), Rm = r_mod(p);
        for (int k = 0; k < 12; k++) {
            uint64_t s0 = 1 + rng() % (p - 1);
            uint64_t n = rng() % 300;
            if (k == 0) n = 0;
            if (k == 1) { s0 = p - 1; n = 1; }
            if (k == 2 && p > 1000) { s0 = p - 200; n = 199; }
            if (s0 + n > p) n = p - s0;   // keep every s in (0, p)
            for (int deg = 2; deg <= 3; deg++) {
                uint64_t c0, c1;
                if (deg == 3) run_chunk<3>(s0, n, m, R2, Rm, c0, c1);
                else run_chunk<2>(s0, n, m, R2, Rm, c0, c1);
                uint64_t e0 = 1, e1 = 0;
                for (uint64_t s = s0; s < s0 + n; s++) {
                    uint64_t u = powmod(s, deg, p);
                    e1 = (mulmod(e1, u, p) + e0) % p;
                    e0 = mulmod(e0, u, p);
                }
                if (c0 % p != e0 || c1 % p != e1 || c0 >= 2 * p || c1 >= 4 * p) {
                    printf("FAIL run_chunk<%d> p=%llu s0=%llu n=%llu\n", deg, (unsigned long long)p,
                           (unsigned long long)s0, (unsigned long long)n);
                    return 1;
                }
                checks++;
            }
        }
    }
    // the blocked hot loop gives the same pair as the one-term loop
    for (uint64_t p : ps) {
        if (p < 11) continue;
        Mont m = make_mont(p);
        const uint64_t R2 = r2_mod(p), Rm = r_mod(p);
        for (int k = 0; k < 6; k++) {
            uint64_t s0 = 1 + rng() % (p - 1);
            uint64_t n = rng() % 700;
            if (k == 0) n = 0;
            if (k == 1) n = 5;
            if (k == 2) n = 16 * 20 * 3 + 77;   // several reduction periods at p near 2^40
            if (k == 4) n = 32 * 37 * 2 + 31;   // periods of the Taylor-coefficient tables (53 - b blocks)
            if (k == 3) n = 8 * 13 + 8;         // a period boundary at K = 8, p near 2^40
            if (s0 + n > p) n = p - s0;
            uint64_t r0, r1;
            uint64_t x0, x1;
            run_chunk<3>(s0, n, m, R2, Rm, r0, r1);
            // blocked loop: plain residues in [0, p), the same ratio as run_chunk
            auto cmpf = [&](uint64_t y0, uint64_t y1, const char *what) {
                // y1 / y0 == r1 / r0 (mod p)  <=>  y1 r0 == r1 y0; c0 vanishes for
                // both or neither (only possible for the composite test moduli)
                if (y0 >= p || y1 >= p || (y0 == 0) != (r0 % p == 0) ||
                    mulmod(y1, r0 % p, p) != mulmod(r1 % p, y0, p)) {
                    printf("FAIL %s p=%llu s0=%llu n=%llu\n", what, (unsigned long long)p, (unsigned long long)s0,
                           (unsigned long long)n);
                    return false;
                }
                checks++;
                return true;
            };
            // block count / reduction period shared with other lanes: all, some or
            // none of this lane's blocks, the lane's own period or a shorter one
            const uint64_t own_period = 53 - (64 - __builtin_clzll(p));
            const uint64_t psh = k % 2 ? own_period : 7;
            auto nbsh_of = [&](uint64_t K) { return k % 3 == 0 ? n / K : k % 3 == 1 ? n / K / 3 : 0; };
            if (p < (1ull << 40)) {
                run_chunk_logd<3, 3>(s0, n, p, nbsh_of(3), psh, x0, x1); if (!cmpf(x0, x1, "B logd k3")) return 1;
                run_chunk_logd<3, 4>(s0, n, p, nbsh_of(4), psh, x0, x1); if (!cmpf(x0, x1, "B logd k4")) return 1;
                run_chunk_logd<3, 8>(s0, n, p, nbsh_of(8), psh, x0, x1); if (!cmpf(x0, x1, "B logd k8")) return 1;
                run_chunk_logd<3, 12>(s0, n, p, nbsh_of(12), psh, x0, x1); if (!cmpf(x0, x1, "B logd k12")) return 1;
                run_chunk_logd<3, 16>(s0, n, p, nbsh_of(16), psh, x0, x1); if (!cmpf(x0, x1, "B logd k16")) return 1;
                run_chunk_logd<3, 20>(s0, n, p, nbsh_of(20), psh, x0, x1); if (!cmpf(x0, x1, "B logd k20")) return 1;
                run_chunk_logd<3, 24>(s0, n, p, nbsh_of(24), psh, x0, x1); if (!cmpf(x0, x1, "B logd k24")) return 1;
                run_chunk_logd<3, 26>(s0, n, p, nbsh_of(26), psh, x0, x1); if (!cmpf(x0, x1, "B logd k26")) return 1;
                run_chunk_logd<3, 28>(s0, n, p, nbsh_of(28), psh, x0, x1); if (!cmpf(x0, x1, "B logd k28")) return 1;
            }
            run_chunk<2>(s0, n, m, R2, Rm, r0, r1);
            if (p < (1ull << 40)) {
                run_chunk_logd<2, 2>(s0, n, p, nbsh_of(2), psh, x0, x1); if (!cmpf(x0, x1, "E logd k2")) return 1;
                run_chunk_logd<2, 4>(s0, n, p, nbsh_of(4), psh, x0, x1); if (!cmpf(x0, x1, "E logd k4")) return 1;
                run_chunk_logd<2, 8>(s0, n, p, nbsh_of(8), psh, x0, x1); if (!cmpf(x0, x1, "E logd k8")) return 1;
                run_chunk_logd<2, 16>(s0, n, p, nbsh_of(16), psh, x0, x1); if (!cmpf(x0, x1, "E logd k16")) return 1;
                run_chunk_logd<2, 24>(s0, n, p, nbsh_of(24), psh, x0, x1); if (!cmpf(x0, x1, "E logd k24")) return 1;
                run_chunk_logd<2, 28>(s0, n, p, nbsh_of(28), psh, x0, x1); if (!cmpf(x0, x1, "E logd k28")) return 1;
                run_chunk_logd<2, 32>(s0, n, p, nbsh_of(32), psh, x0, x1); if (!cmpf(x0, x1, "E logd k32")) return 1;
                run_chunk_logd<2, 34>(s0, n, p, nbsh_of(34), psh, x0, x1); if (!cmpf(x0, x1, "E logd k34")) return 1;
                run_chunk_logd<2, 36>(s0, n, p, nbsh_of(36), psh, x0, x1); if (!cmpf(x0, x1, "E logd k36")) return 1;
            }
        }
        // f_mulmod / f_reduce: exact at the bounds the loop relies on
        if (p < (1ull << 40)) {
            Fmod f;
            f.p = (double)p;
            f.pinv = 1.0 / f.p;
            auto smod = [&](__int128 v) { __int128 r = v % (__int128)p; return (uint64_t)(r < 0 ? r + p : r); };
            // |r| <= p/2 + |ab| 2^-52 (plus rounding slack) for |ab| < 2^51 p
            auto chkm = [&](int64_t a, int64_t b, double bound) {
                const double r = f_mulmod((double)a, (double)b, f);
                const __int128 want = (__int128)a * b;
                if (r != std::floor(r) || std::fabs(r) > bound * f.p || smod((__int128)(int64_t)r) != smod(want)) {
                    printf("FAIL f_mulmod p=%llu a=%lld b=%lld r=%.1f\n", (unsigned long long)p, (long long)a,
                           (long long)b, r);
                    return false;
                }
                checks++;
                return true;
            };
            // residues and running pair: |a| <= 2.3p (unreduced set-up entries,
            // the pair's c1), |b| <= 5.6p (Q of the s^-3 loop)
            const int64_t A = (int64_t)(2.3 * (double)p), B = (int64_t)(5.6 * (double)p);
            const int64_t ea[] = {0, 1, -1, A, -A, (int64_t)p / 2, -(int64_t)p / 2, (int64_t)p - 1};
            const int64_t eb[] = {0, 1, -1, B, -B, B - 1, (int64_t)p, -(int64_t)p, (int64_t)(0.51 * (double)p)};
            for (int64_t a : ea)
                for (int64_t b : eb)
                    if (!chkm(a, b, 0.574)) return 1;
            for (int k = 0; k < 20000; k++) {
                const int64_t a = (int64_t)(rng() % (2 * (uint64_t)A + 1)) - A;
                const int64_t b = (int64_t)(rng() % (2 * (uint64_t)B + 1)) - B;
                if (!chkm(a, b, 0.574)) return 1;
            }
            // a table value entry entering a product unreduced, 53 - bitlen(p)
            // blocks after a reduction at most (|G| <= 0.574 p 2^(52 - bitlen)),
            // times a reduced operand (|x| <= 0.574 p): |r| <= 0.83 p
            const int bl = 64 - __builtin_clzll(p);
            const int64_t Gm = (int64_t)std::ldexp(0.574 * (double)p, 52 - bl), X = (int64_t)(0.574 * (double)p);
            const int64_t eg[] = {Gm, -Gm, Gm - 1, Gm / 3, 1};
            const int64_t ex[] = {X, -X, X - 1, 1, -1, 0};
            for (int64_t g : eg)
                for (int64_t x : ex)
                    if (!chkm(g, x, 0.83)) return 1;
            for (int k = 0; k < 20000; k++) {
                const int64_t g = (int64_t)(rng() % (2 * (uint64_t)Gm + 1)) - Gm;
                const int64_t x = (int64_t)(rng() % (2 * (uint64_t)X + 1)) - X;
                if (!chkm(g, x, 0.83)) return 1;
            }
            for (int k = 0; k < 20000; k++) {
                const int64_t x = (int64_t)(rng() % ((1ull << 54) + 1)) - (int64_t)(1ull << 53);
                const double r = f_reduce((double)x, f);
                if (std::fabs(r) > 0.51 * f.p || smod((__int128)(int64_t)r) != smod(x)) {
                    printf("FAIL f_reduce p=%llu x=%lld\n", (unsigned long long)p, (long long)x);
                    return 1;
                }
                if (f_canon((double)x, f) != smod(x)) { printf("FAIL f_canon\n"); return 1; }
                checks += 2;
            }
        }
    }
    // chunk -> sum lookup skips empty sums
    {
        const uint64_t off[] = {0, 0, 3, 3, 3, 7, 8, 8};   // 7 sums, total 8 chunks
        const uint32_t want[] = {1, 1, 1, 4, 4, 4, 4, 5};
        for (uint64_t c = 0; c < 8; c++)
            if (find_seg(off, 7, c) != want[c]) { printf("FAIL find_seg %llu\n", (unsigned long long)c); return 1; }
        checks += 8;
    }
    // floor(len / C) through a rounded reciprocal: multiples of C, their
    // neighbours and random lengths up to 2^41, chunk sizes from 64 to 2^32
    {
        std::vector<uint64_t> cs = {1, 3, 64, 192, 4096, 65536, 680000, 680064, (1ull << 20) + 64, (1ull << 32)};
        for (int i = 0; i < 200; i++) cs.push_back(((rng() % (1ull << 26)) + 1) * 64);
        for (uint64_t C : cs) {
            const double inv = 1.0 / (double)C;
            auto one = [&](uint64_t len) {
                if (full_chunks(len, C, inv) != len / C) {
                    printf("FAIL full_chunks len=%llu C=%llu\n", (unsigned long long)len, (unsigned long long)C);
                    return false;
                }
                checks++;
                return true;
            };
            for (int i = 0; i < 200; i++) {
                const uint64_t k = (uint64_t)(rng() % ((1ull << 41) / C + 1));
                for (uint64_t len : {k * C, k * C + 1, k * C + C - 1, k ? k * C - 1 : 0, (uint64_t)(rng() % (1ull << 41))})
                    if (!one(len)) return 1;
            }
            for (uint64_t len : {(1ull << 40) - 1, (1ull << 40), (1ull << 41) - 1})
                if (!one(len)) return 1;
        }
    }
    // f_mulmod_add at the edges of its range: |ab| < 2^51 p, |e| < 2^50
    {
        std::vector<uint64_t> qs = {11, 13, 53, 1000003, 99999999977ull, (1ull << 40) - 87, (1ull << 39) + 1};
        for (int i = 0; i < 40; i++) qs.push_back((rng() % ((1ull << 40) - 11)) | 1ull);
        for (uint64_t p : qs) {
            Fmod f;
            f.p = (double)p;
            f.pinv = 1.0 / f.p;
            const int64_t E = (int64_t)(1ull << 50) - 1;
            const int64_t A = (int64_t)(0.51 * (double)p);               // a reduced entry
            const int64_t B = (int64_t)std::min<uint64_t>((1ull << 41) - 1, (uint64_t)(((u128)1 << 51) * p / (A + 1) - 1));
            auto chk = [&](int64_t a, int64_t b, int64_t e) {
                const double r = f_mulmod_add((double)a, (double)b, (double)e, f);
                const __int128 want = ((__int128)a * b + e) % (__int128)p;
                const __int128 got = (__int128)(int64_t)r % (__int128)p;
                if (std::fabs(r) >= 0.51 * f.p || r != std::floor(r) || (got - want) % (__int128)p != 0) {
                    printf("FAIL f_mulmod_add p=%llu a=%lld b=%lld e=%lld\n", (unsigned long long)p, (long long)a,
                           (long long)b, (long long)e);
                    return false;
                }
                checks++;
                return true;
            };
            for (int64_t a : {A, -A, (int64_t)1, (int64_t)0})
                for (int64_t b : {B, -B, B - 1, (int64_t)1})
                    for (int64_t e : {E, -E, (int64_t)0, (int64_t)p, -(int64_t)p})
                        if (!chk(a, b, e)) return 1;
            for (int i = 0; i < 20000; i++) {
                const int64_t a = (int64_t)(rng() % (2 * (uint64_t)A + 1)) - A;
                const int64_t b = (int64_t)(rng() % (2 * (uint64_t)B + 1)) - B;
                const int64_t e = (int64_t)(rng() % (2 * (uint64_t)E + 1)) - E;
                if (!chk(a, b, e)) return 1;
            }
        }
    }
    // the plan's interval endpoints and limb reductions against 128-bit / and %
    {
        std::vector<uint64_t> qs = {11, 13, 1000003, 99999999977ull, 100000000003ull, (1ull << 40) - 87,
                                    (1ull << 40) - 1, (1ull << 39) + 1, (1ull << 32) + 15};
        for (int i = 0; i < 200; i++) qs.push_back((rng() % ((1ull << 40) - 11)) | 1ull);
        std::vector<std::pair<uint64_t, uint64_t>> fr = {{0, 1}, {1, 2}, {1, 3}, {2, 5}, {1, 1}, {491, 960400},
                                                         {127, 246960}, {9887, 19208000}, {1, 1920},
                                                         {(1ull << 62) - 1, (1ull << 62)}, {1, (1ull << 63) - 1},
                                                         {(1ull << 63) - 2, (1ull << 63) - 1}};
        for (int i = 0; i < 300; i++) {
            const uint64_t b = (rng() >> (rng() % 63)) | 1ull;
            fr.push_back({rng() % (b + 1), b});
        }
        for (uint64_t p : qs) {
            for (auto [a, b] : fr) {
                const uint64_t want = (uint64_t)((u128)a * p / b);
                if (floor_mul_div(a, p, b) != want) {
                    printf("FAIL floor_mul_div a=%llu p=%llu b=%llu\n", (unsigned long long)a, (unsigned long long)p,
                           (unsigned long long)b);
                    return 1;
                }
                if (a >= 1) {
                    const uint64_t want1 = (uint64_t)(((u128)a * p - 1) / b);
                    if (floor_mul_minus1_div(a, p, b) != want1) {
                        printf("FAIL floor_mul_minus1_div a=%llu p=%llu b=%llu\n", (unsigned long long)a,
                               (unsigned long long)p, (unsigned long long)b);
                        return 1;
                    }
                }
                checks += 2;
            }
            for (uint64_t r : {(uint64_t)0, (uint64_t)1, p - 1, p / 2, rng() % p})
                for (uint32_t limb : {0u, 1u, 0xFFFFFFFFu, (uint32_t)rng()}) {
                    const uint64_t want = (uint64_t)((((u128)r << 32) | limb) % p);
                    if (shift_in_limb(r, limb, p) != want) {
                        printf("FAIL shift_in_limb r=%llu limb=%u p=%llu\n", (unsigned long long)r, limb,
                               (unsigned long long)p);
                        return 1;
                    }
                    checks++;
                }
        }
    }
    // Server step composition: the cap, the budget, the even share, at least
    // one prime, and no prime left out that the budget and the cap allow.
    {
        std::uniform_real_distribution<double> lg(0.0, 1.0);
        auto fail = [](const char *what, int t) {
            printf("FAIL step_share %s case %d\n", what, t);
            return 1;
        };
        for (int t = 0; t < 20000; t++) {
            const size_t n = 1 + rng() % 40;
            const double step_terms = std::ldexp(1.0, 20 + (int)(rng() % 21));
            const uint64_t ns_choice[] = {1, 12, 61597, (1ull << 23) + 5, 1 + rng() % 100000};
            const uint64_t NS = ns_choice[rng() % 5];
            std::vector<ShareReq> c(n);
            for (auto &r : c) {
                r.left = (rng() % 3 == 0) ? 1 : 1 + rng() % ((rng() % 2) ? 100 : 65536);
                r.tpp = std::pow(10.0, 3.0 + 8.0 * lg(rng));
            }
            std::sort(c.begin(), c.end(),
                      [](const ShareReq &a, const ShareReq &b) { return (double)a.left * a.tpp < (double)b.left * b.tpp; });
            std::vector<uint32_t> give(n, 0xDEADu);
            const uint64_t nq = step_share(c.data(), n, step_terms, NS, give.data());
            const uint64_t cap = ((double)c[0].left * c[0].tpp * 8.0 <= step_terms) ? (1ull << 22) : (1ull << 23);
            const uint64_t max_q = std::max<uint64_t>(1, cap / NS);
            uint64_t sum = 0;
            double terms = 0;
            for (size_t k = 0; k < n; k++) {
                if (give[k] > c[k].left) return fail("more than left", t);
                sum += give[k];
                terms += give[k] * c[k].tpp;
            }
            if (sum != nq) return fail("count", t);
            if (nq < 1 || nq > max_q) return fail("cap", t);
            if (nq > 1 && terms > step_terms * (1 + 1e-9)) return fail("budget", t);
            if (nq < max_q) {
                for (size_t k = 0; k < n; k++) {
                    const uint64_t even = (uint64_t)(step_terms / (double)n / c[k].tpp);
                    if (give[k] < std::min<uint64_t>(c[k].left, even)) return fail("even share", t);
                }
                for (size_t k = 0; k < n; k++)
                    if (give[k] < c[k].left) {
                        if (step_terms - terms >= c[k].tpp * (1 + 1e-9)) return fail("left out", t);
                        break;
                    }
            }
            checks += 5;
        }
        // a single prime near 1e11 beside a long interval: the cap halves
        // (68 primes of 61,597 sums), and without it the step reaches 136
        std::vector<ShareReq> c = {{1, 4.9e9}, {40000, 4.9e9}};
        std::vector<uint32_t> give(2);
        if (step_max_primes(c[0], std::ldexp(1.0, 38), 61597) != 68) return fail("small cap", -1);
        if (step_max_primes(c[1], std::ldexp(1.0, 38), 61597) != 136) return fail("full cap", -1);
        const uint64_t nq = step_share(c.data(), 2, std::ldexp(1.0, 45), 61597, give.data());
        if (nq != 68 || give[0] != 1 || give[1] != 67) return fail("fixed case", -1);
        // one prime over the whole budget still makes a step of one prime
        std::vector<ShareReq> big = {{3, 1e12}};
        if (step_share(big.data(), 1, std::ldexp(1.0, 38), 61597, give.data()) != 1 || give[0] != 1)
            return fail("oversized prime", -1);
        checks += 6;
    }
    printf("OK %ld\n", checks);
    return 0;
}
