/*
 * wv_oracle.c -- plain, slow CPU oracle for B_{p-3} mod p and E_{p-3} mod p.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header
 * or table with the HIP product path: every routine here is written from the
 * paper (Booker, Hathi, Mossinghoff, Trudgian, "Wolstenholme and Vandiver
 * primes", arXiv:2101.11157) with unsigned __int128 products and the C `%`
 * operator, and nothing is blocked, fused or reordered beyond what the cited
 * definition states.
 *
 * Contents
 *   orc_interval          endpoints of the open interval x*p < s < y*p
 *                         (Section 2, definition of S_l, eqnDefnS)
 *   orc_sum_direct        sum of (+-1)^s s^-l, one modular inverse per term
 *                         (eqnDefnS written out)
 *   orc_sum_poly          the same sum by the polynomial trick of Section 3:
 *                         c0,c1 of prod(z + s^l), S = c1/c0 (eqnComputeS),
 *                         pieces combined by eqnCombinePairs
 *   orc_congruence        L^-1 * sum c_i S(x_i,y_i) mod p for one congruence
 *   orc_congruence_many   the same over a list of primes (OpenMP over primes)
 *   orc_bernoulli_rec     B_{p-3} mod p from the recurrence that the EGF
 *                         z/(e^z-1) implies (Section 1, Bernoulli EGF)
 *   orc_euler_rec         E_{p-3} mod p from sec z * cos z = 1 (Section 1,
 *                         Euler EGF, secant convention)
 *   orc_bernoulli_all,    B_{2k} mod p and E_{2k} mod p for every 2k <= p-3
 *   orc_euler_all         (the same two recurrences, every even index kept;
 *                         irregular and E-irregular pairs, Section 1)
 *   orc_harmonic2_mod_p2  sum_{0<k<p} k^-2 mod p^2 (Section 1, eqnWolst)
 *   orc_harmonic1_mod_p2  sum_{0<k<p} k^-1 mod p^2 (Section 1, first display)
 *   orc_primes            plain sieve of Eratosthenes on [lo, hi)
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef unsigned __int128 u128;

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) {
    return (uint64_t)(((u128)a * b) % m);
}

static uint64_t addmod(uint64_t a, uint64_t b, uint64_t m) {
    return (uint64_t)(((u128)a + b) % m);
}

static uint64_t submod(uint64_t a, uint64_t b, uint64_t m) {
    return (uint64_t)(((u128)a + m - (b % m)) % m);
}

/* Reduce a signed integer into [0, m). */
static uint64_t smod(int64_t a, uint64_t m) {
    if (a >= 0) return (uint64_t)a % m;
    uint64_t r = (uint64_t)(-(a + 1)) % m; /* -(a+1) >= 0, avoids overflow at INT64_MIN */
    return (m - 1 - r);
}

/* Inverse of a mod m (gcd(a,m)=1, m < 2^62) by the extended Euclidean
 * algorithm; returns 0 if a is not invertible. */
uint64_t orc_invmod(uint64_t a, uint64_t m) {
    int64_t r0 = (int64_t)m, r1 = (int64_t)(a % m);
    int64_t t0 = 0, t1 = 1;
    while (r1 != 0) {
        int64_t q = r0 / r1;
        int64_t r2 = r0 - q * r1;
        int64_t t2 = t0 - q * t1;
        r0 = r1; r1 = r2;
        t0 = t1; t1 = t2;
    }
    if (r0 != 1) return 0;
    return smod(t0, m);
}

/* Open interval x*p < s < y*p with x = xa/xb, y = ya/yb (Section 2, eqnDefnS):
 * the smallest integer above xa*p/xb and the largest integer below ya*p/yb.
 * Sets *lo > *hi when the interval holds no integer. */
void orc_interval(uint64_t p, uint64_t xa, uint64_t xb, uint64_t ya, uint64_t yb,
                  uint64_t *lo, uint64_t *hi) {
    u128 xn = (u128)xa * p;          /* x*p = xn / xb */
    u128 yn = (u128)ya * p;          /* y*p = yn / yb */
    uint64_t l = (uint64_t)(xn / xb) + 1;             /* s*xb > xn  */
    uint64_t h = (uint64_t)((yn + yb - 1) / yb) - 1;  /* s*yb < yn  */
    *lo = l;
    *hi = h;
}

/* s^ell mod p with the sign (-1)^s when alt != 0 (the S-tilde of eqnMacE). */
static uint64_t term_power(uint64_t s, int ell, int alt, uint64_t p) {
    uint64_t r = s % p, u = 1;
    for (int i = 0; i < ell; i++) u = mulmod(u, r, p);
    if (alt && (s & 1)) u = (p - u) % p;
    return u;
}

/* eqnDefnS written out: sum over s in [lo, hi] of (+-1)^s * s^-ell mod p,
 * with one extended-Euclid inverse per term. */
uint64_t orc_sum_direct(uint64_t p, uint64_t lo, uint64_t hi, int ell, int alt) {
    uint64_t acc = 0;
    if (lo > hi) return 0;
    for (uint64_t s = lo; s <= hi; s++) {
        uint64_t u = term_power(s, ell, alt, p);
        acc = addmod(acc, orc_invmod(u, p), p);
    }
    return acc;
}

/* eqnComputeS over s in [lo, hi]: c0 <- 1, c1 <- 0, then for each s
 * c1 <- c1*u + c0, c0 <- c0*u with u = (+-1)^s s^ell.  Then
 * prod(z + u_s) = c0 + c1 z + ..., and sum 1/u_s = c1/c0. */
void orc_sum_poly_pair(uint64_t p, uint64_t lo, uint64_t hi, int ell, int alt,
                       uint64_t *c0_out, uint64_t *c1_out) {
    uint64_t c0 = 1, c1 = 0;
    for (uint64_t s = lo; s <= hi && lo <= hi; s++) {
        uint64_t u = term_power(s, ell, alt, p);
        c1 = addmod(mulmod(c1, u, p), c0, p);
        c0 = mulmod(c0, u, p);
    }
    *c0_out = c0 % p;
    *c1_out = c1 % p;
}

/* eqnCombinePairs: (c1 z + c0)(c1' z + c0') mod z^2. */
static void combine_pairs(uint64_t p, uint64_t *c0, uint64_t *c1, uint64_t d0, uint64_t d1) {
    uint64_t n1 = addmod(mulmod(*c0, d1, p), mulmod(*c1, d0, p), p);
    uint64_t n0 = mulmod(*c0, d0, p);
    *c0 = n0;
    *c1 = n1;
}

/* S over [lo, hi] by eqnComputeS, the range cut into `pieces` consecutive
 * pieces that run on separate threads and are joined with eqnCombinePairs. */
uint64_t orc_sum_poly(uint64_t p, uint64_t lo, uint64_t hi, int ell, int alt, int nthreads) {
    if (lo > hi) return 0;
    uint64_t n = hi - lo + 1;
    int pieces = nthreads > 1 ? 4 * nthreads : 1;
    if ((uint64_t)pieces > n) pieces = (int)n;
    uint64_t *pc0 = (uint64_t *)malloc(sizeof(uint64_t) * pieces);
    uint64_t *pc1 = (uint64_t *)malloc(sizeof(uint64_t) * pieces);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (int i = 0; i < pieces; i++) {
        uint64_t a = lo + (uint64_t)((u128)n * i / pieces);
        uint64_t b = lo + (uint64_t)((u128)n * (i + 1) / pieces) - 1;
        orc_sum_poly_pair(p, a, b, ell, alt, &pc0[i], &pc1[i]);
    }
    uint64_t c0 = 1, c1 = 0;
    for (int i = 0; i < pieces; i++) combine_pairs(p, &c0, &c1, pc0[i], pc1[i]);
    free(pc0);
    free(pc1);
    return mulmod(c1, orc_invmod(c0, p), p);
}

/* One congruence  lhs * X == sum_i coef_i * S(x_i, y_i)  (mod p), solved for X.
 * x_i = xa[i]/xb[i], y_i = ya[i]/yb[i]; method 0 = direct inverses, 1 = the
 * polynomial method.  Returns UINT64_MAX when lhs == 0 mod p (congruence not
 * usable at this p). */
uint64_t orc_congruence(uint64_t p, int nterms, const int64_t *coef,
                        const uint64_t *xa, const uint64_t *xb,
                        const uint64_t *ya, const uint64_t *yb,
                        int64_t lhs, int ell, int alt, int method, int nthreads) {
    uint64_t L = smod(lhs, p);
    if (L == 0) return UINT64_MAX;
    uint64_t acc = 0;
    for (int i = 0; i < nterms; i++) {
        uint64_t lo, hi;
        orc_interval(p, xa[i], xb[i], ya[i], yb[i], &lo, &hi);
        uint64_t S = (method == 0) ? orc_sum_direct(p, lo, hi, ell, alt)
                                   : orc_sum_poly(p, lo, hi, ell, alt, nthreads);
        acc = addmod(acc, mulmod(smod(coef[i], p), S, p), p);
    }
    return mulmod(acc, orc_invmod(L, p), p);
}

/* orc_congruence over many primes, one prime per thread. */
void orc_congruence_many(const uint64_t *primes, size_t n, int nterms, const int64_t *coef,
                         const uint64_t *xa, const uint64_t *xb,
                         const uint64_t *ya, const uint64_t *yb,
                         int64_t lhs, int ell, int alt, int method, int nthreads,
                         uint64_t *out) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (size_t i = 0; i < n; i++)
        out[i] = orc_congruence(primes[i], nterms, coef, xa, xb, ya, yb, lhs, ell, alt, method, 1);
}

/* B_{p-3} mod p from the recurrence sum_{j=0}^{m} C(m+1, j) B_j = 0 (m >= 1),
 * which the Bernoulli EGF z/(e^z - 1) implies.  All divisions are by m+1 <= p-2,
 * and no B_j with j <= p-3 has p in its denominator (p-1 does not divide j), so
 * the recurrence may be run in F_p.  O(p^2); for small p. */
uint64_t orc_bernoulli_rec(uint64_t p) {
    uint64_t n_max = p - 3;
    uint64_t *B = (uint64_t *)calloc(n_max + 1, sizeof(uint64_t));
    uint64_t *row = (uint64_t *)calloc(p + 1, sizeof(uint64_t)); /* C(n, .) mod p */
    B[0] = 1;
    row[0] = 1;                 /* row for n = 0 */
    uint64_t n_row = 0;
    for (uint64_t m = 1; m <= n_max; m++) {
        /* advance Pascal's row to n = m+1 */
        while (n_row < m + 1) {
            n_row++;
            row[n_row] = 1;
            for (uint64_t j = n_row - 1; j >= 1; j--) row[j] = addmod(row[j], row[j - 1], p);
        }
        uint64_t acc = 0;
        for (uint64_t j = 0; j < m; j++) acc = addmod(acc, mulmod(row[j], B[j], p), p);
        /* (m+1) B_m = -acc */
        B[m] = mulmod((p - acc) % p, orc_invmod((m + 1) % p, p), p);
    }
    uint64_t r = B[n_max];
    free(B);
    free(row);
    return r;
}

/* E_{p-3} mod p from sec z * cos z = 1: for n >= 1,
 * sum_{j=0}^{floor(n/2)} (-1)^j C(n, 2j) E_{n-2j} = 0  (Euler EGF, secant).
 * Integers throughout, so run in F_p.  O(p^2); for small p. */
uint64_t orc_euler_rec(uint64_t p) {
    uint64_t n_max = p - 3;
    uint64_t *E = (uint64_t *)calloc(n_max + 1, sizeof(uint64_t));
    uint64_t *row = (uint64_t *)calloc(p + 1, sizeof(uint64_t));
    E[0] = 1;
    row[0] = 1;
    uint64_t n_row = 0;
    for (uint64_t n = 1; n <= n_max; n++) {
        while (n_row < n) {
            n_row++;
            row[n_row] = 1;
            for (uint64_t j = n_row - 1; j >= 1; j--) row[j] = addmod(row[j], row[j - 1], p);
        }
        /* E_n = -sum_{j>=1} (-1)^j C(n,2j) E_{n-2j} */
        uint64_t acc = 0;
        for (uint64_t j = 1; 2 * j <= n; j++) {
            uint64_t t = mulmod(row[2 * j], E[n - 2 * j], p);
            acc = (j & 1) ? submod(acc, t, p) : addmod(acc, t, p);
        }
        E[n] = (p - acc) % p;
    }
    uint64_t r = E[n_max];
    free(E);
    free(row);
    return r;
}

/* B_{2k} mod p into out[k-1] for k = 1 .. (p-3)/2: the recurrence of
 * orc_bernoulli_rec, every even index kept.  O(p^2); for small p. */
void orc_bernoulli_all(uint64_t p, uint64_t *out) {
    uint64_t n_max = p - 3;
    uint64_t *B = (uint64_t *)calloc(n_max + 1, sizeof(uint64_t));
    uint64_t *row = (uint64_t *)calloc(p + 1, sizeof(uint64_t));
    B[0] = 1;
    row[0] = 1;
    uint64_t n_row = 0;
    for (uint64_t m = 1; m <= n_max; m++) {
        while (n_row < m + 1) {
            n_row++;
            row[n_row] = 1;
            for (uint64_t j = n_row - 1; j >= 1; j--) row[j] = addmod(row[j], row[j - 1], p);
        }
        uint64_t acc = 0;
        for (uint64_t j = 0; j < m; j++) acc = addmod(acc, mulmod(row[j], B[j], p), p);
        B[m] = mulmod((p - acc) % p, orc_invmod((m + 1) % p, p), p);
    }
    for (uint64_t k = 1; 2 * k <= n_max; k++) out[k - 1] = B[2 * k];
    free(B);
    free(row);
}

/* E_{2k} mod p into out[k-1] for k = 1 .. (p-3)/2: the recurrence of
 * orc_euler_rec, every even index kept.  O(p^2); for small p. */
void orc_euler_all(uint64_t p, uint64_t *out) {
    uint64_t n_max = p - 3;
    uint64_t *E = (uint64_t *)calloc(n_max + 1, sizeof(uint64_t));
    uint64_t *row = (uint64_t *)calloc(p + 1, sizeof(uint64_t));
    E[0] = 1;
    row[0] = 1;
    uint64_t n_row = 0;
    for (uint64_t n = 1; n <= n_max; n++) {
        while (n_row < n) {
            n_row++;
            row[n_row] = 1;
            for (uint64_t j = n_row - 1; j >= 1; j--) row[j] = addmod(row[j], row[j - 1], p);
        }
        uint64_t acc = 0;
        for (uint64_t j = 1; 2 * j <= n; j++) {
            uint64_t t = mulmod(row[2 * j], E[n - 2 * j], p);
            acc = (j & 1) ? submod(acc, t, p) : addmod(acc, t, p);
        }
        E[n] = (p - acc) % p;
    }
    for (uint64_t k = 1; 2 * k <= n_max; k++) out[k - 1] = E[2 * k];
    free(E);
    free(row);
}

/* sum_{0<k<p} k^-2 mod p^2, one inverse mod p^2 per term (p < 2^31). */
uint64_t orc_harmonic2_mod_p2(uint64_t p) {
    uint64_t m = p * p, acc = 0;
    for (uint64_t k = 1; k < p; k++) {
        uint64_t ik = orc_invmod(k, m);
        acc = addmod(acc, mulmod(ik, ik, m), m);
    }
    return acc;
}

/* sum_{0<k<p} k^-1 mod p^2 (p < 2^31). */
uint64_t orc_harmonic1_mod_p2(uint64_t p) {
    uint64_t m = p * p, acc = 0;
    for (uint64_t k = 1; k < p; k++) acc = addmod(acc, orc_invmod(k, m), m);
    return acc;
}

/* Primes in [lo, hi) by a plain sieve of Eratosthenes: base primes up to
 * sqrt(hi) by the same sieve, then multiples crossed off in the window.
 * Writes up to cap primes; returns how many there are. */
uint64_t orc_primes(uint64_t lo, uint64_t hi, uint64_t *out, uint64_t cap) {
    if (hi <= lo) return 0;
    uint64_t r = 1;
    while ((r + 1) * (r + 1) <= hi) r++;          /* r = isqrt(hi) (or just below) */
    while (r * r > hi) r--;
    char *small = (char *)calloc(r + 2, 1);       /* small[i] = 1: i composite */
    for (uint64_t i = 2; i * i <= r + 1; i++)
        if (!small[i])
            for (uint64_t j = i * i; j <= r + 1; j += i) small[j] = 1;
    uint64_t w = hi - lo;
    char *comp = (char *)calloc(w, 1);
    for (uint64_t i = 2; i <= r + 1; i++) {
        if (small[i]) continue;
        uint64_t start = ((lo + i - 1) / i) * i;
        if (start < i * i) start = i * i;
        for (uint64_t j = start; j < hi; j += i) comp[j - lo] = 1;
    }
    uint64_t n = 0;
    for (uint64_t k = 0; k < w; k++) {
        uint64_t v = lo + k;
        if (v < 2 || comp[k]) continue;
        if (n < cap) out[n] = v;
        n++;
    }
    free(small);
    free(comp);
    return n;
}

int orc_max_threads(void) { return omp_get_max_threads(); }
