// wv_kernels.hip -- HIP kernels and the C ABI of libwvprime.so (gfx950).
//
// Pipeline for a batch of primes (Booker, Hathi, Mossinghoff, Trudgian,
// arXiv:2101.11157):
//   sieve    segmented Eratosthenes, one 2^20-integer segment per workgroup,
//            odd-only bitmap in LDS (the paper enumerates primes with an
//            external sieve, Section 3 "Results"; any exact sieve will do)
//   plan     per prime: congruence choice, open-interval endpoints
//            x p < s < y p (Section 2, eqnDefnS), chunk counts; exclusive scan
//   sum      persistent term-sum kernel: every lane runs eqnComputeS
//            (c1 <- c1 u + c0, c0 <- c0 u, u = s^3 or s^2) over a chunk of
//            consecutive s, with u stepped by finite differences (Section 3,
//            first improvement for p > 6e10); a wave whose 64 chunks belong to
//            one sum joins them with a butterfly of eqnCombinePairs
//   reduce   one wave per (prime, sum): eqnCombinePairs over its chunk pairs
//   finalize per prime: S_i = c1_i/c0_i, X = L^-1 sum coef_i S_i (the
//            specialised congruences of Sections 3 and 5), one Fermat inverse
//            per residue, flags for X == 0.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "mont.hpp"
#include "sum_core.hpp"
#include "wv_tables.hpp"
#include "wvprime.h"

namespace wv {

// --------------------------------------------------------------------------
// constants and records
// --------------------------------------------------------------------------

constexpr int kSegLog = 20;                    // sieve segment: 2^20 integers
constexpr uint64_t kSegSpan = 1ull << kSegLog;
constexpr int kSegBits = 1 << (kSegLog - 1);   // odd integers per segment
constexpr int kSegWords = kSegBits / 32;       // 16384 words = 64 KiB of LDS
constexpr uint32_t kBaseLimit = 1u << 20;      // base primes below 2^20 cover p < 2^40
constexpr int kTotalTerms = 256;               // all tables' terms together

struct DevTerm {
    int64_t coef;
    uint32_t xa, xb, ya, yb;
};
struct DevTable {
    int32_t deg, n, off, pad;
    int64_t lhs;
};

__constant__ DevTerm c_terms[kTotalTerms];
__constant__ DevTable c_tables[WV_TABLE_COUNT];

struct PrimeRec {      // 32 bytes
    uint64_t p;
    uint64_t r2;       // R^2 mod p
    uint64_t one;      // R mod p
    uint32_t ninv;     // -p^-1 mod 2^32
    uint8_t tb, te;    // congruences used
    uint8_t ok, pad;
};

struct SegRec {        // one (prime, sum)
    uint64_t lo;       // first s
    uint64_t len;      // number of s; 0 for an unused slot
    uint32_t prime;    // index in the batch
    uint32_t deg;      // 3 (B) or 2 (E)
};

struct Pair {
    uint64_t c0, c1;
};

__device__ __forceinline__ Mont mont_of(const PrimeRec &r) {
    Mont m;
    m.p = r.p;
    m.p0 = (uint32_t)r.p;
    m.p1 = (uint32_t)(r.p >> 32);
    m.ninv = r.ninv;
    return m;
}

// Wave-uniform values are moved into scalar registers with readfirstlane /
// readlane, so that every branch and loop exit that depends on them is a
// scalar branch.  A cross-lane read through a vector shuffle inside a loop lets
// the compiler split the loop per lane, and lanes can then read a register of
// a lane that is parked on another path.
__device__ __forceinline__ uint64_t readfirst_u64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask) {
    uint32_t lo = __shfl_xor((int)(uint32_t)v, mask, 64);
    uint32_t hi = __shfl_xor((int)(uint32_t)(v >> 32), mask, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Butterfly of eqnCombinePairs across the 64 lanes of a wave; every lane
// ends with the product of all 64 pairs (same prime on all lanes).
__device__ __forceinline__ void wave_pair_reduce(uint64_t &c0, uint64_t &c1, const Mont &m) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        uint64_t d0 = shfl_xor_u64(c0, off);
        uint64_t d1 = shfl_xor_u64(c1, off);
        pair_mul(c0, c1, d0, d1, m);
    }
}

// --------------------------------------------------------------------------
// sieve
// --------------------------------------------------------------------------

// Odd primes 3 <= q < 2^20 into out (ascending); *n_out = count.  One block of
// 1024 threads; bit i of the LDS bitmap stands for 2i+1.
__global__ void __launch_bounds__(1024) k_base_sieve(uint32_t *out, uint32_t *n_out) {
    __shared__ uint32_t bits[kSegWords];
    __shared__ uint32_t small[256];
    __shared__ uint32_t nsmall;
    __shared__ uint32_t scan[1024];
    const int tid = threadIdx.x;
    for (int w = tid; w < kSegWords; w += 1024) bits[w] = 0;
    if (tid == 0) nsmall = 0;
    __syncthreads();
    // odd primes below 1024 = sqrt(2^20), by trial division
    if (tid < 512) {
        uint32_t n = 2 * tid + 1;
        bool pr = n >= 3;
        for (uint32_t d = 3; d * d <= n && pr; d += 2)
            if (n % d == 0) pr = false;
        if (pr) small[atomicAdd(&nsmall, 1u)] = n;
    }
    __syncthreads();
    const uint32_t ns = nsmall;
    for (uint32_t k = 0; k < ns; k++) {
        uint32_t q = small[k];
        for (uint32_t mlt = q * q + 2 * q * tid; mlt < kBaseLimit; mlt += 2 * q * 1024) {
            uint32_t i = mlt >> 1;
            atomicOr(&bits[i >> 5], 1u << (i & 31));
        }
    }
    __syncthreads();
    if (tid == 0) bits[0] |= 1u;   // 1 is not prime
    __syncthreads();
    // compaction: 16 words per thread, block exclusive scan of the counts
    uint32_t cnt = 0;
    for (int w = tid * 16; w < tid * 16 + 16; w++) cnt += __popc(~bits[w]);
    scan[tid] = cnt;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = tid >= off ? scan[tid - off] : 0;
        __syncthreads();
        scan[tid] += v;
        __syncthreads();
    }
    uint32_t pos = scan[tid] - cnt;
    for (int w = tid * 16; w < tid * 16 + 16; w++) {
        uint32_t free = ~bits[w];
        while (free) {
            int b = __ffs(free) - 1;
            free &= free - 1;
            out[pos++] = 2u * (uint32_t)(w * 32 + b) + 1u;
        }
    }
    if (tid == 1023) *n_out = scan[1023];
}

// Segment `blockIdx.x` covers [L, L + 2^20) with L = base + blockIdx.x * 2^20
// (base even); bit i stands for L + 2i + 1.  Marks odd multiples of every odd
// base prime q with q^2 < min(L + 2^20, hi), then keeps the primes p with
// max(lo, 5) <= p < hi.  Writes the count to counts[seg] and, when bits_out is
// non-null, the prime bitmap (1 = prime) to bits_out + seg * kSegWords.
__global__ void __launch_bounds__(1024) k_seg_sieve(uint64_t lo, uint64_t hi, uint64_t base,
                                                    const uint32_t *__restrict__ bp, uint32_t n_bp,
                                                    uint32_t *__restrict__ bits_out,
                                                    uint32_t *__restrict__ counts) {
    __shared__ uint32_t bits[kSegWords];
    __shared__ uint32_t red[16];
    const int tid = threadIdx.x;
    const uint64_t L = base + (uint64_t)blockIdx.x * kSegSpan;
    const uint64_t H = min(L + kSegSpan, hi);
    for (int w = tid; w < kSegWords; w += 1024) bits[w] = 0;
    __syncthreads();
    // primes below 2048 (the first 308 odd ones): all threads stride one prime
    const uint32_t n_coop = min(n_bp, 308u);
    for (uint32_t k = 0; k < n_coop; k++) {
        const uint64_t q = bp[k];
        if (q * q >= H) break;
        uint64_t x = max(q * q, L + 1);
        uint64_t m0 = ((x + q - 1) / q) * q;
        if (!(m0 & 1)) m0 += q;
        const uint64_t i0 = (m0 - L - 1) >> 1;
        for (uint64_t i = i0 + (uint64_t)tid * q; i < (uint64_t)kSegBits; i += 1024 * q)
            atomicOr(&bits[i >> 5], 1u << (i & 31));
    }
    // larger primes: one prime per thread
    for (uint32_t k = n_coop + tid; k < n_bp; k += 1024) {
        const uint64_t q = bp[k];
        if (q * q >= H) break;
        uint64_t x = max(q * q, L + 1);
        uint64_t m0 = ((x + q - 1) / q) * q;
        if (!(m0 & 1)) m0 += q;
        for (uint64_t i = (m0 - L - 1) >> 1; i < (uint64_t)kSegBits; i += q)
            atomicOr(&bits[i >> 5], 1u << (i & 31));
    }
    __syncthreads();
    // keep max(lo,5) <= n < hi, n = L + 2i + 1
    const uint64_t nlo = max(lo, (uint64_t)5);
    uint32_t cnt = 0;
    for (int w = tid; w < kSegWords; w += 1024) {
        uint32_t v = ~bits[w];
        const uint64_t n0 = L + 64ull * w + 1;           // number of bit 0 of this word
        const uint64_t n31 = n0 + 62;
        if (n0 < nlo || n31 >= hi) {
            uint32_t mask = 0;
            for (int b = 0; b < 32; b++) {
                uint64_t n = n0 + 2ull * b;
                if (n >= nlo && n < hi) mask |= 1u << b;
            }
            v &= mask;
        }
        if (bits_out) bits_out[(size_t)blockIdx.x * kSegWords + w] = v;
        cnt += __popc(v);
    }
    // block sum of the counts
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor((int)cnt, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = cnt;
    __syncthreads();
    if (tid == 0) {
        uint32_t t = 0;
        for (int i = 0; i < 16; i++) t += red[i];
        counts[blockIdx.x] = t;
    }
    (void)H;
}

// Writes the primes of segment blockIdx.x, ascending, at out + off[seg].
__global__ void __launch_bounds__(1024) k_seg_compact(uint64_t base, const uint32_t *__restrict__ bits_in,
                                                      const uint64_t *__restrict__ off,
                                                      uint64_t *__restrict__ out) {
    __shared__ uint32_t scan[1024];
    const int tid = threadIdx.x;
    const uint32_t *bits = bits_in + (size_t)blockIdx.x * kSegWords;
    const uint64_t L = base + (uint64_t)blockIdx.x * kSegSpan;
    uint32_t cnt = 0;
    for (int w = tid * 16; w < tid * 16 + 16; w++) cnt += __popc(bits[w]);
    scan[tid] = cnt;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint32_t v = tid >= o ? scan[tid - o] : 0;
        __syncthreads();
        scan[tid] += v;
        __syncthreads();
    }
    uint64_t pos = off[blockIdx.x] + scan[tid] - cnt;
    for (int w = tid * 16; w < tid * 16 + 16; w++) {
        uint32_t v = bits[w];
        while (v) {
            int b = __ffs(v) - 1;
            v &= v - 1;
            out[pos++] = L + 2ull * (uint64_t)(w * 32 + b) + 1ull;
        }
    }
}

// --------------------------------------------------------------------------
// exclusive scan of uint64 (three passes)
// --------------------------------------------------------------------------

constexpr int kScanTile = 1024;   // 256 threads x 4

__global__ void __launch_bounds__(256) k_scan_tiles(const uint64_t *__restrict__ in, uint64_t n,
                                                    uint64_t *__restrict__ out, uint64_t *__restrict__ tile_sum) {
    __shared__ uint64_t s[256];
    const int tid = threadIdx.x;
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + tid * 4;
    uint64_t v[4], run = 0;
    for (int k = 0; k < 4; k++) {
        v[k] = base + k < n ? in[base + k] : 0;
        run += v[k];
    }
    s[tid] = run;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        uint64_t t = tid >= o ? s[tid - o] : 0;
        __syncthreads();
        s[tid] += t;
        __syncthreads();
    }
    uint64_t acc = s[tid] - run;
    for (int k = 0; k < 4; k++) {
        if (base + k < n) out[base + k] = acc;
        acc += v[k];
    }
    if (tid == 255) tile_sum[blockIdx.x] = s[255];
}

__global__ void __launch_bounds__(1024) k_scan_carry(uint64_t *__restrict__ tile_sum, uint64_t n_tiles,
                                                     uint64_t *__restrict__ total) {
    __shared__ uint64_t s[1024];
    __shared__ uint64_t carry;
    const int tid = threadIdx.x;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (uint64_t b = 0; b < n_tiles; b += 1024) {
        uint64_t v = b + tid < n_tiles ? tile_sum[b + tid] : 0;
        s[tid] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            uint64_t t = tid >= o ? s[tid - o] : 0;
            __syncthreads();
            s[tid] += t;
            __syncthreads();
        }
        if (b + tid < n_tiles) tile_sum[b + tid] = carry + s[tid] - v;
        __syncthreads();
        if (tid == 0) carry += s[1023];
        __syncthreads();
    }
    if (tid == 0) *total = carry;
}

__global__ void __launch_bounds__(256) k_scan_add(uint64_t *__restrict__ out, uint64_t n,
                                                  const uint64_t *__restrict__ tile_sum) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] += tile_sum[i / kScanTile];
}

// --------------------------------------------------------------------------
// plan
// --------------------------------------------------------------------------

__device__ __forceinline__ uint64_t smod_dev(int64_t a, uint64_t p) {
    int64_t r = a % (int64_t)p;
    return (uint64_t)(r < 0 ? r + (int64_t)p : r);
}

// One thread per prime.  Slot layout: B sums of prime i at i*nB + j, E sums at
// n*nB + i*nE + j (all Bernoulli work first, then all Euler work).
__global__ void __launch_bounds__(256) k_plan(const uint64_t *__restrict__ primes, uint32_t n, int tb_cfg,
                                              int te_cfg, int nB, int nE, PrimeRec *__restrict__ pr,
                                              SegRec *__restrict__ segs, uint64_t *__restrict__ terms) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t p = primes[i];
    const bool ok = p >= 5 && p < WV_P_MAX && (p & 1);
    PrimeRec r;
    r.p = ok ? p : 11;   // keep the arithmetic defined for rejected inputs
    r.tb = (uint8_t)(p == 5 ? WV_TABLE_BB1 : p == 7 ? WV_TABLE_V12 : tb_cfg);
    r.te = (uint8_t)(p < 11 ? WV_TABLE_E1 : te_cfg);
    Mont m = make_mont(r.p);
    r.ninv = m.ninv;
    r.one = r_mod(r.p);
    r.r2 = r2_mod(r.p);
    r.ok = ok;
    r.pad = 0;
    pr[i] = r;
    for (int side = 0; side < 2; side++) {
        const DevTable t = c_tables[side == 0 ? r.tb : r.te];
        const int nslots = side == 0 ? nB : nE;
        for (int j = 0; j < nslots; j++) {
            const size_t slot = side == 0 ? (size_t)i * nB + j : (size_t)n * nB + (size_t)i * nE + j;
            SegRec s;
            s.prime = i;
            s.deg = (uint32_t)t.deg;
            s.lo = 1;
            s.len = 0;
            if (ok && j < t.n) {
                const DevTerm d = c_terms[t.off + j];
                // open interval (xa/xb) p < s < (ya/yb) p
                const uint64_t lo = (d.xa * p) / d.xb + 1;
                const uint64_t hi = (d.ya * p - 1) / d.yb;
                s.lo = lo;
                s.len = hi >= lo ? hi - lo + 1 : 0;
            }
            segs[slot] = s;
            terms[slot] = s.len;
        }
    }
}

// Chunk size: at least `chunk_cfg` terms, and large enough that the total
// number of chunks stays within `max_chunks` (the partial-pair buffer).
__global__ void k_pick_chunk(const uint64_t *__restrict__ total_terms, uint64_t nseg, uint64_t chunk_cfg,
                             uint64_t max_chunks, uint64_t *__restrict__ chunk_out) {
    const uint64_t T = *total_terms;
    uint64_t room = max_chunks > nseg ? max_chunks - nseg : 1;
    uint64_t c = (T + room - 1) / room;
    c = (c + 63) & ~63ull;
    *chunk_out = max(chunk_cfg, max(c, (uint64_t)64));
}

__global__ void __launch_bounds__(256) k_chunk_count(const uint64_t *__restrict__ terms, uint64_t nseg,
                                                     const uint64_t *__restrict__ chunk,
                                                     uint64_t *__restrict__ cnt) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nseg) return;
    const uint64_t C = *chunk;
    cnt[i] = (terms[i] + C - 1) / C;
}

__global__ void k_zero_u64(uint64_t *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

// --------------------------------------------------------------------------
// term-sum kernel
// --------------------------------------------------------------------------

// Per-lane work of one chunk: the blocked loop with K terms per block when
// the chunk is long enough to amortise the difference tables, else one term
// per iteration.
template <int DEG, int K>
__device__ __forceinline__ void chunk_pair(uint64_t s0, uint64_t cnt, const Mont &m, uint64_t r2, uint64_t one,
                                           uint64_t &c0, uint64_t &c1) {
    if (K > 1 && cnt >= (uint64_t)4 * (DEG * K + 1) * K) run_chunk_blocked<DEG, K>(s0, cnt, m, r2, one, c0, c1);
    else run_chunk<DEG>(s0, cnt, m, r2, one, c0, c1);
}

// Persistent: each wave takes 64 consecutive chunks at a time from `counter`
// until every chunk is done.  A wave whose chunks all belong to one sum stores
// their butterfly product at partials[first chunk]; any other wave stores one
// pair per chunk at partials[chunk].  KB / KE: terms per block on the
// Bernoulli (s^3) and Euler (s^2) sides.
template <int KB, int KE>
__global__ void __launch_bounds__(256) k_sum(const SegRec *__restrict__ segs, const uint64_t *__restrict__ off,
                                             uint32_t nseg, const PrimeRec *__restrict__ pr,
                                             const uint64_t *__restrict__ chunk_ptr, Pair *__restrict__ partials,
                                             unsigned long long *__restrict__ counter) {
    const uint64_t total = off[nseg];
    const uint64_t C = *chunk_ptr;
    const int lane = threadIdx.x & 63;
    // A wave can take at most total/64 + 1 batches; the bound is a second exit.
    const uint64_t max_iter = total / 64 + 2;
    for (uint64_t iter = 0; iter < max_iter; iter++) {
        uint64_t got = 0;
        if (lane == 0) got = atomicAdd(counter, 64ull);
        const uint64_t base = readfirst_u64(got);   // whole wave active: lane 0 is first
        if (base >= total) break;
        const uint64_t chunk = base + lane;
        const bool active = chunk < total;
        uint32_t seg = 0xffffffffu;
        uint64_t c0 = 1, c1 = 0;
        Mont m;
        m.p = 11; m.p0 = 11; m.p1 = 0; m.ninv = neg_inv32(11);
        if (active) {
            seg = find_seg(off, nseg, chunk);
            const SegRec sr = segs[seg];
            const PrimeRec P = pr[sr.prime];
            m = mont_of(P);
            const uint64_t o = (chunk - off[seg]) * C;
            const uint64_t s0 = sr.lo + o;
            const uint64_t cnt = min(C, sr.len - o);
            if (sr.deg == 3) chunk_pair<3, KB>(s0, cnt, m, P.r2, P.one, c0, c1);
            else chunk_pair<2, KE>(s0, cnt, m, P.r2, P.one, c0, c1);
        }
        const uint32_t seg0 = __builtin_amdgcn_readlane(seg, 0);
        const uint32_t segl = __builtin_amdgcn_readlane(seg, 63);
        const bool uniform = (seg0 == segl) && (base + 63 < total);   // scalar
        if (uniform) {
            wave_pair_reduce(c0, c1, m);
            if (lane == 0) partials[base] = Pair{c0, c1};
        } else if (active) {
            partials[chunk] = Pair{c0, c1};
        }
    }
}

typedef void (*SumKernel)(const SegRec *, const uint64_t *, uint32_t, const PrimeRec *, const uint64_t *, Pair *,
                          unsigned long long *);

struct SumVariant {
    int kb, ke;
    SumKernel fn;
};

// Compiled block shapes (terms per block, Bernoulli side / Euler side).
static const SumVariant kSumVariants[] = {
    {1, 1, k_sum<1, 1>},   {4, 4, k_sum<4, 4>},   {8, 8, k_sum<8, 8>},
    {8, 16, k_sum<8, 16>}, {16, 8, k_sum<16, 8>}, {16, 16, k_sum<16, 16>},
};
constexpr int kNumSumVariants = (int)(sizeof(kSumVariants) / sizeof(kSumVariants[0]));

// --------------------------------------------------------------------------
// per-sum reduction and finalize
// --------------------------------------------------------------------------

// One wave per (prime, sum): joins the stored pairs of chunks [off[j], off[j+1]).
__global__ void __launch_bounds__(256) k_reduce(const SegRec *__restrict__ segs, const uint64_t *__restrict__ off,
                                                uint32_t nseg, const PrimeRec *__restrict__ pr,
                                                const Pair *__restrict__ partials, Pair *__restrict__ seg_pairs) {
    const uint32_t j = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= nseg) return;   // scalar: the whole wave exits together
    const uint64_t a = off[j], b = off[j + 1];
    const Mont m = mont_of(pr[segs[j].prime]);
    uint64_t c0 = 1, c1 = 0;
    const uint64_t ff = (a + 63) & ~63ull;   // first 64-aligned window start
    const uint64_t lf = b & ~63ull;          // end of the last full window
    if (ff >= lf) {
        for (uint64_t i = a + lane; i < b; i += 64) {
            const Pair q = partials[i];
            pair_mul(c0, c1, q.c0, q.c1, m);
        }
    } else {
        for (uint64_t i = a + lane; i < ff; i += 64) {
            const Pair q = partials[i];
            pair_mul(c0, c1, q.c0, q.c1, m);
        }
        for (uint64_t w = ff + 64ull * lane; w < lf; w += 64ull * 64) {
            const Pair q = partials[w];
            pair_mul(c0, c1, q.c0, q.c1, m);
        }
        for (uint64_t i = lf + lane; i < b; i += 64) {
            const Pair q = partials[i];
            pair_mul(c0, c1, q.c0, q.c1, m);
        }
    }
    wave_pair_reduce(c0, c1, m);
    if (lane == 0) seg_pairs[j] = Pair{c0, c1};
}

// L^-1 sum_i coef_i c1_i / c0_i mod p for one congruence; pairs at
// seg_pairs[first + j].  Running fraction N/D in Montgomery values.
__device__ uint64_t combine_residue(const DevTable &t, const Pair *__restrict__ sp, size_t first, const Mont &m,
                                    uint64_t r2, uint64_t one) {
    const uint64_t p = m.p;
    uint64_t N = 0, D = one;
    for (int j = 0; j < t.n; j++) {
        const Pair q = sp[first + j];
        const uint64_t cR = to_mont(smod_dev(c_terms[t.off + j].coef, p), r2, m);
        const uint64_t num = mmul(mmul(cR, q.c1, m), D, m);       // coef c1 D / R
        N = mmul(N, q.c0, m) + num;                                 // (N c0 + coef c1 D) / R
        D = mmul(D, q.c0, m);                                       // D c0 / R
    }
    const uint64_t LR = to_mont(smod_dev(t.lhs, p), r2, m);
    const uint64_t X = mmul(D, LR, m);                              // D L
    const uint64_t XR = mmul(X, r2, m);                             // D L R
    const uint64_t inv = mpow(XR, p - 2, one, m);                   // (D L)^-1 R
    return red1(mmul(N, inv, m), p);                                // N / (D L)
}

// S_j = c1_j / c0_j, canonical, for every (prime, sum) slot.
__global__ void __launch_bounds__(256) k_sum_values(const SegRec *__restrict__ segs, const PrimeRec *__restrict__ pr,
                                                    const Pair *__restrict__ sp, uint64_t nseg,
                                                    uint64_t *__restrict__ out) {
    const uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= nseg) return;
    const PrimeRec P = pr[segs[j].prime];
    const Mont m = mont_of(P);
    const Pair q = sp[j];
    const uint64_t inv = mpow(mmul(q.c0, P.r2, m), P.p - 2, P.one, m);   // c0^-1 R
    out[j] = P.ok ? red1(mmul(q.c1, inv, m), P.p) : 0;
}

__global__ void __launch_bounds__(256) k_finalize(const PrimeRec *__restrict__ pr, const Pair *__restrict__ sp,
                                                  uint32_t n, int nB, int nE, wv_result *__restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const PrimeRec P = pr[i];
    wv_result r;
    r.reserved = 0;
    if (!P.ok) {
        r.p = 0;
        r.b = 0;
        r.e = 0;
        r.flags = 0xFFFFFFFFu;
        out[i] = r;
        return;
    }
    const Mont m = mont_of(P);
    r.p = P.p;
    r.b = combine_residue(c_tables[P.tb], sp, (size_t)i * nB, m, P.r2, P.one);
    r.e = combine_residue(c_tables[P.te], sp, (size_t)n * nB + (size_t)i * nE, m, P.r2, P.one);
    r.flags = (r.b == 0 ? WV_FLAG_WOLSTENHOLME : 0u) | (r.e == 0 ? WV_FLAG_VANDIVER : 0u);
    out[i] = r;
}

}  // namespace wv

// ==========================================================================
// host side
// ==========================================================================

using namespace wv;

namespace {

struct DevBuf {
    void *ptr = nullptr;
    size_t cap = 0;
};

enum { EV_START, EV_SIEVE, EV_PLAN, EV_SUM, EV_REDUCE, EV_FINAL, EV_COUNT };

constexpr uint64_t kDefaultChunk = 1ull << 16;
constexpr uint64_t kMaxChunks = 1ull << 24;   // partial pairs held at once (256 MiB)
constexpr uint64_t kWindowSegs = 4;           // sieve segments per search batch

}  // namespace

struct wv_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev[EV_COUNT] = {};
    int tb = WV_TABLE_BB30, te = WV_TABLE_EE33;
    uint64_t chunk_cfg = 0;
    int num_cus = 0;
    int variant = 2;                    // index into kSumVariants
    int sum_blocks[16] = {};            // persistent grid per variant
    uint32_t n_base = 0;
    DevBuf base_primes, primes, pr, segs, terms, cnt, off, tiles, scal, partials, seg_pairs, results,
        seg_counts, seg_bits, seg_off;
    wv_stats stats{};
};

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? WV_OK : WV_EHIP; }

#define WV_TRY(expr)                         \
    do {                                     \
        int _rc = (expr);                    \
        if (_rc != WV_OK) return _rc;        \
    } while (0)
#define WV_HIP(expr)                                             \
    do {                                                         \
        hipError_t _e = (expr);                                  \
        if (_e != hipSuccess) {                                  \
            if (getenv("WV_DEBUG"))                              \
                fprintf(stderr, "wvprime: %s:%d %s: %s\n", __FILE__, __LINE__, #expr, hipGetErrorString(_e)); \
            return _e == hipErrorOutOfMemory ? WV_ENOMEM : WV_EHIP; \
        }                                                        \
    } while (0)

int ensure(DevBuf &b, size_t bytes) {
    if (b.cap >= bytes && b.ptr) return WV_OK;
    if (b.ptr) {
        WV_HIP(hipFree(b.ptr));
        b.ptr = nullptr;
        b.cap = 0;
    }
    size_t want = std::max(bytes, (size_t)256);
    WV_HIP(hipMalloc(&b.ptr, want));
    b.cap = want;
    return WV_OK;
}

template <class T>
T *as(DevBuf &b) { return reinterpret_cast<T *>(b.ptr); }

uint64_t mulmod_h(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((unsigned __int128)a * b % m); }

uint64_t powmod_h(uint64_t a, uint64_t e, uint64_t m) {
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

int table_slots(int id) { return kTables[id].n; }

int upload_tables() {
    DevTerm terms[kTotalTerms];
    DevTable tabs[WV_TABLE_COUNT];
    int off = 0;
    for (int i = 0; i < kNumTables; i++) {
        tabs[i].deg = kTables[i].deg;
        tabs[i].n = kTables[i].n;
        tabs[i].off = off;
        tabs[i].pad = 0;
        tabs[i].lhs = kTables[i].lhs;
        for (int j = 0; j < kTables[i].n; j++) {
            const TermDef &t = kTables[i].t[j];
            terms[off + j] = DevTerm{t.coef, t.xa, t.xb, t.ya, t.yb};
        }
        off += kTables[i].n;
    }
    WV_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_terms), terms, sizeof(DevTerm) * off));
    WV_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tables), tabs, sizeof(tabs)));
    return WV_OK;
}

// Exclusive scan of n uint64 at `in` into `out` (n+1 entries; out[n] = total).
int scan_u64(wv_ctx *c, const uint64_t *in, uint64_t n, uint64_t *out, hipStream_t st) {
    const uint64_t tiles = std::max<uint64_t>(1, (n + kScanTile - 1) / kScanTile);
    WV_TRY(ensure(c->tiles, tiles * sizeof(uint64_t)));
    uint64_t *ts = as<uint64_t>(c->tiles);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(256), 0, st, in, n, out, ts);
    hipLaunchKernelGGL(k_scan_carry, dim3(1), dim3(1024), 0, st, ts, tiles, out + n);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256 + (n == 0))), dim3(256), 0, st, out, n,
                       (const uint64_t *)ts);
    WV_HIP(hipGetLastError());
    return WV_OK;
}

// plan -> scan -> sum -> reduce -> finalize for n primes already on the device.
int run_batch(wv_ctx *c, const uint64_t *d_primes, uint32_t n, wv_result *d_out, hipStream_t st, bool timed) {
    const int nB = std::max(table_slots(c->tb), 1);
    const int nE = std::max(table_slots(c->te), 1);
    const uint64_t nseg = (uint64_t)n * (nB + nE);
    WV_TRY(ensure(c->pr, (size_t)n * sizeof(PrimeRec)));
    WV_TRY(ensure(c->segs, nseg * sizeof(SegRec)));
    WV_TRY(ensure(c->terms, nseg * sizeof(uint64_t)));
    WV_TRY(ensure(c->cnt, nseg * sizeof(uint64_t)));
    WV_TRY(ensure(c->off, (nseg + 1) * sizeof(uint64_t)));
    WV_TRY(ensure(c->scal, 8 * sizeof(uint64_t)));
    // partial pairs: at most total_terms / chunk + nseg chunks (k_pick_chunk keeps
    // total_terms / chunk <= cap - nseg), so cap >= 2 nseg always leaves room
    const uint64_t cap = std::max<uint64_t>(kMaxChunks, 2 * nseg);
    WV_TRY(ensure(c->partials, cap * sizeof(Pair)));
    WV_TRY(ensure(c->seg_pairs, nseg * sizeof(Pair)));
    uint64_t *scal = as<uint64_t>(c->scal);   // [0] total terms, [1] chunk, [2] counter, [3] total B terms
    uint64_t *toff = as<uint64_t>(c->off);    // reused: prefix of terms, then of chunks
    const uint64_t chunk_cfg = c->chunk_cfg ? c->chunk_cfg : kDefaultChunk;

    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, scal, 8);
    hipLaunchKernelGGL(k_plan, dim3((n + 255) / 256), dim3(256), 0, st, d_primes, n, c->tb, c->te, nB, nE,
                       as<PrimeRec>(c->pr), as<SegRec>(c->segs), as<uint64_t>(c->terms));
    WV_HIP(hipGetLastError());
    // total terms (prefix of the per-slot term counts) -> chunk size -> chunk prefix
    WV_TRY(scan_u64(c, as<uint64_t>(c->terms), nseg, toff, st));
    hipLaunchKernelGGL(k_pick_chunk, dim3(1), dim3(1), 0, st, toff + nseg, nseg, chunk_cfg, cap, scal + 1);
    if (timed) {
        // keep the totals for the statistics: terms overall and Bernoulli-side
        WV_HIP(hipMemcpyAsync(scal + 0, toff + nseg, sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
        WV_HIP(hipMemcpyAsync(scal + 3, toff + (uint64_t)n * nB, sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
    }
    hipLaunchKernelGGL(k_chunk_count, dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, st,
                       (const uint64_t *)as<uint64_t>(c->terms), nseg, (const uint64_t *)(scal + 1),
                       as<uint64_t>(c->cnt));
    WV_TRY(scan_u64(c, as<uint64_t>(c->cnt), nseg, toff, st));
    WV_HIP(hipGetLastError());
    if (timed) WV_HIP(hipEventRecord(c->ev[EV_PLAN], st));

    hipLaunchKernelGGL(kSumVariants[c->variant].fn, dim3(c->sum_blocks[c->variant]), dim3(256), 0, st,
                       (const SegRec *)as<SegRec>(c->segs),
                       (const uint64_t *)toff, (uint32_t)nseg, (const PrimeRec *)as<PrimeRec>(c->pr),
                       (const uint64_t *)(scal + 1), as<Pair>(c->partials),
                       (unsigned long long *)(scal + 2));
    WV_HIP(hipGetLastError());
    if (timed) WV_HIP(hipEventRecord(c->ev[EV_SUM], st));

    const uint64_t rthreads = nseg * 64;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((rthreads + 255) / 256)), dim3(256), 0, st,
                       (const SegRec *)as<SegRec>(c->segs), (const uint64_t *)toff, (uint32_t)nseg,
                       (const PrimeRec *)as<PrimeRec>(c->pr), (const Pair *)as<Pair>(c->partials),
                       as<Pair>(c->seg_pairs));
    WV_HIP(hipGetLastError());
    if (timed) WV_HIP(hipEventRecord(c->ev[EV_REDUCE], st));

    hipLaunchKernelGGL(k_finalize, dim3((n + 255) / 256), dim3(256), 0, st, (const PrimeRec *)as<PrimeRec>(c->pr),
                       (const Pair *)as<Pair>(c->seg_pairs), n, nB, nE, d_out);
    WV_HIP(hipGetLastError());
    if (timed) WV_HIP(hipEventRecord(c->ev[EV_FINAL], st));
    return WV_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
    return ms;
}

// Adds the timings and sizes of the batch that just completed to c->stats.
int collect_stats(wv_ctx *c, uint32_t n, bool with_sieve) {
    WV_HIP(hipEventSynchronize(c->ev[EV_FINAL]));
    wv_stats &s = c->stats;
    const hipEvent_t before_plan = with_sieve ? c->ev[EV_SIEVE] : c->ev[EV_START];
    if (with_sieve) s.ms_sieve += elapsed(c->ev[EV_START], c->ev[EV_SIEVE]);
    s.ms_plan += elapsed(before_plan, c->ev[EV_PLAN]);
    s.ms_sum += elapsed(c->ev[EV_PLAN], c->ev[EV_SUM]);
    s.ms_reduce += elapsed(c->ev[EV_SUM], c->ev[EV_REDUCE]);
    s.ms_finalize += elapsed(c->ev[EV_REDUCE], c->ev[EV_FINAL]);
    s.ms_total += elapsed(c->ev[EV_START], c->ev[EV_FINAL]);
    const int nB = std::max(table_slots(c->tb), 1), nE = std::max(table_slots(c->te), 1);
    uint64_t host[4];
    WV_HIP(hipMemcpy(host, c->scal.ptr, sizeof(host), hipMemcpyDeviceToHost));
    uint64_t chunks = 0;
    const uint64_t nseg = (uint64_t)n * (nB + nE);
    WV_HIP(hipMemcpy(&chunks, as<uint64_t>(c->off) + nseg, sizeof(uint64_t), hipMemcpyDeviceToHost));
    s.n_primes += n;
    s.n_sums += nseg;
    s.n_chunks += chunks;
    s.n_terms += host[0];
    s.n_terms_b += host[3];
    s.chunk_terms = host[1];
    s.block_k_b = (uint32_t)kSumVariants[c->variant].kb;
    s.block_k_e = (uint32_t)kSumVariants[c->variant].ke;
    s.grid = (uint32_t)c->sum_blocks[c->variant];
    return WV_OK;
}

int check_device(wv_ctx *c) {
    WV_HIP(hipSetDevice(c->device));
    return WV_OK;
}

}  // namespace

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
        for (int v = 0; v < kNumSumVariants; v++) {
            int per_cu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kSumVariants[v].fn, 256, 0) != hipSuccess ||
                per_cu < 1)
                per_cu = 1;
            c->sum_blocks[v] = c->num_cus * per_cu;
        }
        if ((rc = upload_tables()) != WV_OK) break;
        if ((rc = ensure(c->base_primes, kBaseLimit / 2 * sizeof(uint32_t))) != WV_OK) break;
        if ((rc = ensure(c->scal, 8 * sizeof(uint64_t))) != WV_OK) break;
        hipLaunchKernelGGL(k_base_sieve, dim3(1), dim3(1024), 0, c->stream, as<uint32_t>(c->base_primes),
                           reinterpret_cast<uint32_t *>(c->scal.ptr));
        if (hipGetLastError() != hipSuccess) { rc = WV_EHIP; break; }
        uint32_t nb = 0;
        if (hipMemcpyAsync(&nb, c->scal.ptr, sizeof(nb), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) { rc = WV_EHIP; break; }
        c->n_base = nb;
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
    DevBuf *bufs[] = {&c->base_primes, &c->primes, &c->pr, &c->segs, &c->terms, &c->cnt, &c->off, &c->tiles,
                      &c->scal, &c->partials, &c->seg_pairs, &c->results, &c->seg_counts, &c->seg_bits,
                      &c->seg_off};
    for (DevBuf *b : bufs)
        if (b->ptr) (void)hipFree(b->ptr);
    for (int i = 0; i < EV_COUNT; i++)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return WV_OK;
}

int wv_set_tables(wv_ctx *c, int b_table, int e_table) {
    if (!c) return WV_EINVAL;
    if (b_table < WV_TABLE_BB1 || b_table > WV_TABLE_BB30) return WV_EINVAL;
    if (e_table < WV_TABLE_EE3 || e_table > WV_TABLE_EE33) return WV_EINVAL;
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
    for (int v = 0; v < kNumSumVariants; v++) {
        if (kSumVariants[v].kb == kb && kSumVariants[v].ke == ke) {
            c->variant = v;
            return WV_OK;
        }
    }
    return WV_EINVAL;
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
    if (hi <= 5 || hi <= lo) return WV_OK;
    const uint64_t base = lo & ~1ull;
    const uint64_t nseg_total = (hi - base + kSegSpan - 1) / kSegSpan;
    const uint64_t batch = 1 << 16;
    WV_TRY(ensure(c->seg_counts, batch * sizeof(uint32_t)));
    std::vector<uint32_t> host(batch);
    uint64_t total = 0;
    for (uint64_t s0 = 0; s0 < nseg_total; s0 += batch) {
        const uint64_t ns = std::min(batch, nseg_total - s0);
        hipLaunchKernelGGL(k_seg_sieve, dim3((unsigned)ns), dim3(1024), 0, c->stream, lo, hi, base + s0 * kSegSpan,
                           (const uint32_t *)as<uint32_t>(c->base_primes), c->n_base, (uint32_t *)nullptr,
                           as<uint32_t>(c->seg_counts));
        WV_HIP(hipGetLastError());
        WV_HIP(hipMemcpyAsync(host.data(), c->seg_counts.ptr, ns * sizeof(uint32_t), hipMemcpyDeviceToHost,
                              c->stream));
        WV_HIP(hipStreamSynchronize(c->stream));
        for (uint64_t i = 0; i < ns; i++) total += host[i];
    }
    *n = total;
    return WV_OK;
}

int wv_search_range(wv_ctx *c, uint64_t lo, uint64_t hi, wv_result *out, size_t cap, size_t *n_out,
                    uint64_t *hits, size_t hit_cap, size_t *n_hits) {
    if (!c || !n_out || lo > hi || (hit_cap && !hits)) return WV_EINVAL;
    if (hi > WV_P_MAX) return WV_EDOMAIN;
    WV_TRY(check_device(c));
    // count first, so that a short buffer is reported before any work
    uint64_t total = 0;
    WV_TRY(wv_count_primes(c, lo, hi, &total));
    *n_out = (size_t)total;
    if (n_hits) *n_hits = 0;
    if (total > cap) return WV_ETRUNC;
    if (total > 0 && !out) return WV_EINVAL;
    c->stats = wv_stats{};
    if (total == 0) return WV_OK;
    const uint64_t base0 = lo & ~1ull;
    const uint64_t nseg_total = (hi - base0 + kSegSpan - 1) / kSegSpan;
    WV_TRY(ensure(c->seg_counts, kWindowSegs * sizeof(uint32_t)));
    WV_TRY(ensure(c->seg_bits, kWindowSegs * kSegWords * sizeof(uint32_t)));
    WV_TRY(ensure(c->seg_off, (kWindowSegs + 1) * sizeof(uint64_t)));
    WV_TRY(ensure(c->tiles, 64 * sizeof(uint64_t)));
    size_t written = 0, nh = 0;
    std::vector<uint32_t> counts(kWindowSegs);
    for (uint64_t s0 = 0; s0 < nseg_total; s0 += kWindowSegs) {
        const uint64_t ns = std::min(kWindowSegs, nseg_total - s0);
        const uint64_t base = base0 + s0 * kSegSpan;
        WV_HIP(hipEventRecord(c->ev[EV_START], c->stream));
        hipLaunchKernelGGL(k_seg_sieve, dim3((unsigned)ns), dim3(1024), 0, c->stream, lo, hi, base,
                           (const uint32_t *)as<uint32_t>(c->base_primes), c->n_base, as<uint32_t>(c->seg_bits),
                           as<uint32_t>(c->seg_counts));
        WV_HIP(hipGetLastError());
        WV_HIP(hipMemcpyAsync(counts.data(), c->seg_counts.ptr, ns * sizeof(uint32_t), hipMemcpyDeviceToHost,
                              c->stream));
        WV_HIP(hipStreamSynchronize(c->stream));
        std::vector<uint64_t> offs(ns + 1, 0);
        for (uint64_t i = 0; i < ns; i++) offs[i + 1] = offs[i] + counts[i];
        const uint64_t np = offs[ns];
        if (np == 0) continue;
        if (written + np > cap) return WV_EHIP;   // sieve disagreed with the count pass
        WV_TRY(ensure(c->primes, np * sizeof(uint64_t)));
        WV_TRY(ensure(c->results, np * sizeof(wv_result)));
        WV_HIP(hipMemcpyAsync(c->seg_off.ptr, offs.data(), (ns + 1) * sizeof(uint64_t), hipMemcpyHostToDevice,
                              c->stream));
        hipLaunchKernelGGL(k_seg_compact, dim3((unsigned)ns), dim3(1024), 0, c->stream, base,
                           (const uint32_t *)as<uint32_t>(c->seg_bits), (const uint64_t *)as<uint64_t>(c->seg_off),
                           as<uint64_t>(c->primes));
        WV_HIP(hipGetLastError());
        WV_HIP(hipEventRecord(c->ev[EV_SIEVE], c->stream));
        WV_TRY(run_batch(c, as<uint64_t>(c->primes), (uint32_t)np, as<wv_result>(c->results), c->stream, true));
        WV_HIP(hipMemcpyAsync(out + written, c->results.ptr, np * sizeof(wv_result), hipMemcpyDeviceToHost,
                              c->stream));
        WV_TRY(collect_stats(c, (uint32_t)np, true));
        WV_HIP(hipStreamSynchronize(c->stream));
        for (uint64_t i = 0; i < np; i++) {
            if (out[written + i].flags) {
                if (nh < hit_cap) hits[nh] = out[written + i].p;
                nh++;
            }
        }
        written += np;
    }
    if (n_hits) *n_hits = nh;
    return WV_OK;
}

int wv_eval_primes(wv_ctx *c, const uint64_t *primes, size_t n, wv_result *out) {
    if (!c) return WV_EINVAL;
    if (n == 0) return WV_OK;
    if (!primes || !out) return WV_EINVAL;
    if (n > 0xFFFFFFFFull) return WV_EINVAL;
    for (size_t i = 0; i < n; i++) {
        if (primes[i] < 5 || primes[i] >= WV_P_MAX) return WV_EDOMAIN;
        if (!is_prime_u64(primes[i])) return WV_ENOTPRIME;
    }
    WV_TRY(check_device(c));
    c->stats = wv_stats{};
    WV_TRY(ensure(c->primes, n * sizeof(uint64_t)));
    WV_TRY(ensure(c->results, n * sizeof(wv_result)));
    WV_HIP(hipEventRecord(c->ev[EV_START], c->stream));
    WV_HIP(hipMemcpyAsync(c->primes.ptr, primes, n * sizeof(uint64_t), hipMemcpyHostToDevice, c->stream));
    WV_TRY(run_batch(c, as<uint64_t>(c->primes), (uint32_t)n, as<wv_result>(c->results), c->stream, true));
    WV_HIP(hipMemcpyAsync(out, c->results.ptr, n * sizeof(wv_result), hipMemcpyDeviceToHost, c->stream));
    WV_TRY(collect_stats(c, (uint32_t)n, false));
    WV_HIP(hipStreamSynchronize(c->stream));
    return WV_OK;
}

int wv_eval_sums(wv_ctx *c, const uint64_t *primes, size_t n, uint64_t *out_b, uint64_t *out_e) {
    if (!c) return WV_EINVAL;
    if (n == 0) return WV_OK;
    if (!primes || !out_b || !out_e || n > 0xFFFFFFFFull) return WV_EINVAL;
    for (size_t i = 0; i < n; i++) {
        if (primes[i] < 5 || primes[i] >= WV_P_MAX) return WV_EDOMAIN;
        if (!is_prime_u64(primes[i])) return WV_ENOTPRIME;
    }
    WV_TRY(check_device(c));
    const int nB = std::max(table_slots(c->tb), 1), nE = std::max(table_slots(c->te), 1);
    const uint64_t nseg = (uint64_t)n * (nB + nE);
    WV_TRY(ensure(c->primes, n * sizeof(uint64_t)));
    WV_TRY(ensure(c->results, std::max(n * sizeof(wv_result), (size_t)nseg * sizeof(uint64_t))));
    WV_HIP(hipMemcpyAsync(c->primes.ptr, primes, n * sizeof(uint64_t), hipMemcpyHostToDevice, c->stream));
    WV_TRY(run_batch(c, as<uint64_t>(c->primes), (uint32_t)n, as<wv_result>(c->results), c->stream, false));
    // the results buffer is free again once finalize has run: reuse it for the sums
    uint64_t *d_sums = as<uint64_t>(c->results);
    hipLaunchKernelGGL(k_sum_values, dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, c->stream,
                       (const SegRec *)as<SegRec>(c->segs), (const PrimeRec *)as<PrimeRec>(c->pr),
                       (const Pair *)as<Pair>(c->seg_pairs), nseg, d_sums);
    WV_HIP(hipGetLastError());
    WV_HIP(hipMemcpyAsync(out_b, d_sums, (size_t)n * nB * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
    WV_HIP(hipMemcpyAsync(out_e, d_sums + (size_t)n * nB, (size_t)n * nE * sizeof(uint64_t),
                          hipMemcpyDeviceToHost, c->stream));
    WV_HIP(hipStreamSynchronize(c->stream));
    return WV_OK;
}

int wv_eval_primes_async(wv_ctx *c, const uint64_t *d_primes, size_t n, wv_result *d_out, void *hip_stream) {
    if (!c) return WV_EINVAL;
    if (n == 0) return WV_OK;
    if (!d_primes || !d_out || n > 0xFFFFFFFFull) return WV_EINVAL;
    WV_TRY(check_device(c));
    return run_batch(c, d_primes, (uint32_t)n, d_out, (hipStream_t)hip_stream, false);
}

}  // extern "C"
