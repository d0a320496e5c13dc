// wv_kernels.hip -- HIP kernels of libwvprime.so (gfx950) and their launchers.
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
#include "wv_internal.hpp"

namespace wv {

// --------------------------------------------------------------------------
// constants and records
// --------------------------------------------------------------------------

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

// v of lane (lane ^ X) within the same 32-lane half (0 < X < 32): ds_swizzle
// in bit-mask mode (offset = and-mask 0x1f | or-mask 0 << 5 | xor-mask X << 10).
// The pattern is an immediate, so unlike ds_bpermute no per-lane address
// register is held; the persistent sum kernel would otherwise keep those
// addresses live across its loop and spill them.
template <int X>
__device__ __forceinline__ uint32_t swz_xor(uint32_t v) {
    static_assert(X > 0 && X < 32, "swizzle reaches within a 32-lane half");
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1f | (X << 10));
}

template <int X>
__device__ __forceinline__ uint64_t swz_xor_u64(uint64_t v) {
    return ((uint64_t)swz_xor<X>((uint32_t)(v >> 32)) << 32) | swz_xor<X>((uint32_t)v);
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// minimum over the 64 lanes of a fully active wave, as a wave-uniform value
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    v = min(v, swz_xor<16>(v));
    v = min(v, swz_xor<8>(v));
    v = min(v, swz_xor<4>(v));
    v = min(v, swz_xor<2>(v));
    v = min(v, swz_xor<1>(v));
    // readlane returns int: compare as unsigned (0xffffffff is the largest value)
    const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
    const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)v, 32);
    return a < b ? a : b;
}

// Butterfly of eqnCombinePairs across the 64 lanes of a fully active wave
// (same prime on all lanes): each 32-lane half by swizzles, then the two
// halves through scalar reads; every lane ends with the product of all 64
// pairs.
template <int X>
__device__ __forceinline__ void pair_swz_step(uint64_t &c0, uint64_t &c1, const Mont &m) {
    const uint64_t d0 = swz_xor_u64<X>(c0);
    const uint64_t d1 = swz_xor_u64<X>(c1);
    pair_mul(c0, c1, d0, d1, m);
}

__device__ __forceinline__ void wave_pair_reduce(uint64_t &c0, uint64_t &c1, const Mont &m) {
    pair_swz_step<16>(c0, c1, m);
    pair_swz_step<8>(c0, c1, m);
    pair_swz_step<4>(c0, c1, m);
    pair_swz_step<2>(c0, c1, m);
    pair_swz_step<1>(c0, c1, m);
    const uint64_t d0 = readlane_u64(c0, 32), d1 = readlane_u64(c1, 32);
    c0 = readlane_u64(c0, 0);
    c1 = readlane_u64(c1, 0);
    pair_mul(c0, c1, d0, d1, m);
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

// Segment desc[blockIdx.x]; bit i stands for L + 2i + 1.  Marks odd multiples
// of every odd base prime q with q^2 < min(L + 2^20, hi), then keeps the
// primes p with max(lo, 5) <= p < hi.  Writes the count to counts[seg] and,
// when bits_out is non-null, the prime bitmap (1 = prime) to
// bits_out + seg * kSegWords.
__global__ void __launch_bounds__(1024) k_seg_sieve(const SegDesc *__restrict__ desc,
                                                    const uint32_t *__restrict__ bp, uint32_t n_bp,
                                                    uint32_t *__restrict__ bits_out,
                                                    uint32_t *__restrict__ counts) {
    __shared__ uint32_t bits[kSegWords];
    __shared__ uint32_t red[16];
    const int tid = threadIdx.x;
    const SegDesc d = desc[blockIdx.x];
    const uint64_t L = d.L, lo = d.lo, hi = d.hi;
    const uint64_t H = min(L + kSegSpan, hi);
    for (int w = tid; w < kSegWords; w += 1024) bits[w] = 0;
    __syncthreads();
    // only [max(lo, L + 1), H) is kept (the count masks the rest): composites
    // are marked there, bits i < i_end hold n = L + 2i + 1 up to H
    const uint64_t first = max(lo, L + 1);
    const uint64_t i_end = min((uint64_t)kSegBits, (H - L + 1) >> 1);
    // primes below 2048 (the first 308 odd ones): all threads stride one prime
    const uint32_t n_coop = min(n_bp, 308u);
    for (uint32_t k = 0; k < n_coop; k++) {
        const uint64_t q = bp[k];
        if (q * q >= H) break;
        uint64_t x = max(q * q, first);
        uint64_t m0 = ((x + q - 1) / q) * q;
        if (!(m0 & 1)) m0 += q;
        const uint64_t i0 = (m0 - L - 1) >> 1;
        for (uint64_t i = i0 + (uint64_t)tid * q; i < i_end; i += 1024 * q)
            atomicOr(&bits[i >> 5], 1u << (i & 31));
    }
    // larger primes: one prime per thread
    for (uint32_t k = n_coop + tid; k < n_bp; k += 1024) {
        const uint64_t q = bp[k];
        if (q * q >= H) break;
        uint64_t x = max(q * q, first);
        uint64_t m0 = ((x + q - 1) / q) * q;
        if (!(m0 & 1)) m0 += q;
        for (uint64_t i = (m0 - L - 1) >> 1; i < i_end; i += q)
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
}

// Writes the primes of segment blockIdx.x, ascending, at out + off[seg].
__global__ void __launch_bounds__(1024) k_seg_compact(const SegDesc *__restrict__ desc,
                                                      const uint32_t *__restrict__ bits_in,
                                                      const uint64_t *__restrict__ off,
                                                      uint64_t *__restrict__ out, uint64_t limit) {
    __shared__ uint32_t scan[1024];
    const int tid = threadIdx.x;
    const uint32_t *bits = bits_in + (size_t)blockIdx.x * kSegWords;
    const uint64_t L = desc[blockIdx.x].L;
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
            if (pos < limit) out[pos] = L + 2ull * (uint64_t)(w * 32 + b) + 1ull;
            pos++;
        }
    }
}

// Exclusive prefix of ns <= 1024 segment counts (one workgroup).  A total
// other than `expect` (the count the caller sized the output for) leaves every
// offset at `expect`, so the compaction writes nothing, and zeroes the output.
__global__ void __launch_bounds__(256) k_seg_offsets(const uint32_t *__restrict__ counts, uint32_t ns, uint64_t expect,
                                                     uint64_t *__restrict__ off, uint64_t *__restrict__ primes) {
    __shared__ uint64_t total;
    if (threadIdx.x == 0) {
        uint64_t a = 0;
        for (uint32_t i = 0; i < ns; i++) {
            off[i] = a;
            a += counts[i];
        }
        off[ns] = a;
        total = a;
    }
    __syncthreads();
    if (expect == UINT64_MAX || total == expect) return;   // UINT64_MAX: no count to check
    for (uint32_t i = threadIdx.x; i <= ns; i += 256) off[i] = expect;
    for (uint64_t i = threadIdx.x; i < expect; i += 256) primes[i] = 0;
}

// --------------------------------------------------------------------------
// exclusive scan of uint64 (three passes)
// --------------------------------------------------------------------------

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

// A signed integer of any size (limbs of its magnitude, base 2^32, least
// significant first) mod p, canonical.
__device__ uint64_t limbs_mod(const uint32_t *__restrict__ limb, uint32_t off, int nlimb, bool neg, uint64_t p) {
    uint64_t r = 0;
    for (int k = nlimb - 1; k >= 0; k--) r = shift_in_limb(r, limb[off + k], p);
    return neg && r ? p - r : r;
}

// Table of one side for prime p: the configured one where it applies, else
// the table it names for the primes it does not serve (a chain of defined
// tables with falling min_p that ends at a compiled table; fb if a chain were
// ever longer than the registry); the root forms for p = 5 and 7 (readings of
// the paper: the specialised tables need p >= 11).
__device__ int pick_table(TableStore ts, int side, uint64_t p, int cfg, int fb) {
    if (side == 0 && p == 5) return WV_TABLE_BB1;
    if (side == 0 && p == 7) return WV_TABLE_V12;
    if (side == 1 && p < 11) return WV_TABLE_E1;
    int t = cfg;
    for (int hop = 0; hop <= kMaxTableChain && t >= WV_TABLE_COUNT; hop++) {
        const TableHead h = ts.head[t];
        if (p >= h.min_p && limbs_mod(ts.limb, h.lhs_off, h.lhs_nlimb, false, p) != 0) return t;
        t = h.below;
    }
    return t >= WV_TABLE_COUNT ? fb : t;
}

// One thread per prime: PrimeRec, the table of each side and the residues of
// their left sides.
__global__ void __launch_bounds__(256) k_plan_primes(const uint64_t *__restrict__ primes, uint32_t n, int tb_cfg,
                                                     int te_cfg, int fb, int fe, TableStore ts,
                                                     PrimeRec *__restrict__ pr, uint64_t *__restrict__ lhsmod) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t p = primes[i];
    const bool ok = p >= 5 && p < WV_P_MAX && (p & 1);
    PrimeRec r;
    r.p = ok ? p : 11;   // keep the arithmetic defined for rejected inputs
    r.tb = (uint8_t)pick_table(ts, 0, r.p, tb_cfg, fb);
    r.te = (uint8_t)pick_table(ts, 1, r.p, te_cfg, fe);
    Mont m = make_mont(r.p);
    r.ninv = m.ninv;
    r.one = r_mod(r.p);
    r.r2 = r2_mod(r.p);
    r.ok = ok;
    r.pad = 0;
    pr[i] = r;
    for (int side = 0; side < 2; side++) {
        const TableHead h = ts.head[side == 0 ? r.tb : r.te];
        lhsmod[2 * (size_t)i + side] = limbs_mod(ts.limb, h.lhs_off, h.lhs_nlimb, h.lhs_neg != 0, r.p);
    }
}

// One thread per (prime, sum) slot.  Slot layout: B sums of prime i at
// i*nB + j, E sums at n*nB + i*nE + j (all Bernoulli work first, then all Euler
// work).  pr, segs, terms and coefs point at the batch's first entries;
// `prime_base` is added to the prime index stored in each SegRec (the batch's
// offset in a larger prime array, as in the request server's pool).  Open
// interval (xa/xb) p < s < (ya/yb) p, in 128-bit products (eqnDefnS).
__global__ void __launch_bounds__(256) k_plan_slots(uint32_t n, int nB, int nE, TableStore ts,
                                                    const PrimeRec *__restrict__ pr, SegRec *__restrict__ segs,
                                                    uint64_t *__restrict__ terms, uint64_t *__restrict__ coefs,
                                                    uint32_t prime_base) {
    const uint64_t slot = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nb_slots = (uint64_t)n * nB;
    if (slot >= nb_slots + (uint64_t)n * nE) return;
    const int side = slot < nb_slots ? 0 : 1;
    const uint64_t k = side == 0 ? slot : slot - nb_slots;
    const int per = side == 0 ? nB : nE;
    // k < 2^32: a batch holds at most 2^27 slots and the server's pool fewer
    // than 2^32 (both checked by the host), so 32-bit division will do
    const uint32_t i = (uint32_t)k / (uint32_t)per;
    const int j = (int)((uint32_t)k - i * (uint32_t)per);
    const PrimeRec r = pr[i];
    const TableHead h = ts.head[side == 0 ? r.tb : r.te];
    SegRec s;
    s.prime = prime_base + i;
    s.deg = (uint32_t)h.deg;
    s.lo = 1;
    s.len = 0;
    uint64_t c = 0;
    if (r.ok && j < h.n) {
        const TableTerm d = ts.term[h.term_off + j];
        const uint64_t p = r.p;
        const uint64_t lo = floor_mul_div(d.xa, p, d.xb) + 1;
        const uint64_t hi = floor_mul_minus1_div(d.ya, p, d.yb);
        s.lo = lo;
        s.len = hi >= lo ? hi - lo + 1 : 0;
        c = limbs_mod(ts.limb, d.limb_off, d.nlimb, d.neg != 0, p);
    }
    segs[slot] = s;
    terms[slot] = s.len;
    coefs[slot] = c;
}

__global__ void k_set_u64(uint64_t *p, int n, uint64_t v) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = v;
}

__global__ void k_copy_u64(const uint64_t *__restrict__ s, uint64_t *__restrict__ d, int n) {
    if ((int)threadIdx.x < n) d[threadIdx.x] = s[threadIdx.x];
}

__global__ void __launch_bounds__(256) k_copy_pad(const uint64_t *__restrict__ src, uint64_t n,
                                                  uint64_t *__restrict__ dst, uint64_t n_pad) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n_pad) dst[i] = i < n ? src[i] : 0;
}

__global__ void __launch_bounds__(256) k_copy_results(const wv_result *__restrict__ src, uint64_t n,
                                                      wv_result *__restrict__ dst) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Chunk size: at least `chunk_cfg` terms, and large enough that the total
// number of chunks stays within `max_chunks` (the partial-pair buffer).
// Terms per lane chunk.  chunk_cfg > 0 is used as given; 0 picks
// sqrt(2 S T / lanes) (S = kChunkSetup), which minimises the per-chunk set-up
// of the blocked loop (about S terms of work per chunk) plus the lanes left
// idle when the last full chunks finish (about half a chunk per lane; the
// sums' shorter tail chunks run last, sorted by length, and fill that gap),
// clamped to [kChunkMin, kChunkMax].  Either way at least
// T / (max_chunks - nseg), so the partial pairs fit, rounded up to a multiple
// of 64.
__global__ void k_pick_chunk(const uint64_t *__restrict__ total_terms, uint64_t nseg, uint64_t chunk_cfg,
                             uint64_t max_chunks, uint64_t lanes, uint64_t *__restrict__ chunk_out) {
    const uint64_t T = *total_terms;
    uint64_t want = chunk_cfg ? chunk_cfg : adaptive_chunk(T, lanes);
    uint64_t room = max_chunks > nseg ? max_chunks - nseg : 1;
    uint64_t c = (T + room - 1) / room;
    c = max(c, want);
    c = (c + 63) & ~63ull;
    *chunk_out = max(c, (uint64_t)64);
}

// Chunk layout of a batch: every sum of len terms gets len / C full chunks of
// exactly C terms, numbered sum by sum, and, when C does not divide len, one
// tail chunk of len % C terms.  The tails follow all full chunks, grouped into
// kTailClasses classes (tail_class: length, longest first, then side), so that
// the 64 chunks a wave takes have (nearly) equal lengths and one side, and the
// shortest work comes last.  Slots below nb_slots are s^-3 sums.
//
// A workgroup takes kLayoutTile consecutive sums and counts its tails per
// class in LDS; one lane per distinct class of a wave adds the wave's count
// (most tails of a batch fall in a few classes, so per-lane atomics would
// queue on one address), and the workgroup adds its counts to the global
// ones once per class.
constexpr int kLayoutItems = 16;
constexpr uint64_t kLayoutTile = 256ull * kLayoutItems;

// Adds, for every distinct key among the lanes with `has`, the number of
// such lanes holding it to ctr[key]; returns this lane's rank among them
// (the counter's old value plus the lanes below it with the same key).
// Called by the whole wave.
__device__ __forceinline__ uint32_t wave_rank_add(uint32_t *ctr, uint32_t key, bool has) {
    const int lane = threadIdx.x & 63;
    uint64_t pending = __ballot(has);
    uint32_t rank = 0;
    while (pending) {
        const int leader = __builtin_ctzll(pending);
        const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
        const uint64_t m = __ballot(has && key == k);
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&ctr[k], (uint32_t)__popcll(m));
        base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
        if (has && key == k) rank = base + (uint32_t)__popcll(m & ((1ull << lane) - 1));
        pending &= ~m;
    }
    return rank;
}

// cnt[i] = full chunks of sum i; tail counts per class into hist.
__global__ void __launch_bounds__(256) k_chunk_split(const uint64_t *__restrict__ terms, uint64_t nseg,
                                                     uint64_t nb_slots, const uint64_t *__restrict__ layout,
                                                     uint64_t *__restrict__ cnt, unsigned long long *__restrict__ hist) {
    __shared__ uint32_t local[kTailClasses];
    if (threadIdx.x < kTailClasses) local[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t C = layout[0];
    const double invC = 1.0 / (double)C;
    const uint64_t first = (uint64_t)blockIdx.x * kLayoutTile;
    for (int it = 0; it < kLayoutItems; it++) {
        const uint64_t i = first + (uint64_t)it * 256 + threadIdx.x;
        uint32_t cls = 0;
        bool has = false;
        if (i < nseg) {
            const uint64_t t = terms[i];
            const uint64_t q = full_chunks(t, C, invC);
            cnt[i] = q;
            const uint64_t rem = t - q * C;
            if (rem) {
                has = true;
                cls = tail_class(rem, C, i < nb_slots ? 3u : 2u);
            }
        }
        (void)wave_rank_add(local, cls, has);
    }
    __syncthreads();
    if (threadIdx.x < kTailClasses && local[threadIdx.x])
        atomicAdd(&hist[threadIdx.x], (unsigned long long)local[threadIdx.x]);
}

// One thread: first position of each class (cursor), the number of tails
// (layout[2]) and of all chunks (*total = full + tails).
__global__ void k_tail_base(const unsigned long long *__restrict__ hist, unsigned long long *__restrict__ cursor,
                            uint64_t *__restrict__ layout, uint64_t *__restrict__ total) {
    uint64_t acc = 0;
    for (int b = 0; b < kTailClasses; b++) {
        cursor[b] = acc;
        acc += hist[b];
    }
    layout[2] = acc;
    *total = layout[1] + acc;
}

// tails[pos] = i for each sum with a tail, pos within its class's range: the
// workgroup counts its tails per class, reserves that many places of each
// class at once, then hands them out.
__global__ void __launch_bounds__(256) k_tail_place(const uint64_t *__restrict__ terms, uint64_t nseg,
                                                    uint64_t nb_slots, const uint64_t *__restrict__ layout,
                                                    unsigned long long *__restrict__ cursor,
                                                    uint32_t *__restrict__ tails) {
    __shared__ uint32_t local[kTailClasses];
    __shared__ unsigned long long base[kTailClasses];
    if (threadIdx.x < kTailClasses) local[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t C = layout[0];
    const double invC = 1.0 / (double)C;
    const uint64_t first = (uint64_t)blockIdx.x * kLayoutTile;
    uint32_t cls[kLayoutItems];
    uint32_t has_mask = 0;
WV_UNROLL
    for (int it = 0; it < kLayoutItems; it++) {
        const uint64_t i = first + (uint64_t)it * 256 + threadIdx.x;
        cls[it] = 0;
        if (i < nseg) {
            const uint64_t t = terms[i];
            const uint64_t rem = t - full_chunks(t, C, invC) * C;
            if (rem) {
                has_mask |= 1u << it;
                cls[it] = tail_class(rem, C, i < nb_slots ? 3u : 2u);
            }
        }
        (void)wave_rank_add(local, cls[it], (has_mask >> it) & 1u);
    }
    __syncthreads();
    if (threadIdx.x < kTailClasses) {
        const uint32_t n = local[threadIdx.x];
        base[threadIdx.x] = n ? atomicAdd(&cursor[threadIdx.x], (unsigned long long)n) : 0ull;
        local[threadIdx.x] = 0;
    }
    __syncthreads();
WV_UNROLL
    for (int it = 0; it < kLayoutItems; it++) {
        const bool has = (has_mask >> it) & 1u;
        const uint32_t r = wave_rank_add(local, cls[it], has);
        if (has) tails[base[cls[it]] + r] = (uint32_t)(first + (uint64_t)it * 256 + threadIdx.x);
    }
}

// --------------------------------------------------------------------------
// term-sum kernel
// --------------------------------------------------------------------------

// Per-lane work of one chunk: the blocked loop with K terms per block (stepped
// through the Taylor coefficients of prod_j (x + j)) when the chunk is long
// enough to amortise building the difference tables, else one term per
// iteration.  Building the tables costs about 6 K (DEG + 1) (K + 1)
// operations (25,000 at K = 28 on the s^-3 side); a block then costs about 6.5
// per term against about 43 for the one-term Montgomery loop, so the blocked
// loop wins from roughly 700 terms: it is taken from 8 K (DEG + 1).
template <int DEG, int K>
__device__ __forceinline__ bool chunk_blocked(uint64_t cnt) {
    return K > 1 && cnt >= (uint64_t)8 * (DEG + 1) * K;
}

// Blocks between table reductions for p < 2^b (b <= 40): 53 - b.
__device__ __forceinline__ uint32_t table_period(uint64_t p) { return 53u - (64u - (uint32_t)__clzll(p)); }

// nb_shared / period_shared: blocks and reduction period every lane of the
// wave shares (wave minima), so those blocks run under scalar loop control.
template <int DEG, int K>
__device__ __forceinline__ void chunk_pair(uint64_t s0, uint64_t cnt, const Mont &m, uint64_t r2, uint64_t one,
                                           uint32_t nb_shared, uint32_t period_shared, uint64_t &c0,
                                           uint64_t &c1) {
    if constexpr (K > 1) {
        if (chunk_blocked<DEG, K>(cnt)) {
            run_chunk_logd<DEG, K>(s0, cnt, m.p, nb_shared, period_shared, c0, c1);
            return;
        }
    }
    run_chunk<DEG>(s0, cnt, m, r2, one, c0, c1);
}

// Persistent: each wave takes 64 consecutive chunks at a time from `counter`
// until every chunk is done.  layout = {C, full chunks F, tails}: chunks below
// F are full chunks (found through off, the prefix of full chunks per sum),
// the others are the tails in the order of `tails`.  A wave whose chunks are
// all full chunks of one sum stores their butterfly product at partials[first
// chunk]; otherwise each full chunk stores its pair at partials[chunk] and
// each tail at seg_pairs[sum].  KB / KE: terms per block on the Bernoulli
// (s^3) and Euler (s^2) sides.  A wave that leaves through its iteration bound
// instead of finding the chunks exhausted sets *err (chunks may be missing).
template <int KB, int KE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_sum(
    const SegRec *__restrict__ segs, const uint64_t *__restrict__ off, uint32_t nseg, const PrimeRec *__restrict__ pr,
    const uint64_t *__restrict__ layout, const uint32_t *__restrict__ tails, Pair *__restrict__ partials,
    Pair *__restrict__ seg_pairs, unsigned long long *__restrict__ counter, uint64_t end,
    unsigned long long *__restrict__ err) {
    // chunks [counter start, min(end, total)); end is a multiple of 64 or past the total
    const uint64_t C = layout[0];
    const uint64_t F = layout[1];
    const uint64_t total = min(F + layout[2], end);
    const int lane = threadIdx.x & 63;
    // 1/C, wave-uniform: kept in scalar registers, not vector ones
    const double invC = __longlong_as_double((long long)readfirst_u64((uint64_t)__double_as_longlong(1.0 / (double)C)));
    // A wave can take at most total/64 + 1 batches; the bound is a second exit.
    const uint64_t max_iter = total / 64 + 2;
    bool drained = false;
    for (uint64_t iter = 0; iter < max_iter; iter++) {
        uint64_t got = 0;
        if (lane == 0) got = atomicAdd(counter, 64ull);
        const uint64_t base = readfirst_u64(got);   // whole wave active: lane 0 is first
        if (base >= total) {
            drained = true;
            break;
        }
        const uint64_t chunk = base + lane;
        const bool active = chunk < total;
        uint32_t seg = 0xffffffffu;
        uint64_t c0 = 1, c1 = 0;
        Mont m;
        m.p = 11; m.p0 = 11; m.p1 = 0; m.ninv = neg_inv32(11);
        uint64_t s0 = 0, cnt = 0, r2 = 0, one = 0;
        uint32_t deg = 0;
        // lanes that take no blocked loop do not lower the wave's shared counts
        uint32_t nb_lane = 0xffffffffu, period_lane = 0xffffffffu;
        if (active) {
            uint64_t o;
            if (chunk < F) {
                seg = find_seg(off, nseg, chunk);
                o = (chunk - off[seg]) * C;
            } else {
                seg = tails[chunk - F];
                o = full_chunks(segs[seg].len, C, invC) * C;
            }
            const SegRec sr = segs[seg];
            const PrimeRec P = pr[sr.prime];
            m = mont_of(P);
            r2 = P.r2;
            one = P.one;
            s0 = sr.lo + o;
            cnt = min(C, sr.len - o);
            deg = sr.deg;
            const bool blk = deg == 3 ? chunk_blocked<3, KB>(cnt) : chunk_blocked<2, KE>(cnt);
            if (blk) {
                nb_lane = (uint32_t)min(cnt / (deg == 3 ? KB : KE), (uint64_t)0xfffffffeu);
                period_lane = table_period(m.p);
            }
        }
        // the whole wave is active here (the loop exit above is wave-uniform)
        const uint32_t nb_shared = wave_min_u32(nb_lane);
        const uint32_t period_shared = wave_min_u32(period_lane);
        const uint32_t seg0 = __builtin_amdgcn_readlane(seg, 0);
        const uint32_t segl = __builtin_amdgcn_readlane(seg, 63);
        // all 64 chunks full (base + 64 <= F) and of one sum; scalar
        const bool uniform = (seg0 == segl) && (base + 63 < F);
        // where this lane's pair goes when the wave does not join them: only
        // this address stays live across the sums (the chunk and sum indices
        // do not), which keeps the chunk set-up's registers out of scratch
        Pair *dst = nullptr;
        if (active && !uniform) dst = chunk < F ? partials + chunk : seg_pairs + seg;
        if (active) {
            if (deg == 3) chunk_pair<3, KB>(s0, cnt, m, r2, one, nb_shared, period_shared, c0, c1);
            else chunk_pair<2, KE>(s0, cnt, m, r2, one, nb_shared, period_shared, c0, c1);
        }
        if (uniform) {
            // one prime for the whole wave: its constants are loaded again
            // (scalar) rather than kept in vector registers across the sums
            const Mont mu = mont_of(pr[segs[seg0].prime]);
            wave_pair_reduce(c0, c1, mu);
            if (lane == 0) partials[base] = Pair{c0, c1};
        } else if (dst) {
            *dst = Pair{c0, c1};
        }
    }
    if (!drained && lane == 0) atomicOr(err, 1ull);
}

typedef void (*SumKernel)(const SegRec *, const uint64_t *, uint32_t, const PrimeRec *, const uint64_t *,
                          const uint32_t *, Pair *, Pair *, unsigned long long *, uint64_t, unsigned long long *);

struct SumVariant {
    int kb, ke;
    SumKernel fn;
};

// Compiled block shapes (terms per block, Bernoulli side / Euler side).
static const SumVariant kSumVariants[] = {
    {1, 1, k_sum<1, 1>}, {4, 4, k_sum<4, 4>}, {8, 8, k_sum<8, 8>}, {12, 16, k_sum<12, 16>},
    {16, 24, k_sum<16, 24>}, {20, 28, k_sum<20, 28>}, {24, 32, k_sum<24, 32>}, {26, 34, k_sum<26, 34>},
    {28, 32, k_sum<28, 32>}, {28, 36, k_sum<28, 36>},
};
constexpr int kNumSumVariants = (int)(sizeof(kSumVariants) / sizeof(kSumVariants[0]));

// --------------------------------------------------------------------------
// per-sum reduction and finalize
// --------------------------------------------------------------------------

// Sums with at most this many full chunks are joined by one lane each.
constexpr uint64_t kReduceLaneChunks = 16;

// Every (prime, sum) j: joins the stored pairs of its full chunks
// [off[j], off[j+1]) and, when C does not divide its length, the pair its tail
// chunk left in seg_pairs[j]; the result replaces seg_pairs[j].  A wave takes
// 64 consecutive sums: a lane joins its own sum when it has few full chunks,
// and the wave joins each of the others together (lanes stride its chunks,
// then a butterfly).
__global__ void __launch_bounds__(256) k_reduce(const SegRec *__restrict__ segs, const uint64_t *__restrict__ off,
                                                uint32_t nseg, const PrimeRec *__restrict__ pr,
                                                const Pair *__restrict__ partials,
                                                const uint64_t *__restrict__ layout, Pair *__restrict__ seg_pairs) {
    const uint64_t C = layout[0];
    const double invC = 1.0 / (double)C;
    // wave-stride loop over groups of 64 sums (one launch covers at most 2^32
    // work-items)
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t ngroups = (nseg + 63) >> 6;
    const int lane = threadIdx.x & 63;
    for (uint32_t gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; gw < ngroups; gw += nwaves) {
        const uint32_t g = __builtin_amdgcn_readfirstlane(gw);   // scalar: loop exits are wave-uniform
        const uint32_t j = g * 64 + lane;
        bool big = false;
        if (j < nseg) {
            const uint64_t a = off[j], b = off[j + 1];
            big = b - a > kReduceLaneChunks;
            if (!big) {
                const SegRec sr = segs[j];
                const Mont m = mont_of(pr[sr.prime]);
                uint64_t c0 = 1, c1 = 0;
                if (sr.len != full_chunks(sr.len, C, invC) * C) {
                    const Pair q = seg_pairs[j];
                    c0 = q.c0;
                    c1 = q.c1;
                }
                for (uint64_t i = a; i < b; i++) {
                    const Pair q = partials[i];
                    pair_mul(c0, c1, q.c0, q.c1, m);
                }
                seg_pairs[j] = Pair{c0, c1};
            }
        }
        uint64_t todo = __ballot(big);
        while (todo) {
            const int l = __builtin_ctzll(todo);
            todo &= todo - 1;
            const uint32_t k = g * 64 + l;   // wave-uniform
            const uint64_t a = off[k], b = off[k + 1];
            const SegRec sr = segs[k];
            const Mont m = mont_of(pr[sr.prime]);
            uint64_t c0 = 1, c1 = 0;
            if (lane == 0 && sr.len != full_chunks(sr.len, C, invC) * C) {
                const Pair q = seg_pairs[k];
                c0 = q.c0;
                c1 = q.c1;
            }
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
            if (lane == 0) seg_pairs[k] = Pair{c0, c1};
        }
    }
}

// The fraction N/D = sum_j coef_j c1_j / c0_j (Montgomery values; any common
// factor of N and D is harmless) over the sums j = j0, j0 + stride, ... of a
// congruence of n sums, for a wave whose lanes start at consecutive j0: each
// lane folds its sums into a running fraction, and a butterfly adds the
// lanes' fractions (N1/D1 + N2/D2 = (N1 D2 + N2 D1) / (D1 D2)), so every lane
// ends with the wave's.  Pairs at sp[first + j], coefficients mod p at
// coef[first + j].  The whole wave must be active.
__device__ void fraction_part(int n, const Pair *__restrict__ sp, const uint64_t *__restrict__ coef, size_t first,
                              const Mont &m, uint64_t r2, uint64_t one, int j0, int stride, uint64_t &N,
                              uint64_t &D) {
    N = 0;
    D = one;
    for (int j = j0; j < n; j += stride) {
        const Pair q = sp[first + j];
        const uint64_t cR = to_mont(coef[first + j], r2, m);
        const uint64_t num = mmul(mmul(cR, q.c1, m), D, m);       // coef c1 D / R
        N = mmul(N, q.c0, m) + num;                                 // (N c0 + coef c1 D) / R
        D = mmul(D, q.c0, m);                                       // D c0 / R
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint64_t N2 = shfl_xor_u64(N, off), D2 = shfl_xor_u64(D, off);
        N = mmul(N, D2, m) + mmul(N2, D, m);
        D = mmul(D, D2, m);
    }
}

// N / (D L) mod p, canonical (N, D Montgomery values, L the left side mod p).
__device__ uint64_t fraction_residue(uint64_t N, uint64_t D, uint64_t lhs, const Mont &m, uint64_t r2, uint64_t one) {
    const uint64_t p = m.p;
    const uint64_t LR = to_mont(lhs, r2, m);
    const uint64_t X = mmul(D, LR, m);                              // D L
    const uint64_t XR = mmul(X, r2, m);                             // D L R
    const uint64_t inv = mpow(XR, p - 2, one, m);                   // (D L)^-1 R
    return red1(mmul(N, inv, m), p);                                // N / (D L)
}

// acc[target[t]] <- acc[target[t]] * tp[t] in F_p[z]/(z^2) (eqnCombinePairs),
// one thread per task; each target appears at most once per launch.
__global__ void __launch_bounds__(256) k_fold(const SegRec *__restrict__ tasks, const uint32_t *__restrict__ target,
                                              const Pair *__restrict__ tp, uint32_t ntask,
                                              const PrimeRec *__restrict__ pr, Pair *__restrict__ acc) {
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= ntask) return;
    const Mont m = mont_of(pr[tasks[t].prime]);
    Pair a = acc[target[t]];
    pair_mul(a.c0, a.c1, tp[t].c0, tp[t].c1, m);
    acc[target[t]] = a;
}

__global__ void __launch_bounds__(256) k_fill_pairs(Pair *__restrict__ p, uint64_t n, uint64_t c0, uint64_t c1) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = Pair{c0, c1};
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

// The residues and flags of prime i by a workgroup of four waves: waves 0
// and 1 take the Bernoulli side's sums (every other group of 64), waves 2
// and 3 the Euler side's; the two halves of each side are joined through LDS
// and the residue taken by the side's first wave.  Four times the
// parallelism of one wave per prime, which left the fraction loop waiting on
// its loads.  A prime that the plan rejected, or every prime of a batch whose
// term sums reported an error (*err), gets p = 0 and flags 0xFFFFFFFF.
// Called by the whole workgroup; writes *out.
__device__ void finalize_prime_wg(const TableStore &ts, const PrimeRec *__restrict__ pr,
                                  const Pair *__restrict__ sp, const uint64_t *__restrict__ coefs,
                                  const uint64_t *__restrict__ lhsmod, uint32_t n, int nB, int nE, uint32_t i,
                                  const unsigned long long *__restrict__ err, wv_result *__restrict__ out) {
    __shared__ uint64_t part[4][2];
    __shared__ uint64_t res[2];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const PrimeRec P = pr[i];
    const bool bad = !P.ok || (err && *err);   // the same for the whole workgroup
    if (bad) {
        if (threadIdx.x == 0) *out = wv_result{0, 0, 0, 0xFFFFFFFFu, 0};
        return;
    }
    const Mont m = mont_of(P);
    const int side = wave >> 1, half = wave & 1;
    const int ns = ts.head[side == 0 ? P.tb : P.te].n;
    const size_t first = side == 0 ? (size_t)i * nB : (size_t)n * nB + (size_t)i * nE;
    uint64_t N, D;
    fraction_part(ns, sp, coefs, first, m, P.r2, P.one, half * 64 + lane, 128, N, D);
    if (lane == 0) {
        part[wave][0] = N;
        part[wave][1] = D;
    }
    __syncthreads();
    if (half == 0) {
        const uint64_t N2 = part[wave + 1][0], D2 = part[wave + 1][1];
        const uint64_t Nt = mmul(N, D2, m) + mmul(N2, D, m), Dt = mmul(D, D2, m);
        const uint64_t r = fraction_residue(Nt, Dt, lhsmod[2 * (size_t)i + side], m, P.r2, P.one);
        if (lane == 0) res[side] = r;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        wv_result r;
        r.p = P.p;
        r.b = res[0];
        r.e = res[1];
        r.flags = (r.b == 0 ? WV_FLAG_WOLSTENHOLME : 0u) | (r.e == 0 ? WV_FLAG_VANDIVER : 0u);
        r.reserved = 0;
        *out = r;
    }
}

// One workgroup per prime of a batch.
__global__ void __launch_bounds__(256) k_finalize_wg(TableStore ts, const PrimeRec *__restrict__ pr,
                                                     const Pair *__restrict__ sp, const uint64_t *__restrict__ coefs,
                                                     const uint64_t *__restrict__ lhsmod, uint32_t n, int nB, int nE,
                                                     wv_result *__restrict__ out,
                                                     const unsigned long long *__restrict__ err) {
    finalize_prime_wg(ts, pr, sp, coefs, lhsmod, n, nB, nE, blockIdx.x, err, out + blockIdx.x);
}

// One workgroup per prime of several pool requests (fr[k]: slots [base, base
// + n), results at out[out0 ..]; out0 ascending from 0, `total` primes in
// all).
__global__ void __launch_bounds__(256) k_finalize_multi(TableStore ts, const PrimeRec *__restrict__ pr,
                                                        const Pair *__restrict__ acc,
                                                        const uint64_t *__restrict__ coefs,
                                                        const uint64_t *__restrict__ lhsmod,
                                                        const FinReq *__restrict__ fr, uint32_t nfr, uint32_t total,
                                                        int nB, int nE, wv_result *__restrict__ out,
                                                        const unsigned long long *__restrict__ err) {
    const uint32_t w = blockIdx.x;
    uint32_t a = 0, b = nfr;  // the last request with out0 <= w
    while (b - a > 1) {
        const uint32_t m = (a + b) >> 1;
        if (fr[m].out0 <= w) a = m;
        else b = m;
    }
    const FinReq f = fr[a];
    const size_t per = (size_t)nB + nE;
    finalize_prime_wg(ts, pr + f.base, acc + (size_t)f.base * per, coefs + (size_t)f.base * per,
                      lhsmod + 2 * (size_t)f.base, f.n, nB, nE, w - f.out0, err, out + w);
}

// Tasks of a request-server step (one thread each): B tasks of the step's nq
// primes first, then E tasks; prime q of the step lies in the last span whose
// q0 <= q.
__global__ void __launch_bounds__(256) k_step_expand(const StepSpan *__restrict__ sp, uint32_t nsp, uint32_t nq,
                                                     int nB, int nE, const SegRec *__restrict__ segs,
                                                     SegRec *__restrict__ tasks, uint64_t *__restrict__ terms,
                                                     uint32_t *__restrict__ target) {
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    const uint64_t nbt = (uint64_t)nq * nB;
    if (t >= nbt + (uint64_t)nq * nE) return;
    const bool bern = t < nbt;
    const uint64_t k = bern ? t : t - nbt;
    const uint64_t per = bern ? (uint64_t)nB : (uint64_t)nE;
    const uint32_t q = (uint32_t)(k / per);
    const uint64_t j = k % per;
    uint32_t a = 0, b = nsp;
    while (b - a > 1) {
        const uint32_t m = (a + b) >> 1;
        if (sp[m].q0 <= q) a = m;
        else b = m;
    }
    const StepSpan s = sp[a];
    const uint64_t i = (uint64_t)s.i0 + (q - s.q0);
    const uint64_t g = s.seg0 + (bern ? i * nB + j : (uint64_t)s.nreq * nB + i * nE + j);
    const SegRec r = segs[g];
    tasks[t] = r;
    terms[t] = r.len;
    target[t] = (uint32_t)g;
}


// ==========================================================================
// launchers
// ==========================================================================

static unsigned blocks_for(uint64_t n, unsigned per) { return (unsigned)((n + per - 1) / per + (n == 0)); }

// A dispatch holds fewer than 2^32 work-items (the packet's grid size is 32
// bits): launches of one thread per item refuse larger counts instead of
// running a truncated grid.
static bool too_many(uint64_t items) { return items >= (1ull << 32) - 256; }

hipError_t launch_base_sieve(hipStream_t st, uint32_t *out, uint32_t *n_out) {
    hipLaunchKernelGGL(k_base_sieve, dim3(1), dim3(1024), 0, st, out, n_out);
    return hipGetLastError();
}

hipError_t launch_seg_sieve(hipStream_t st, const SegDesc *desc, unsigned ns, const uint32_t *bp, uint32_t n_bp,
                            uint32_t *bits_out, uint32_t *counts) {
    hipLaunchKernelGGL(k_seg_sieve, dim3(ns), dim3(1024), 0, st, desc, bp, n_bp, bits_out, counts);
    return hipGetLastError();
}

hipError_t launch_seg_compact(hipStream_t st, const SegDesc *desc, unsigned ns, const uint32_t *bits,
                              const uint64_t *off, uint64_t *out, uint64_t limit) {
    hipLaunchKernelGGL(k_seg_compact, dim3(ns), dim3(1024), 0, st, desc, bits, off, out, limit);
    return hipGetLastError();
}

hipError_t launch_seg_offsets(hipStream_t st, const uint32_t *counts, unsigned ns, uint64_t expect, uint64_t *off,
                              uint64_t *primes) {
    if (ns > 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_seg_offsets, dim3(1), dim3(256), 0, st, counts, ns, expect, off, primes);
    return hipGetLastError();
}

hipError_t launch_scan(hipStream_t st, const uint64_t *in, uint64_t n, uint64_t *out, uint64_t *tiles) {
    if (too_many(n)) return hipErrorInvalidConfiguration;
    const uint64_t nt = std::max<uint64_t>(1, (n + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(256), 0, st, in, n, out, tiles);
    hipLaunchKernelGGL(k_scan_carry, dim3(1), dim3(1024), 0, st, tiles, nt, out + n);
    hipLaunchKernelGGL(k_scan_add, dim3(blocks_for(n, 256)), dim3(256), 0, st, out, n, (const uint64_t *)tiles);
    return hipGetLastError();
}

hipError_t launch_plan(hipStream_t st, const uint64_t *primes, uint32_t n, int tb, int te, int fb, int fe, int nB,
                       int nE, TableStore ts, PrimeRec *pr, SegRec *segs, uint64_t *terms, uint64_t *coefs,
                       uint64_t *lhsmod, uint32_t prime_base) {
    hipLaunchKernelGGL(k_plan_primes, dim3(blocks_for(n, 256)), dim3(256), 0, st, primes, n, tb, te, fb, fe, ts, pr,
                       lhsmod);
    const uint64_t nseg = (uint64_t)n * (nB + nE);
    if (too_many(nseg)) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_plan_slots, dim3(blocks_for(nseg, 256)), dim3(256), 0, st, n, nB, nE, ts, pr, segs, terms,
                       coefs, prime_base);
    return hipGetLastError();
}

hipError_t launch_pick_chunk(hipStream_t st, const uint64_t *total_terms, uint64_t nseg, uint64_t chunk_cfg, uint64_t lanes,
                             uint64_t cap, uint64_t *chunk_out) {
    hipLaunchKernelGGL(k_pick_chunk, dim3(1), dim3(1), 0, st, total_terms, nseg, chunk_cfg, cap, lanes, chunk_out);
    return hipGetLastError();
}

hipError_t launch_chunk_layout(hipStream_t st, const uint64_t *terms, uint64_t nseg, uint64_t nb_slots, uint64_t *layout,
                               uint64_t *cnt, uint64_t *off, uint64_t *scan_tiles, unsigned long long *hist,
                               uint32_t *tails, uint64_t *total_chunks) {
    if (too_many(nseg)) return hipErrorInvalidConfiguration;
    unsigned long long *cursor = hist + kTailClasses;
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(2 * kTailClasses), 0, st, (uint64_t *)hist, 2 * kTailClasses,
                       (uint64_t)0);
    hipLaunchKernelGGL(k_chunk_split, dim3(blocks_for(nseg, kLayoutTile)), dim3(256), 0, st, terms, nseg, nb_slots,
                       (const uint64_t *)layout, cnt, hist);
    const hipError_t e = launch_scan(st, cnt, nseg, off, scan_tiles);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_copy_u64, dim3(1), dim3(64), 0, st, (const uint64_t *)(off + nseg), layout + 1, 1);
    hipLaunchKernelGGL(k_tail_base, dim3(1), dim3(1), 0, st, (const unsigned long long *)hist, cursor, layout,
                       total_chunks);
    hipLaunchKernelGGL(k_tail_place, dim3(blocks_for(nseg, kLayoutTile)), dim3(256), 0, st, terms, nseg, nb_slots,
                       (const uint64_t *)layout, cursor, tails);
    return hipGetLastError();
}

hipError_t launch_set_u64(hipStream_t st, uint64_t *dst, int n, uint64_t value) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, st, dst, n, value);
    return hipGetLastError();
}

hipError_t launch_copy_u64(hipStream_t st, const uint64_t *src, uint64_t *dst, int n) {
    hipLaunchKernelGGL(k_copy_u64, dim3(1), dim3(64), 0, st, src, dst, n);
    return hipGetLastError();
}

int num_sum_variants() { return kNumSumVariants; }
int sum_variant_kb(int v) { return kSumVariants[v].kb; }
int sum_variant_ke(int v) { return kSumVariants[v].ke; }

hipError_t sum_variant_occupancy(int v, int *blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, kSumVariants[v].fn, 256, 0);
}

hipError_t launch_sum(hipStream_t st, int v, unsigned grid, const SegRec *segs, const uint64_t *off, uint32_t nseg,
                      const PrimeRec *pr, const uint64_t *layout, const uint32_t *tails, Pair *partials,
                      Pair *seg_pairs, unsigned long long *counter, uint64_t end, unsigned long long *err) {
    hipLaunchKernelGGL(kSumVariants[v].fn, dim3(grid), dim3(256), 0, st, segs, off, nseg, pr, layout, tails,
                       partials, seg_pairs, counter, end, err);
    return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t st, const SegRec *segs, const uint64_t *off, uint32_t nseg, const PrimeRec *pr,
                         const Pair *partials, const uint64_t *layout, Pair *seg_pairs) {
    // a wave per 64 sums, at most 2^20 workgroups (2^28 work-items; a
    // dispatch holds < 2^32)
    const unsigned grid = std::min<unsigned>(blocks_for((uint64_t)nseg, 256), 1u << 20);
    hipLaunchKernelGGL(k_reduce, dim3(grid), dim3(256), 0, st, segs, off, nseg, pr, partials, layout, seg_pairs);
    return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t st, TableStore ts, const PrimeRec *pr, const Pair *sp, const uint64_t *coefs,
                           const uint64_t *lhsmod, uint32_t n, int nB, int nE, wv_result *out,
                           const unsigned long long *err) {
    if (n == 0) return hipSuccess;
    if (too_many((uint64_t)n * 256)) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_finalize_wg, dim3(n), dim3(256), 0, st, ts, pr, sp, coefs, lhsmod, n, nB, nE, out, err);
    return hipGetLastError();
}

hipError_t launch_sum_values(hipStream_t st, const SegRec *segs, const PrimeRec *pr, const Pair *sp, uint64_t nseg,
                             uint64_t *out) {
    if (too_many(nseg)) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_sum_values, dim3(blocks_for(nseg, 256)), dim3(256), 0, st, segs, pr, sp, nseg, out);
    return hipGetLastError();
}

hipError_t launch_fold(hipStream_t st, const SegRec *tasks, const uint32_t *target, const Pair *tp, uint32_t ntask,
                       const PrimeRec *pr, Pair *acc) {
    hipLaunchKernelGGL(k_fold, dim3(blocks_for(ntask, 256)), dim3(256), 0, st, tasks, target, tp, ntask, pr, acc);
    return hipGetLastError();
}

hipError_t launch_step_expand(hipStream_t st, const StepSpan *sp, uint32_t nsp, uint32_t nq, int nB, int nE,
                              const SegRec *segs, SegRec *tasks, uint64_t *terms, uint32_t *target) {
    const uint64_t nt = (uint64_t)nq * (nB + nE);
    if (too_many(nt) || nsp == 0) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_step_expand, dim3(blocks_for(nt, 256)), dim3(256), 0, st, sp, nsp, nq, nB, nE, segs, tasks,
                       terms, target);
    return hipGetLastError();
}

hipError_t launch_finalize_multi(hipStream_t st, TableStore ts, const PrimeRec *pr, const Pair *acc,
                                 const uint64_t *coefs, const uint64_t *lhsmod, const FinReq *fr, uint32_t nfr,
                                 uint32_t total, int nB, int nE, wv_result *out, const unsigned long long *err) {
    if (too_many((uint64_t)total * 256) || nfr == 0) return hipErrorInvalidConfiguration;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize_multi, dim3(total), dim3(256), 0, st, ts, pr, acc, coefs, lhsmod, fr, nfr, total, nB,
                       nE, out, err);
    return hipGetLastError();
}

hipError_t launch_fill_pairs(hipStream_t st, Pair *p, uint64_t n, uint64_t c0, uint64_t c1) {
    if (too_many(n)) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_fill_pairs, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, c0, c1);
    return hipGetLastError();
}

hipError_t launch_copy_pad(hipStream_t st, const uint64_t *src, uint64_t n, uint64_t *dst, uint64_t n_pad) {
    hipLaunchKernelGGL(k_copy_pad, dim3(blocks_for(n_pad, 256)), dim3(256), 0, st, src, n, dst, n_pad);
    return hipGetLastError();
}

// Residue statistics of Sections 3 and 5: bin k = floor((2s + p) bins / (2p))
// of the symmetric residue s in (-p/2, p/2] (2s + p in [1, 2p - 1], so k is in
// [0, bins); the product is below 2^57 for p < 2^40, bins <= 2^16), and the
// near misses |s| < bound.
__global__ void __launch_bounds__(256) k_stats(const wv_result *__restrict__ res, uint32_t n, uint32_t bins,
                                               uint64_t bound, unsigned long long *__restrict__ hist,
                                               wv_near *__restrict__ near, unsigned long long *__restrict__ near_n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const wv_result r = res[i];
    const uint64_t p = r.p;
    const uint64_t half = (p - 1) / 2;
    for (int w = 0; w < 2; w++) {
        const uint64_t v = w == 0 ? r.b : r.e;
        const int64_t s = v > half ? (int64_t)v - (int64_t)p : (int64_t)v;
        const uint64_t k = (uint64_t)(2 * s + (int64_t)p) * bins / (2 * p);
        atomicAdd(&hist[(uint64_t)w * bins + k], 1ull);
        const uint64_t a = s < 0 ? (uint64_t)(-s) : (uint64_t)s;
        if (a < bound) {
            const unsigned long long slot = atomicAdd(near_n, 1ull);
            if (slot < 2ull * n) near[slot] = wv_near{p, s, (uint32_t)(w == 0 ? WV_NEAR_B : WV_NEAR_E), 0u};
        }
    }
}

hipError_t launch_stats(hipStream_t st, const wv_result *res, uint32_t n, uint32_t bins, uint64_t bound,
                        unsigned long long *hist, wv_near *near, unsigned long long *near_n) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_stats, dim3(blocks_for(n, 256)), dim3(256), 0, st, res, n, bins, bound, hist, near, near_n);
    return hipGetLastError();
}

hipError_t launch_copy_results(hipStream_t st, const wv_result *src, uint64_t n, wv_result *dst) {
    hipLaunchKernelGGL(k_copy_results, dim3(blocks_for(n, 256)), dim3(256), 0, st, src, n, dst);
    return hipGetLastError();
}

}  // namespace wv
