// wv_irregular.hip -- irregular and E-irregular pairs: B_{2k} mod p and
// E_{2k} mod p for every 2 <= 2k <= p - 3 (Section 1), from the paper's
// congruences for general index:
//
//   C_k(a,b,c) B_{2k} == sum_i S_{2k-1}(x_i, y_i)   (mod p)     (Section 2:
//     the family (2, b, b+1) over sum_{m <= b/2} (m/(b+1), m/b): b = 3, i.e.
//     (1/4, 1/3), for every k, then b = 4, 5, ... where C_k(2,3,4) vanishes),
//   C_k(a,b,c) = (a^{p-2k} + b^{p-2k} - c^{p-2k} - 1) / (4k),
//   (-1)^k 4^{k-1} (9^k + 1) E_t == 2^t (S_t(0, 1/12) - S_t(5/12, 1/2))
//     (mod p), t = p - 1 - 2k  (eqnEMac2, Section 4: McIntosh's congruence
//     with one subdivision), and where 9^k == -1 (mod p)
//   (-1)^k 4^{2k-1} E_t == S_t(0, 1/4)   (mod p)  (eqnE1, sign read as (-1)^k),
//
// with S_l(x, y) = sum_{xp < s < yp} s^l (eqnDefnS) for positive l.  Every k
// needs its own exponent, so the power sums of each range are computed for all
// exponents at once: a wave owns 1024 consecutive s (16 per lane) and a block
// of up to 2048 exponents, steps x <- x s^2 through them, and the partial sums
// go through LDS (one transpose per 32 exponents) into exact double-precision
// totals (integers below 2^53, so the order of the atomic additions does not
// matter).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "sum_core.hpp"
#include "wv_ctx.hpp"

namespace wv {
namespace {

struct IrrTask {          // +- sum_{lo <= s < hi} s^t for t = t0, t0 + 2, ..., t0 + 2 (nt - 1)
    uint64_t p, lo, hi;
    uint64_t out;         // index in V of the first exponent's total (tasks may share it)
    uint32_t t0, nt;
    uint32_t ct;          // matrix-core path: exponents per row = 16 ct (1 <= ct <= 8)
    uint32_t neg;         // 1: the sums enter V negated
};

struct IrrPrime {         // one prime of a batch
    uint64_t p;
    uint64_t vb, ve;      // its Bernoulli (odd t = 2k - 1) and Euler (even t = 2k) totals in V
    uint64_t res;         // index of its first residue in the b / e output arrays
    uint32_t nt;          // (p - 3) / 2
    uint32_t pad;
};

struct IrrFix {           // an index whose first congruence degenerates (its left side is 0 mod p)
    uint32_t prime, k;    // Bernoulli side: B_{2k}; Euler side: E_{2k}
};

constexpr int kIrrLaneS = 16;                        // s per lane
constexpr uint64_t kIrrWaveS = 64 * kIrrLaneS;       // s per wave (one work unit)
constexpr int kIrrBlock = 32;                        // exponents per transpose
constexpr uint32_t kIrrUnitT = 2048;                 // exponents per work unit
constexpr int kIrrStride = 65;                       // LDS row stride (doubles)
constexpr uint64_t kIrrMaxV = 1ull << 27;            // totals per batch (1 GiB)
constexpr uint64_t kIrrMaxUnits = (1ull << 24) - 64;  // units per launch (fewer than 2^32 work-items)

__host__ __device__ inline uint64_t floor_div(uint64_t a, uint64_t b) { return a / b; }

// first and one-past-last s of x p < s < y p, x = xa/xb, y = ya/yb (p prime > xb, yb)
__host__ __device__ inline void open_range(uint64_t p, uint64_t xa, uint64_t xb, uint64_t ya, uint64_t yb,
                                           uint64_t &lo, uint64_t &hi) {
    lo = floor_div(xa * p, xb) + 1;
    hi = ya * p % yb ? floor_div(ya * p, yb) + 1 : ya * p / yb;   // s < y p
    if (hi < lo) hi = lo;
}

__device__ inline double fpow_e(double a, uint64_t e, const Fmod &f) {
    double r = 1.0;
    while (e) {
        if (e & 1) r = f_mulmod(r, a, f);
        a = f_mulmod(a, a, f);
        e >>= 1;
    }
    return r;
}

// a^e for e < 8 without branches
__device__ inline double fpow_lt8(double a, uint32_t e, const Fmod &f) {
    const double a2 = f_mulmod(a, a, f), a4 = f_mulmod(a2, a2, f);
    double r = (e & 1) ? a : 1.0;
    const double r2 = f_mulmod(r, a2, f);
    r = (e & 2) ? r2 : r;
    const double r4 = f_mulmod(r, a4, f);
    return (e & 4) ? r4 : r;
}

__device__ inline uint64_t u_pow(uint64_t a, uint64_t e, const Fmod &f) {
    return f_canon(fpow_e((double)a, e, f), f);
}

// C_k(a, b, c) mod p for 1 <= k <= (p - 3) / 2
__device__ inline uint64_t c_k(uint64_t a, uint64_t b, uint64_t c, uint64_t k, const Fmod &f, uint64_t p) {
    const uint64_t e = p - 2 * k;
    double num = fpow_e((double)a, e, f) + fpow_e((double)b, e, f) - fpow_e((double)c, e, f) - 1.0;
    const uint64_t n = f_canon(f_reduce(num, f), f);
    const uint64_t inv4k = u_pow((4 * k) % p, p - 2, f);
    return f_canon(f_mulmod((double)n, (double)inv4k, f), f);
}

// ---------------------------------------------------------------------------
// power sums for all exponents
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_irr_sum(const IrrTask *__restrict__ tasks,
                                                 const uint64_t *__restrict__ unit_off, uint32_t ntask,
                                                 uint64_t nunits, double *__restrict__ V) {
    __shared__ double lds[4][kIrrBlock * kIrrStride];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t unit = (uint64_t)blockIdx.x * 4 + wave;   // wave-uniform
    if (unit >= nunits) return;
    const uint32_t j = __builtin_amdgcn_readfirstlane(find_seg(unit_off, ntask, unit));
    const IrrTask T = tasks[j];
    Fmod f;
    f.p = (double)T.p;
    f.pinv = 1.0 / f.p;
    // unit = (s chunk, exponent block): 1024 s times at most kIrrUnitT exponents
    const uint32_t nblk = (T.nt + kIrrUnitT - 1) / kIrrUnitT;
    const uint64_t u = unit - unit_off[j];
    const uint32_t e_first = (uint32_t)(u % nblk) * kIrrUnitT;
    const uint32_t e_end = min(T.nt, e_first + kIrrUnitT);
    const uint64_t s0 = T.lo + (u / nblk) * kIrrWaveS + lane;
    double x[kIrrLaneS], sq[kIrrLaneS];
WV_UNROLL
    for (int m = 0; m < kIrrLaneS; m++) {
        const uint64_t s = s0 + 64 * (uint64_t)m;
        const double sd = (double)s;
        const double s2 = f_mulmod(sd, sd, f);
        const bool in = s < T.hi;
        // s^(t0 + 2 e_first)
        const double xs = fpow_e(sd, T.t0 + 2 * (uint64_t)e_first, f);
        x[m] = in ? xs : 0.0;
        sq[m] = in ? s2 : 0.0;
    }
    double *L = lds[wave];
    for (uint32_t b0 = e_first; b0 < e_end; b0 += kIrrBlock) {
#pragma unroll 2
        for (int e = 0; e < kIrrBlock; e++) {
            double a = 0.0;
WV_UNROLL
            for (int m = 0; m < kIrrLaneS; m++) a += x[m];   // |a| < 16 * 0.574 p, exact
WV_UNROLL
            for (int m = 0; m < kIrrLaneS; m++) x[m] = f_mulmod(x[m], sq[m], f);
            L[e * kIrrStride + lane] = a;
        }
        // the wave's own LDS rows: complete its writes before reading across lanes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // lane l and l + 32 each sum half of exponent (l & 31)'s row
        const int row = lane & 31, half = lane >> 5;
        double t = 0.0;
        for (int m = 0; m < 32; m++) t += L[row * kIrrStride + half * 32 + m];
        t += __shfl_xor(t, 32, 64);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (half == 0 && b0 + row < e_end) atomicAdd(&V[T.out + b0 + row], T.neg ? -t : t);
    }
}

// The same totals as a dense contraction on the matrix cores, for p < 2^24:
// with e = N m + j (N = 16 ct exponents per row, ct chosen per task so that
// the rows fill whole row blocks), s^(t0 + 2e) = A[m][s] B[s][j],
// A[m][s] = s^(t0 + 2N m), B[s][j] = s^(2j), so V[m][j] = sum_s A[m][s] B[s][j].  Residues below 0.574p
// make every product an integer below 0.33 p^2 (< 2^46.4), so the f64
// multiply-adds are exact while a partial sum stays below 2^53: the
// accumulators are reduced mod p after every `period` chunks of 32 s, the
// most whose products stay below 2^52 (32 chunks = 1024 s for p < 2^21, one
// chunk near 2^24), and before their atomic additions.  A
// workgroup takes (task, 128 rows of m, kMmaSb s) with twelve waves in two roles: four producer waves
// build the A (128 x 32) and transposed B (N x 32) slices of the next 32 s in
// one LDS buffer while eight consumer waves run v_mfma_f64_16x16x4 on the
// other (each its 16 rows x N columns, ct operations per 4 s), one barrier per
// 32 s.  Each SIMD holds two consumer waves (one issues while the other waits
// on LDS) and one producer wave, so the table arithmetic on the vector ALU
// overlaps the matrix cores.
constexpr int kMmaRows = 128;                // rows of m per workgroup
constexpr int kMmaKc = 32;                   // s per LDS chunk
constexpr uint64_t kMmaSb = 1024;            // s per workgroup
constexpr uint32_t kMmaReduceMax = 1024 / kMmaKc;   // chunks between reductions of the accumulators, at most
constexpr uint64_t kIrrMmaMaxP = 1ull << 24;
constexpr int kMmaConsumers = 512;           // 8 consumer waves, 16 rows each
constexpr int kMmaThreads = kMmaConsumers + 256;   // and 4 producer waves
constexpr uint64_t kMmaMaxGrid = 1ull << 22;       // workgroups per launch (2^22 x 768 < 2^32 work-items)
// LDS row stride (doubles) of A and of the transposed B: a wave's fragment
// reads (16 rows x 4 s) then touch each bank pair at most twice
constexpr int kMmaAs = kMmaKc + 4;

typedef double v4d __attribute__((ext_vector_type(4)));

// One 32-s chunk of a consumer wave: its 16 rows x 16 CT columns.  CT is
// compile-time; the LDS operands of the next 4-s step are read while the
// matrix operations of the current one run (two register sets; the group
// barriers put the reads (mask 0x100) ahead of the matrix operations (mask
// 0x8), the fence keeps them from being hoisted further).
template <int CT>
__device__ __forceinline__ void mma_chunk(const double *A, const double *B, int wave, int lane, v4d (&acc)[8]) {
    double a[2], b[2][CT];
    const double *Ar = A + (16 * wave + (lane & 15)) * kMmaAs + (lane >> 4);
    const double *Br = B + (lane & 15) * kMmaAs + (lane >> 4);
    auto load = [&](int kk, int slot) {
        a[slot] = Ar[4 * kk];
WV_UNROLL
        for (int n = 0; n < CT; n++) b[slot][n] = Br[16 * n * kMmaAs + 4 * kk];
    };
    load(0, 0);
WV_UNROLL
    for (int kk = 0; kk < kMmaKc / 4; kk++) {
        const int cur = kk & 1;
        if (kk + 1 < kMmaKc / 4) load(kk + 1, cur ^ 1);
WV_UNROLL
        for (int n = 0; n < CT; n++)
            acc[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[cur], b[cur][n], acc[n], 0, 0, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1 + CT, 0);
        __builtin_amdgcn_sched_group_barrier(0x8, CT, 0);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The workgroup's unit (task T, row block rb of M rows, s in [sb0, sb1)) with
// N = 16 CT exponents per row; CT is compile-time so that each width has its
// own accumulators and straight-line matrix code.
template <int CT>
__device__ __forceinline__ void irr_mma_unit(const IrrTask &T, const Fmod &f, uint32_t period, uint32_t rb, uint32_t M,
                                             uint64_t sb0, uint64_t sb1, double (&As)[2][kMmaRows * kMmaAs],
                                             double (&Bs)[2][kMmaRows * kMmaAs], double *__restrict__ V) {
    constexpr uint32_t N = 16 * CT;
    const uint32_t m0 = rb * kMmaRows;
    const uint32_t nchunk = (uint32_t)((sb1 - sb0 + kMmaKc - 1) / kMmaKc);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const bool producer = tid >= kMmaConsumers;   // wave-uniform
    const int ptid = tid - kMmaConsumers;

    // tables of chunk c into buffer c & 1: producer thread (q, g) takes
    // s = sb0 + 32c + q and writes rows 16g .. 16g + 15 of A (A[m][s] =
    // s^(t0 + 2N(m0 + m))) and of the transposed B (Bt[j][s] = s^(2j); rows
    // j >= N are written and never read).  Every power comes from s^2, s^16,
    // s^32, s^(2N) = (s^32)^CT and its squares; the 16 entries of each table
    // run as two chains of 8, so a thread carries four independent chains.
    auto produce = [&](uint32_t c) {
        double *A = As[c & 1];
        double *Bt = Bs[c & 1];
        const int q = ptid & 31, g = ptid >> 5;
        const uint64_t sv = sb0 + (uint64_t)c * kMmaKc + q;
        const bool in = sv < sb1;
        const double sd = (double)sv;
        const double s2 = f_mulmod(sd, sd, f);
        double s16 = s2;
WV_UNROLL
        for (int i = 0; i < 3; i++) s16 = f_mulmod(s16, s16, f);   // s^16
        const double h = f_mulmod(s16, s16, f);                    // s^32
        const double step = fpow_e(h, CT, f);                      // s^(2N)
        double step8 = step;
WV_UNROLL
        for (int i = 0; i < 3; i++) step8 = f_mulmod(step8, step8, f);   // s^(16N)
        const double h16 = f_mulmod(step8, step8, f);                   // s^(32N)
        double h128 = h16;
WV_UNROLL
        for (int i = 0; i < 3; i++) h128 = f_mulmod(h128, h128, f);   // s^(256N)
        // s^(t0) s^(256N rb) s^(32N g) = s^(t0 + 2N (m0 + 16 g))
        const double base = f_mulmod(fpow_e(h128, rb, f), fpow_e(sd, T.t0, f), f);
        double xa0 = f_mulmod(base, fpow_lt8(h16, (uint32_t)g, f), f);
        double xa1 = f_mulmod(xa0, step8, f);
        double xb0 = fpow_lt8(h, (uint32_t)g, f);                      // s^(32g)
        double xb1 = f_mulmod(xb0, s16, f);
WV_UNROLL
        for (int r = 0; r < 8; r++) {
            A[(16 * g + r) * kMmaAs + q] = in ? xa0 : 0.0;
            A[(16 * g + 8 + r) * kMmaAs + q] = in ? xa1 : 0.0;
            Bt[(16 * g + r) * kMmaAs + q] = in ? xb0 : 0.0;
            Bt[(16 * g + 8 + r) * kMmaAs + q] = in ? xb1 : 0.0;
            xa0 = f_mulmod(xa0, step, f);
            xa1 = f_mulmod(xa1, step, f);
            xb0 = f_mulmod(xb0, s2, f);
            xb1 = f_mulmod(xb1, s2, f);
        }
    };

    const bool live = !producer && m0 + 16 * wave < M;   // wave-uniform
    v4d acc[8];
WV_UNROLL
    for (int n = 0; n < CT; n++) acc[n] = v4d{0.0, 0.0, 0.0, 0.0};
    if (producer) produce(0);
    __syncthreads();
    for (uint32_t c = 0; c < nchunk; c++) {
        if (producer) {
            if (c + 1 < nchunk) produce(c + 1);
        } else if (live) {
            mma_chunk<CT>(As[c & 1], Bs[c & 1], wave, lane, acc);
            if (c % period == period - 1) {
WV_UNROLL
                for (int n = 0; n < CT; n++)
WV_UNROLL
                    for (int r = 0; r < 4; r++) acc[n][r] = f_reduce(acc[n][r], f);
            }
        }
        __syncthreads();
    }
    if (!live) return;
    // element r of lane l of a 16 x 16 tile is row l / 16 + 4 r, column l % 16
WV_UNROLL
    for (int n = 0; n < CT; n++) {
WV_UNROLL
        for (int r = 0; r < 4; r++) {
            const uint32_t m = m0 + 16 * wave + (lane >> 4) + 4 * r;
            const uint64_t e = (uint64_t)N * m + 16 * n + (lane & 15);
            if (m < M && e < T.nt) {
                const double v = f_reduce(acc[n][r], f);
                atomicAdd(&V[T.out + e], T.neg ? -v : v);
            }
        }
    }
}

__global__ void __launch_bounds__(kMmaThreads) k_irr_mma(const IrrTask *__restrict__ tasks,
                                                         const uint64_t *__restrict__ unit_off, uint32_t ntask,
                                                         uint64_t nunits, uint64_t unit_base, double *__restrict__ V) {
    __shared__ double As[2][kMmaRows * kMmaAs];
    __shared__ double Bs[2][kMmaRows * kMmaAs];
    const uint64_t unit = unit_base + blockIdx.x;
    if (unit >= nunits) return;   // whole workgroup
    const uint32_t j = find_seg(unit_off, ntask, unit);
    const IrrTask T = tasks[j];
    Fmod f;
    f.p = (double)T.p;
    f.pinv = 1.0 / f.p;
    const uint32_t N = 16 * T.ct;   // exponents per row
    const uint32_t M = (T.nt + N - 1) / N;
    const uint32_t rbs = (M + kMmaRows - 1) / kMmaRows;
    const uint64_t u = unit - unit_off[j];
    const uint32_t rb = (uint32_t)(u % rbs);
    const uint64_t sb0 = T.lo + (u / rbs) * kMmaSb;
    const uint64_t sb1 = min(T.hi, sb0 + kMmaSb);
    // chunks whose products (each below 0.33 p^2) add up to at most 2^52
    const double chunk_bound = 0.33 * f.p * f.p * kMmaKc;
    const uint32_t period = (uint32_t)fmax(1.0, fmin((double)kMmaReduceMax, floor(4503599627370496.0 / chunk_bound)));
    switch (T.ct) {   // workgroup-uniform
        case 1: irr_mma_unit<1>(T, f, period, rb, M, sb0, sb1, As, Bs, V); break;
        case 2: irr_mma_unit<2>(T, f, period, rb, M, sb0, sb1, As, Bs, V); break;
        case 3: irr_mma_unit<3>(T, f, period, rb, M, sb0, sb1, As, Bs, V); break;
        case 4: irr_mma_unit<4>(T, f, period, rb, M, sb0, sb1, As, Bs, V); break;
        case 5: irr_mma_unit<5>(T, f, period, rb, M, sb0, sb1, As, Bs, V); break;
        case 6: irr_mma_unit<6>(T, f, period, rb, M, sb0, sb1, As, Bs, V); break;
        case 7: irr_mma_unit<7>(T, f, period, rb, M, sb0, sb1, As, Bs, V); break;
        default: irr_mma_unit<8>(T, f, period, rb, M, sb0, sb1, As, Bs, V); break;
    }
}

// ---------------------------------------------------------------------------
// residues from the totals
// ---------------------------------------------------------------------------

// One thread per (prime, k): b = B_{2k} mod p from (2,3,4) unless its C_k
// vanishes (then queued for k_irr_fix), e = E_{2k} mod p from eqnEMac2 unless
// its left side vanishes (then queued for k_irr_fix_e).  Counters: [0] queued
// Bernoulli indices, [1] pairs, [2] unresolved, [3] queued Euler indices.
// Zero residues are appended to pairs as (p, 2k, kind).
__global__ void __launch_bounds__(256) k_irr_final(const IrrPrime *__restrict__ pr, const uint64_t *__restrict__ off,
                                                   uint32_t np, const double *__restrict__ V,
                                                   uint64_t *__restrict__ b_out, uint64_t *__restrict__ e_out,
                                                   IrrFix *__restrict__ fix, IrrFix *__restrict__ fix_e,
                                                   unsigned long long *__restrict__ counts,
                                                   wv_irr_pair *__restrict__ pairs, uint64_t pair_cap) {
    const uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= off[np]) return;
    const uint32_t i = find_seg(off, np, g);
    const IrrPrime P = pr[i];
    const uint64_t k = g - off[i] + 1;
    const uint64_t p = P.p;
    Fmod f;
    f.p = (double)p;
    f.pinv = 1.0 / f.p;
    // Bernoulli side: odd exponent t = 2k - 1; with x = 2^(p-2k),
    // 4k C_k(2,3,4) = x + 3^(p-2k) - x^2 - 1 =: n and B_{2k} = S 4k / n
    const uint64_t vb = f_canon(V[P.vb + k - 1], f);
    const double x2 = fpow_e(2.0, p - 2 * k, f);
    const uint64_t c = f_canon(f_reduce(x2 + fpow_e(3.0, p - 2 * k, f) - f_mulmod(x2, x2, f) - 1.0, f), f);
    if (c) {
        const double s4k = f_mulmod((double)vb, (double)((4 * k) % p), f);
        const uint64_t b = f_canon(f_mulmod(s4k, (double)u_pow(c, p - 2, f), f), f);
        if (b_out) b_out[P.res + k - 1] = b;
        if (b == 0) {
            const unsigned long long at = atomicAdd(&counts[1], 1ull);
            if (at < pair_cap) pairs[at] = wv_irr_pair{p, (uint32_t)(2 * k), 1u};
        }
    } else {
        const unsigned long long at = atomicAdd(&counts[0], 1ull);
        fix[at] = IrrFix{i, (uint32_t)k};
    }
    // Euler side: even exponent t = 2k, left-side index k' = (p - 1 - t) / 2.
    // eqnEMac2: (-1)^k' 4^(k'-1) (9^k' + 1) E_t == 2^t T, T = S_t(0, 1/12) -
    // S_t(5/12, 1/2) (the totals); by Fermat 4^(k'-1) = 2^(-2-t) and 9^k' =
    // 3^(-t), so E_t = (-1)^k' 4^(t+1) 3^t T / (3^t + 1), queued for eqnE1
    // where 3^t == -1.
    const uint64_t t = 2 * k;
    const uint64_t kk = (p - 1 - t) / 2;
    const double pow3 = fpow_e(3.0, t, f);
    const uint64_t w = f_canon(pow3 + 1.0, f);
    if (w) {
        const double pow4 = f_mulmod(4.0, fpow_e(16.0, k, f), f);   // 4^(t+1) = 4 16^k
        const double num = f_mulmod(f_mulmod((double)f_canon(V[P.ve + k - 1], f), pow4, f), pow3, f);
        uint64_t e = f_canon(f_mulmod(num, (double)u_pow(w, p - 2, f), f), f);
        if ((kk & 1) && e) e = p - e;
        if (e_out) e_out[P.res + k - 1] = e;
        if (e == 0) {
            const unsigned long long at = atomicAdd(&counts[1], 1ull);
            if (at < pair_cap) pairs[at] = wv_irr_pair{p, (uint32_t)t, 2u};
        }
    } else {
        const unsigned long long at = atomicAdd(&counts[3], 1ull);
        fix_e[at] = IrrFix{i, (uint32_t)k};
    }
}

// One wave per queued Euler index: eqnE1, (-1)^k' 4^(2k'-1) E_t == S_t(0,
// 1/4) with t = 2k and k' = (p - 1 - t) / 2, the sum evaluated directly (one
// power per s); 4^-(2k'-1) = 4^(t+1) by Fermat.
__global__ void __launch_bounds__(256) k_irr_fix_e(const IrrPrime *__restrict__ pr, const IrrFix *__restrict__ fix,
                                                   const unsigned long long *__restrict__ nfix_ptr,
                                                   uint64_t *__restrict__ e_out, unsigned long long *__restrict__ counts,
                                                   wv_irr_pair *__restrict__ pairs, uint64_t pair_cap) {
    const uint64_t w = ((uint64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w >= *nfix_ptr) return;
    const IrrFix F = fix[w];
    const IrrPrime P = pr[F.prime];
    const uint64_t p = P.p, t = 2 * (uint64_t)F.k, kk = (p - 1 - t) / 2;
    Fmod f;
    f.p = (double)p;
    f.pinv = 1.0 / f.p;
    uint64_t lo, hi;
    open_range(p, 0, 1, 1, 4, lo, hi);
    double acc = 0.0;   // exact: fewer than p terms below 0.574 p in magnitude
    for (uint64_t s = lo + lane; s < hi; s += 64) acc += fpow_e((double)s, t, f);
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane != 0) return;
    const double pow4 = f_mulmod(4.0, fpow_e(16.0, F.k, f), f);
    uint64_t e = f_canon(f_mulmod((double)f_canon(f_reduce(acc, f), f), pow4, f), f);
    if ((kk & 1) && e) e = p - e;
    if (e_out) e_out[P.res + F.k - 1] = e;
    if (e == 0) {
        const unsigned long long at = atomicAdd(&counts[1], 1ull);
        if (at < pair_cap) pairs[at] = wv_irr_pair{p, (uint32_t)t, 2u};
    }
}

// One wave per queued k: the next members of the family (2, b, b + 1) of
// Section 2 (C_k(2,b,b+1) B_{2k} == sum_{m=1}^{floor(b/2)} S_{2k-1}(m/(b+1), m/b);
// b = 5 is eqnVandiver) for b = 4, 5, ..., kIrrMaxB with p not dividing
// b (b + 1), each sum evaluated directly (one power per s).  At 2k = (p+1)/2
// every C_k is a sum of Legendre symbols, and the first b with
// (b/p) != ((b+1)/p) (or b = 3 when (2/p) = -1) resolves it.  A k where all
// of them degenerate is marked with the residue UINT64_MAX and counted in
// counts[2].
constexpr uint64_t kIrrMaxB = 64;

__global__ void __launch_bounds__(256) k_irr_fix(const IrrPrime *__restrict__ pr, const IrrFix *__restrict__ fix,
                                                 const unsigned long long *__restrict__ nfix_ptr,
                                                 uint64_t *__restrict__ b_out, unsigned long long *__restrict__ counts,
                                                 wv_irr_pair *__restrict__ pairs, uint64_t pair_cap) {
    const uint64_t w = ((uint64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w >= *nfix_ptr) return;
    const IrrFix F = fix[w];
    const IrrPrime P = pr[F.prime];
    const uint64_t p = P.p, k = F.k;
    Fmod f;
    f.p = (double)p;
    f.pinv = 1.0 / f.p;
    uint64_t b = UINT64_MAX;
    for (uint64_t bb = 4; bb <= kIrrMaxB && b == UINT64_MAX; bb++) {
        if (bb % p == 0 || (bb + 1) % p == 0) continue;
        const uint64_t c = c_k(2, bb, bb + 1, k, f, p);
        if (!c) continue;
        double acc = 0.0;   // exact: fewer than p terms below 0.574 p in magnitude
        for (uint64_t m = 1; m <= bb / 2; m++) {
            uint64_t lo, hi;
            open_range(p, m, bb + 1, m, bb, lo, hi);
            for (uint64_t s = lo + lane; s < hi; s += 64) acc += fpow_e((double)s, 2 * k - 1, f);
        }
        for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
        const uint64_t S = f_canon(f_reduce(acc, f), f);
        b = f_canon(f_mulmod((double)S, (double)u_pow(c, p - 2, f), f), f);
    }
    if (lane != 0) return;
    if (b_out) b_out[P.res + k - 1] = b;
    if (b == UINT64_MAX) {
        atomicAdd(&counts[2], 1ull);
    } else if (b == 0) {
        const unsigned long long at = atomicAdd(&counts[1], 1ull);
        if (at < pair_cap) pairs[at] = wv_irr_pair{p, (uint32_t)(2 * k), 1u};
    }
}

__global__ void k_irr_zero(double *__restrict__ v, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) v[i] = 0.0;
}

unsigned grid_for(uint64_t n, unsigned per) { return (unsigned)((n + per - 1) / per + (n == 0)); }

// One batch of primes (all in [5, WV_IRR_P_MAX)): residues into the device
// arrays b_out / e_out (may be null) at each prime's res offset, zero pairs
// appended to the device list.  Returns the counters {fixups, pairs, unresolved}.
int irr_batch(wv_ctx *c, const std::vector<uint64_t> &ps, uint64_t *d_b, uint64_t *d_e, uint64_t pair_cap,
              uint64_t counts_out[3], float *ms_sum, double *pairs_done) {
    hipStream_t st = c->stream;
    std::vector<IrrTask> tasks;
    std::vector<uint64_t> units(1, 0);
    std::vector<IrrPrime> prs;
    std::vector<uint64_t> roff(1, 0);
    uint64_t vn = 0, res = 0;
    double work = 0.0;
    // the matrix-core path while every partial sum stays exact (unless the
    // vector path is requested)
    const bool mma = c->irr_path != 1 && *std::max_element(ps.begin(), ps.end()) < kIrrMmaMaxP;
    // exponents per row 16 ct: the least work over whole row blocks, each row
    // costing its N multiply-adds per s plus about 8 for building its A entry
    // (one modular product), ties to wider rows
    auto cols_of = [](uint64_t nt) -> uint32_t {
        uint32_t best = 8;
        uint64_t best_w = UINT64_MAX;
        for (uint32_t ct = 8; ct >= 1; ct--) {
            const uint64_t N = 16 * ct, M = (nt + N - 1) / N;
            const uint64_t w = (M + kMmaRows - 1) / kMmaRows * kMmaRows * (N + 8);
            if (w < best_w) best_w = w, best = ct;
        }
        return best;
    };
    auto units_of = [&](uint64_t lo, uint64_t hi, uint64_t nt) -> uint64_t {
        if (mma) {
            const uint64_t N = 16 * cols_of(nt), M = (nt + N - 1) / N;
            return (M + kMmaRows - 1) / kMmaRows * ((hi - lo + kMmaSb - 1) / kMmaSb);
        }
        return (hi - lo + kIrrWaveS - 1) / kIrrWaveS * ((nt + kIrrUnitT - 1) / kIrrUnitT);
    };
    for (uint64_t p : ps) {
        const uint32_t nt = (uint32_t)((p - 3) / 2);
        IrrPrime P{p, vn, vn + nt, res, nt, 0};
        uint64_t lo, hi;
        open_range(p, 1, 4, 1, 3, lo, hi);   // Bernoulli: (1/4, 1/3), odd exponents from 1
        tasks.push_back(IrrTask{p, lo, hi, vn, 1, nt, cols_of(nt), 0});   // Bernoulli: +S(1/4, 1/3)
        units.push_back(units.back() + units_of(lo, hi, nt));
        work += (double)(hi - lo) * nt;
        // Euler (eqnEMac2): S(0, 1/12) - S(5/12, 1/2) into the same totals,
        // even exponents from 2
        open_range(p, 0, 1, 1, 12, lo, hi);
        tasks.push_back(IrrTask{p, lo, hi, vn + nt, 2, nt, cols_of(nt), 0});
        units.push_back(units.back() + units_of(lo, hi, nt));
        work += (double)(hi - lo) * nt;
        open_range(p, 5, 12, 1, 2, lo, hi);
        tasks.push_back(IrrTask{p, lo, hi, vn + nt, 2, nt, cols_of(nt), 1});
        units.push_back(units.back() + units_of(lo, hi, nt));
        work += (double)(hi - lo) * nt;
        vn += 2 * (uint64_t)nt;
        res += nt;
        prs.push_back(P);
        roff.push_back(roff.back() + nt);
    }
    const uint64_t nunits = units.back();
    const uint32_t ntask = (uint32_t)tasks.size(), np = (uint32_t)prs.size();
    WV_TRY(ensure(c, c->irr_tasks, tasks.size() * sizeof(IrrTask)));
    WV_TRY(ensure(c, c->irr_units, units.size() * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->irr_primes, prs.size() * sizeof(IrrPrime)));
    WV_TRY(ensure(c, c->irr_roff, roff.size() * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->irr_v, std::max<uint64_t>(vn, 1) * sizeof(double)));
    WV_TRY(ensure(c, c->irr_fix, 2 * std::max<uint64_t>(res, 1) * sizeof(IrrFix)));   // both sides' queues
    WV_TRY(ensure(c, c->irr_counts, 4 * sizeof(unsigned long long)));
    WV_HIP(hipMemcpyAsync(c->irr_tasks.ptr, tasks.data(), tasks.size() * sizeof(IrrTask), hipMemcpyHostToDevice, st));
    WV_HIP(hipMemcpyAsync(c->irr_units.ptr, units.data(), units.size() * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    WV_HIP(hipMemcpyAsync(c->irr_primes.ptr, prs.data(), prs.size() * sizeof(IrrPrime), hipMemcpyHostToDevice, st));
    WV_HIP(hipMemcpyAsync(c->irr_roff.ptr, roff.data(), roff.size() * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_irr_zero, dim3(grid_for(vn, 256)), dim3(256), 0, st, as<double>(c->irr_v), vn);
    WV_HIP(launch_set_u64(st, as<uint64_t>(c->irr_counts), 4, 0));
    WV_HIP(hipEventRecord(c->ev[EV_SUM0], st));
    if (mma) {
        // one workgroup per unit, in launches of fewer than 2^32 work-items
        for (uint64_t u0 = 0; u0 < nunits; u0 += kMmaMaxGrid) {
            const uint64_t g = std::min<uint64_t>(kMmaMaxGrid, nunits - u0);
            hipLaunchKernelGGL(k_irr_mma, dim3((unsigned)g), dim3(kMmaThreads), 0, st, as<IrrTask>(c->irr_tasks),
                               as<uint64_t>(c->irr_units), ntask, nunits, u0, as<double>(c->irr_v));
        }
    } else {
        hipLaunchKernelGGL(k_irr_sum, dim3(grid_for(nunits, 4)), dim3(256), 0, st, as<IrrTask>(c->irr_tasks),
                           as<uint64_t>(c->irr_units), ntask, nunits, as<double>(c->irr_v));
    }
    WV_HIP(hipGetLastError());
    WV_HIP(hipEventRecord(c->ev[EV_SUM], st));
    auto *counts = as<unsigned long long>(c->irr_counts);
    IrrFix *fix_b = as<IrrFix>(c->irr_fix), *fix_e = fix_b + std::max<uint64_t>(res, 1);
    hipLaunchKernelGGL(k_irr_final, dim3(grid_for(res, 256)), dim3(256), 0, st, as<IrrPrime>(c->irr_primes),
                       as<uint64_t>(c->irr_roff), np, as<double>(c->irr_v), d_b, d_e, fix_b, fix_e, counts,
                       as<wv_irr_pair>(c->irr_pairs), pair_cap);
    WV_HIP(hipGetLastError());
    unsigned long long host[4];
    WV_HIP(hipMemcpyAsync(host, counts, sizeof(host), hipMemcpyDeviceToHost, st));
    WV_HIP(hipStreamSynchronize(st));
    if (host[0] || host[3]) {
        if (host[0])
            hipLaunchKernelGGL(k_irr_fix, dim3(grid_for(host[0] * 64, 256)), dim3(256), 0, st,
                               as<IrrPrime>(c->irr_primes), fix_b, counts, d_b, counts,
                               as<wv_irr_pair>(c->irr_pairs), pair_cap);
        if (host[3])
            hipLaunchKernelGGL(k_irr_fix_e, dim3(grid_for(host[3] * 64, 256)), dim3(256), 0, st,
                               as<IrrPrime>(c->irr_primes), fix_e, counts + 3, d_e, counts,
                               as<wv_irr_pair>(c->irr_pairs), pair_cap);
        WV_HIP(hipGetLastError());
        WV_HIP(hipMemcpyAsync(host, counts, sizeof(host), hipMemcpyDeviceToHost, st));
        WV_HIP(hipStreamSynchronize(st));
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, c->ev[EV_SUM0], c->ev[EV_SUM]);
    *ms_sum += ms;
    *pairs_done += work;
    for (int q = 0; q < 3; q++) counts_out[q] = host[q];
    return WV_OK;
}

// Batches of consecutive primes within the device budgets.
template <class F>
int irr_for_batches(const std::vector<uint64_t> &ps, F &&run) {
    size_t i = 0;
    while (i < ps.size()) {
        std::vector<uint64_t> b;
        uint64_t vn = 0, units = 0;
        while (i < ps.size()) {
            const uint64_t p = ps[i];
            const uint64_t v = p - 3;   // two totals per k
            // three tasks of at most p/12 s each (a bound for either kernel's units)
            const uint64_t u = 3 * (p / 12 / kIrrWaveS + 2) * ((p / 2) / kIrrUnitT + 1);
            if (!b.empty() && (vn + v > kIrrMaxV || units + u > kIrrMaxUnits)) break;
            b.push_back(p);
            vn += v;
            units += u;
            i++;
        }
        WV_TRY(run(b));
    }
    return WV_OK;
}

}  // namespace
}  // namespace wv

using namespace wv;

int wv_set_irregular_path(wv_ctx *c, int path) {
    if (!c || path < 0 || path > 2) return WV_EINVAL;
    c->irr_path = path;
    return WV_OK;
}

int wv_bernoulli_euler_all(wv_ctx *c, uint64_t p, uint64_t *b, uint64_t *e) {
    if (!c || !b || !e) return WV_EINVAL;
    if (p < 5 || p >= WV_IRR_P_MAX) return WV_EDOMAIN;
    if (!is_prime_u64(p)) return WV_ENOTPRIME;
    WV_TRY(check_device(c));
    c->stats = wv_stats{};
    const uint64_t nt = (p - 3) / 2;
    WV_TRY(ensure(c, c->irr_b, nt * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->irr_e, nt * sizeof(uint64_t)));
    WV_TRY(ensure(c, c->irr_pairs, 64 * sizeof(wv_irr_pair)));
    uint64_t counts[3];
    float ms = 0.f;
    double work = 0.0;
    WV_TRY(irr_batch(c, std::vector<uint64_t>{p}, as<uint64_t>(c->irr_b), as<uint64_t>(c->irr_e), 0, counts, &ms,
                     &work));
    WV_HIP(hipMemcpyAsync(b, c->irr_b.ptr, nt * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
    WV_HIP(hipMemcpyAsync(e, c->irr_e.ptr, nt * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
    WV_HIP(hipStreamSynchronize(c->stream));
    c->stats.n_primes = 1;
    c->stats.n_terms = (uint64_t)work;
    c->stats.ms_sum = ms;
    return WV_OK;
}

int wv_irregular_pairs(wv_ctx *c, uint64_t lo, uint64_t hi, wv_irr_pair *out, size_t cap, size_t *n_out,
                       uint64_t *n_primes, uint64_t *n_unresolved) {
    if (!c || !n_out || lo > hi || (cap && !out)) return WV_EINVAL;
    if (hi > WV_IRR_P_MAX) return WV_EDOMAIN;
    WV_TRY(check_device(c));
    c->stats = wv_stats{};
    *n_out = 0;
    // the primes of [lo, hi), sieved on the device in groups of segments
    std::vector<SegDesc> d;
    window_descs(lo, hi, d);
    std::vector<uint64_t> ps;
    for (size_t g = 0; g < d.size(); g += kMaxBatchSegs) {
        const size_t ns = std::min(kMaxBatchSegs, d.size() - g);
        std::vector<uint32_t> counts(ns);
        WV_TRY(sieve_count(c, d.data() + g, ns, true, counts.data()));
        uint64_t np = 0;
        WV_TRY(compact(c, d.data() + g, ns, counts.data(), &np));
        const size_t at = ps.size();
        ps.resize(at + np);
        if (np) {
            WV_HIP(hipMemcpyAsync(ps.data() + at, c->primes.ptr, np * sizeof(uint64_t), hipMemcpyDeviceToHost,
                                  c->stream));
            WV_HIP(hipStreamSynchronize(c->stream));
        }
    }
    std::vector<wv_irr_pair> all;
    uint64_t unresolved = 0;
    float ms = 0.f;
    double work = 0.0;
    const uint64_t pair_cap = 1ull << 20;
    WV_TRY(ensure(c, c->irr_pairs, pair_cap * sizeof(wv_irr_pair)));
    WV_TRY(irr_for_batches(ps, [&](const std::vector<uint64_t> &b) -> int {
        uint64_t counts[3];
        WV_TRY(irr_batch(c, b, nullptr, nullptr, pair_cap, counts, &ms, &work));
        if (counts[1] > pair_cap) return WV_ENOMEM;
        const size_t at = all.size();
        all.resize(at + counts[1]);
        if (counts[1]) {
            WV_HIP(hipMemcpyAsync(all.data() + at, c->irr_pairs.ptr, counts[1] * sizeof(wv_irr_pair),
                                  hipMemcpyDeviceToHost, c->stream));
            WV_HIP(hipStreamSynchronize(c->stream));
        }
        unresolved += counts[2];
        return WV_OK;
    }));
    std::sort(all.begin(), all.end(), [](const wv_irr_pair &a, const wv_irr_pair &b) {
        return a.p != b.p ? a.p < b.p : (a.two_k != b.two_k ? a.two_k < b.two_k : a.kind < b.kind);
    });
    c->stats.n_primes = ps.size();
    c->stats.n_terms = (uint64_t)work;
    c->stats.ms_sum = ms;
    if (n_primes) *n_primes = ps.size();
    if (n_unresolved) *n_unresolved = unresolved;
    *n_out = all.size();
    if (all.size() > cap) return WV_ETRUNC;
    std::copy(all.begin(), all.end(), out);
    return WV_OK;
}
