// peak.hip -- instruction-rate microbenchmarks for the rooflines of the
// term-sum kernel and the matrix-core power sums (libwvpeak.so, C ABI:
// wv_peak_rates, wv_peak_mfma_f64, wv_peak_mfma_f64_sweep).
//
// Each kernel runs NCHAIN independent dependency chains of one VALU
// instruction class per lane, so issue rate (not latency) bounds it.  The
// instruction each loop body compiles to is checked in the gfx950 assembly of
// this file (v_mad_u64_u32, v_mul_lo_u32, v_mul_hi_u32, v_mul_u32_u24,
// v_add_u32, v_lshl_add_u64, v_fma_f64).
#include <hip/hip_runtime.h>
#include <cstdint>

namespace {

constexpr int NCHAIN = 8;
constexpr int UNROLL = 16;

// Each loop body issues exactly one instance of the measured instruction per
// chain (inline asm, so the compiler can neither fold nor reorder the chain).
#define WV_PEAK_KERNEL(NAME, T, INIT, ASM, ...)                                        \
    __global__ void __launch_bounds__(256) NAME(uint64_t *out, uint32_t a, int iters) { \
        T x[NCHAIN];                                                                   \
        const T b = (T)(a | 1u) + (T)threadIdx.x;                                      \
        for (int c = 0; c < NCHAIN; c++) x[c] = INIT;                                  \
        for (int it = 0; it < iters; it++) {                                           \
            _Pragma("unroll") for (int u = 0; u < UNROLL; u++)                         \
            _Pragma("unroll") for (int c = 0; c < NCHAIN; c++) {                       \
                asm volatile(ASM : __VA_ARGS__);                                       \
            }                                                                          \
        }                                                                              \
        uint64_t s = 0;                                                                \
        for (int c = 0; c < NCHAIN; c++) s ^= (uint64_t)x[c];                          \
        out[blockIdx.x * blockDim.x + threadIdx.x] = s;                                \
    }

WV_PEAK_KERNEL(k_mullo, uint32_t, threadIdx.x + c + 1, "v_mul_lo_u32 %0, %0, %1", "+v"(x[c]) : "v"(b))
WV_PEAK_KERNEL(k_mulhi, uint32_t, threadIdx.x * 2654435761u + c, "v_mul_hi_u32 %0, %0, %1", "+v"(x[c]) : "v"(b))
WV_PEAK_KERNEL(k_mul24, uint32_t, threadIdx.x + c + 1, "v_mul_u32_u24 %0, %0, %1", "+v"(x[c]) : "v"(b))
WV_PEAK_KERNEL(k_add32, uint32_t, threadIdx.x + c, "v_add_u32 %0, %0, %1", "+v"(x[c]) : "v"(b))
WV_PEAK_KERNEL(k_add64, uint64_t, threadIdx.x + c, "v_lshl_add_u64 %0, %0, 0, %1", "+v"(x[c]) : "v"(b))
WV_PEAK_KERNEL(k_addco, uint32_t, threadIdx.x + c, "v_add_co_u32 %0, vcc, %0, %1", "+v"(x[c]) : "v"(b) : "vcc")
WV_PEAK_KERNEL(k_addc, uint32_t, threadIdx.x + c, "v_addc_co_u32 %0, vcc, %0, %1, vcc", "+v"(x[c]) : "v"(b) : "vcc")
WV_PEAK_KERNEL(k_cndmask, uint32_t, threadIdx.x + c, "v_cndmask_b32 %0, %0, %1, vcc", "+v"(x[c]) : "v"(b) : "vcc")
WV_PEAK_KERNEL(k_cmp, uint32_t, threadIdx.x + c, "v_cmp_gt_u32 vcc, %0, %1", "+v"(x[c]) : "v"(b) : "vcc")
WV_PEAK_KERNEL(k_min32, uint32_t, threadIdx.x + c, "v_min_u32 %0, %0, %1", "+v"(x[c]) : "v"(b))
WV_PEAK_KERNEL(k_mov32, uint32_t, threadIdx.x + c, "v_mov_b32 %0, %1", "+v"(x[c]) : "v"(b))
WV_PEAK_KERNEL(k_subrev, uint32_t, threadIdx.x + c, "v_sub_u32 %0, %1, %0", "+v"(x[c]) : "v"(b))

__global__ void __launch_bounds__(256) k_mad64(uint64_t *out, uint32_t a, int iters) {
    uint64_t x[NCHAIN];
    const uint32_t b = (a | 1u) + threadIdx.x;
    for (int c = 0; c < NCHAIN; c++) x[c] = threadIdx.x + c;
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int u = 0; u < UNROLL; u++)
#pragma unroll
            for (int c = 0; c < NCHAIN; c++) x[c] = (uint64_t)(uint32_t)x[c] * b + x[c];
    }
    uint64_t s = 0;
    for (int c = 0; c < NCHAIN; c++) s ^= x[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_fma64(uint64_t *out, uint32_t a, int iters) {
    double x[NCHAIN];
    const double m = 1.0 + 1e-9 * (double)(a & 7), d = 1e-7;
    for (int c = 0; c < NCHAIN; c++) x[c] = (double)(threadIdx.x + c);
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int u = 0; u < UNROLL; u++)
#pragma unroll
            for (int c = 0; c < NCHAIN; c++) x[c] = fma(x[c], m, d);
    }
    double s = 0;
    for (int c = 0; c < NCHAIN; c++) s += x[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = (uint64_t)s;
}

typedef void (*kfn)(uint64_t *, uint32_t, int);

typedef double v4d __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4_f64 back to back: NCHAIN independent 16 x 16
// accumulators per wave, 2048 flops per operation.
__global__ void __launch_bounds__(256) k_mfma64(double *out, int iters) {
    v4d acc[NCHAIN];
    for (int c = 0; c < NCHAIN; c++) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
    const double a = 1.0 + 1e-9 * threadIdx.x, b = 1.0 - 1e-9 * threadIdx.x;
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int c = 0; c < NCHAIN; c++) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    double s = 0;
    for (int c = 0; c < NCHAIN; c++) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// The same with a chosen number of accumulator chains and instruction shape:
// SHAPE 16: v_mfma_f64_16x16x4_f64 (2048 flops, 4 doubles of accumulator per
// lane); SHAPE 4: v_mfma_f64_4x4x4_4b_f64 (four 4 x 4 x 4 blocks, 512 flops,
// one double per lane).
template <int SHAPE, int NCH>
__global__ void __launch_bounds__(256) k_mfma64_var(double *out, int iters) {
    const double a = 1.0 + 1e-9 * threadIdx.x, b = 1.0 - 1e-9 * threadIdx.x;
    double s = 0;
    if constexpr (SHAPE == 16) {
        v4d acc[NCH];
        for (int c = 0; c < NCH; c++) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int c = 0; c < NCH; c++) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
        }
        for (int c = 0; c < NCH; c++) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    } else {
        double acc[NCH];
        for (int c = 0; c < NCH; c++) acc[c] = 0.0;
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int c = 0; c < NCH; c++) acc[c] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, acc[c], 0, 0, 0);
        }
        for (int c = 0; c < NCH; c++) s += acc[c];
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

typedef void (*mfn)(double *, int);

struct MfmaVar {
    int shape, chains;
    mfn fn;
};

const MfmaVar kMfmaVars[] = {
    {16, 2, k_mfma64_var<16, 2>}, {16, 4, k_mfma64_var<16, 4>},  {16, 8, k_mfma64_var<16, 8>},
    {16, 16, k_mfma64_var<16, 16>}, {4, 4, k_mfma64_var<4, 4>},  {4, 8, k_mfma64_var<4, 8>},
    {4, 16, k_mfma64_var<4, 16>},
};

}  // namespace

extern "C" {

// Measures lane-operations per second for each instruction class on device
// `dev`: rates[0..13] = v_mad_u64_u32, v_mul_lo_u32, v_mul_hi_u32,
// v_mul_u32_u24, v_add_u32, v_lshl_add_u64, v_fma_f64, v_add_co_u32,
// v_addc_co_u32, v_cndmask_b32, v_cmp_gt_u32, v_min_u32, v_mov_b32,
// v_sub_u32.  Each rate counts one instruction per lane as one operation.
// Returns 0 on success.
#define WV_PEAK_N 14
int wv_peak_count(void) { return WV_PEAK_N; }

int wv_peak_rates(int dev, double *rates) {
    if (!rates) return -1;
    if (hipSetDevice(dev) != hipSuccess) return -6;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return -6;
    const int blocks = prop.multiProcessorCount * 16;
    const int threads = 256;
    const int iters = 2048;
    uint64_t *buf = nullptr;
    if (hipMalloc(&buf, (size_t)blocks * threads * sizeof(uint64_t)) != hipSuccess) return -5;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -6;
    kfn ks[WV_PEAK_N] = {k_mad64, k_mullo, k_mulhi, k_mul24, k_add32, k_add64, k_fma64,
                         k_addco, k_addc, k_cndmask, k_cmp, k_min32, k_mov32, k_subrev};
    int rc = 0;
    for (int k = 0; k < WV_PEAK_N && rc == 0; k++) {
        hipLaunchKernelGGL(ks[k], dim3(blocks), dim3(threads), 0, 0, buf, 12345u, 16);   // warm-up
        (void)hipEventRecord(e0, 0);
        hipLaunchKernelGGL(ks[k], dim3(blocks), dim3(threads), 0, 0, buf, 12345u, iters);
        (void)hipEventRecord(e1, 0);
        if (hipEventSynchronize(e1) != hipSuccess) { rc = -6; break; }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double ops = (double)blocks * threads * iters * UNROLL * NCHAIN;
        rates[k] = ops / (ms * 1e-3);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    return rc;
}

// Dense f64 matrix rate attained on device `dev` (flops per second) by
// independent v_mfma_f64_16x16x4_f64 operations, four waves per SIMD.
// Returns 0 on success.
int wv_peak_mfma_f64(int dev, double *flops) {
    if (!flops) return -1;
    if (hipSetDevice(dev) != hipSuccess) return -6;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return -6;
    const int blocks = prop.multiProcessorCount * 4;
    const int threads = 256;
    const int iters = 8192;
    double *buf = nullptr;
    if (hipMalloc(&buf, (size_t)blocks * threads * sizeof(double)) != hipSuccess) return -5;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -6;
    int rc = 0;
    hipLaunchKernelGGL(k_mfma64, dim3(blocks), dim3(threads), 0, 0, buf, 64);   // warm-up
    (void)hipEventRecord(e0, 0);
    hipLaunchKernelGGL(k_mfma64, dim3(blocks), dim3(threads), 0, 0, buf, iters);
    (void)hipEventRecord(e1, 0);
    if (hipEventSynchronize(e1) != hipSuccess) rc = -6;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *flops = (double)blocks * (threads / 64) * iters * NCHAIN * 2048.0 / (ms * 1e-3);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    return rc;
}

// Sweep of the attained f64 matrix rate over instruction shape (16: 16x16x4,
// 4: 4x4x4 with four blocks), independent accumulator chains per wave and
// waves per SIMD (1, 2, 4, 8).  Writes up to cap rows of four doubles {shape,
// chains, waves per SIMD, flops per second} to out and returns the number of
// rows (negative on a HIP error).
int wv_peak_mfma_f64_sweep(int dev, double *out, int cap) {
    if (!out || cap < 0) return -1;
    if (hipSetDevice(dev) != hipSuccess) return -6;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return -6;
    const int threads = 256;   // four waves: one per SIMD of a CU
    const int iters = 4096;
    const int wps[] = {1, 2, 4, 8};
    double *buf = nullptr;
    if (hipMalloc(&buf, (size_t)prop.multiProcessorCount * 8 * threads * sizeof(double)) != hipSuccess) return -5;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -6;
    int n = 0, rc = 0;
    for (const MfmaVar &v : kMfmaVars) {
        for (int w : wps) {
            if (n >= cap) break;
            const int blocks = prop.multiProcessorCount * w;
            hipLaunchKernelGGL(v.fn, dim3(blocks), dim3(threads), 0, 0, buf, 32);   // warm-up
            (void)hipEventRecord(e0, 0);
            hipLaunchKernelGGL(v.fn, dim3(blocks), dim3(threads), 0, 0, buf, iters);
            (void)hipEventRecord(e1, 0);
            if (hipEventSynchronize(e1) != hipSuccess) { rc = -6; break; }
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const double per = v.shape == 16 ? 2048.0 : 512.0;
            out[4 * n + 0] = v.shape;
            out[4 * n + 1] = v.chains;
            out[4 * n + 2] = w;
            out[4 * n + 3] = (double)blocks * (threads / 64) * iters * v.chains * per / (ms * 1e-3);
            n++;
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    return rc ? rc : n;
}

}  // extern "C"
