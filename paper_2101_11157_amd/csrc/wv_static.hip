// wv_static.hip -- wv_eval_primes_static: the device-pointer evaluation of
// wv_eval_primes_async with every intermediate buffer in one fixed device
// array, for callers that cannot allocate device memory during the call.
//
// The array `scratch` below is a file-scope device variable: the loader
// places one copy on every GPU that loads the library, and it lives until the
// process ends.  Host code never names it in a kernel argument or a copy (in
// host code the name is a host-side stand-in, not a device address): the
// device address of each GPU's copy is looked up once per device, with that
// device current, by static_scratch_setup() (called from wv_create) and kept
// in a per-device table.  Every later use goes through that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "wv_ctx.hpp"

using namespace wv;

namespace {

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Carve-up of the scratch array for a batch at the maximum sizes.
constexpr size_t kOffPr = 0;
constexpr size_t kOffSegs = align256(kOffPr + WV_STATIC_MAX_PRIMES * sizeof(PrimeRec));
constexpr size_t kOffTerms = align256(kOffSegs + WV_STATIC_MAX_SLOTS * sizeof(SegRec));
constexpr size_t kOffCnt = align256(kOffTerms + WV_STATIC_MAX_SLOTS * sizeof(uint64_t));
constexpr size_t kOffOff = align256(kOffCnt + WV_STATIC_MAX_SLOTS * sizeof(uint64_t));
constexpr size_t kOffTiles = align256(kOffOff + (WV_STATIC_MAX_SLOTS + 1) * sizeof(uint64_t));
constexpr size_t kOffScal = align256(kOffTiles + (WV_STATIC_MAX_SLOTS / kScanTile + 2) * sizeof(uint64_t));
constexpr size_t kOffPartials = align256(kOffScal + 8 * sizeof(uint64_t));
constexpr size_t kOffSegPairs = align256(kOffPartials + WV_STATIC_MAX_CHUNKS * sizeof(Pair));
constexpr size_t kOffCoefs = align256(kOffSegPairs + WV_STATIC_MAX_SLOTS * sizeof(Pair));
constexpr size_t kOffLhs = align256(kOffCoefs + WV_STATIC_MAX_SLOTS * sizeof(uint64_t));
constexpr size_t kOffTails = align256(kOffLhs + 2 * WV_STATIC_MAX_PRIMES * sizeof(uint64_t));
constexpr size_t kOffHist = align256(kOffTails + WV_STATIC_MAX_SLOTS * sizeof(uint32_t));
constexpr size_t kScratchBytes = align256(kOffHist + 2 * kTailClasses * sizeof(uint64_t));
static_assert(kScratchBytes <= WV_STATIC_SCRATCH_BYTES, "scratch layout exceeds the documented size");
static_assert(WV_STATIC_MAX_CHUNKS >= 2 * WV_STATIC_MAX_SLOTS, "partial pairs must exceed twice the slots");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};   // device address of `scratch` on each device

BatchBufs carve(void *base) {
    char *b = static_cast<char *>(base);
    BatchBufs r;
    r.pr = reinterpret_cast<PrimeRec *>(b + kOffPr);
    r.segs = reinterpret_cast<SegRec *>(b + kOffSegs);
    r.terms = reinterpret_cast<uint64_t *>(b + kOffTerms);
    r.cnt = reinterpret_cast<uint64_t *>(b + kOffCnt);
    r.off = reinterpret_cast<uint64_t *>(b + kOffOff);
    r.tiles = reinterpret_cast<uint64_t *>(b + kOffTiles);
    r.scal = reinterpret_cast<uint64_t *>(b + kOffScal);
    r.partials = reinterpret_cast<Pair *>(b + kOffPartials);
    r.seg_pairs = reinterpret_cast<Pair *>(b + kOffSegPairs);
    r.coefs = reinterpret_cast<uint64_t *>(b + kOffCoefs);
    r.lhsmod = reinterpret_cast<uint64_t *>(b + kOffLhs);
    r.tails = reinterpret_cast<uint32_t *>(b + kOffTails);
    r.tail_hist = reinterpret_cast<unsigned long long *>(b + kOffHist);
    return r;
}

}  // namespace

static __device__ __align__(256) unsigned char scratch[WV_STATIC_SCRATCH_BYTES];

namespace wv {

// Device address of this device's copy of `scratch` (device current).
int static_scratch_setup(int device, void **addr) {
    *addr = nullptr;
    if (device < 0 || device >= kMaxDevices) return WV_EINVAL;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[device]) {
        void *p = nullptr;
        WV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return WV_EHIP;
        g_addr[device] = p;
    }
    *addr = g_addr[device];
    return WV_OK;
}

}  // namespace wv

extern "C" int wv_eval_primes_static(wv_ctx *c, const uint64_t *d_primes, size_t n, wv_result *d_out,
                                     void *hip_stream) {
    if (!c) return WV_EINVAL;
    if (n == 0) return WV_OK;
    if (!d_primes || !d_out || n > WV_STATIC_MAX_PRIMES) return WV_EINVAL;
    if (!c->scratch) return WV_EHIP;   // looked up by wv_create
    WV_TRY(check_device(c));
    BatchShape sh;
    WV_TRY(batch_shape(c, (uint32_t)n, WV_P_MAX, &sh));   // host arithmetic only; the primes are not read
    if (sh.nseg > WV_STATIC_MAX_SLOTS) return WV_EINVAL;
    // the plan picks the chunk size so that full chunks plus tails fit the
    // fixed partial-pair area (cap >= 2 nseg, see k_pick_chunk)
    sh.cap = WV_STATIC_MAX_CHUNKS;
    const BatchBufs b = carve(c->scratch);
    hipStream_t st = (hipStream_t)hip_stream;
    WV_TRY(enqueue_plan(c, b, d_primes, sh, st));
    WV_TRY(enqueue_sum(c, b, sh, st, 0, UINT64_MAX));
    WV_TRY(enqueue_finish(c, b, sh, st, d_out));
    return WV_OK;
}
