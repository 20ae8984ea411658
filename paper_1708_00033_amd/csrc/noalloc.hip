// Two-electron build that allocates nothing, for callers that cannot call
// hipMalloc: code under HIP graph capture, tight serving loops, harnesses
// that forbid allocation.
//
// The build's per-build scratch (accumulator W, component-scaled density D',
// max|D|, quartet counters, launch queue counters) comes from one file-scope
// device array per GPU instead of context memory.  Host code never uses the
// array's name as an address: hfx_noalloc_init (called by hfx_create with the
// context's device current) reads the array's device address on that device
// once with hipGetSymbolAddress and keeps it per device; every kernel
// argument derives from that address.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "hfx_ctx.h"

#define HFX_NOALLOC_BYTES (32ull << 20)

static __device__ __align__(256) unsigned char scratch[HFX_NOALLOC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices] = {nullptr};   // device address of `scratch` per device

// Layout of the array (byte offsets).
constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kCountersOff = 0;      // HFX_CNT_WORDS quartet-counter words, then the non-finite flag
constexpr size_t kDmaxOff = align256((HFX_CNT_WORDS + 1) * sizeof(unsigned long long));   // 1 x u64
constexpr size_t kWorkOff = kDmaxOff + 256;   // 16 x u64 per launch plan
constexpr size_t kMaxPlans = 512;
constexpr size_t kMatOff = kWorkOff + kMaxPlans * 16 * sizeof(unsigned long long);   // D', then W

}  // namespace

hipError_t hfx_noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = static_cast<unsigned char*>(p);
    return hipSuccess;
}

extern "C" hfx_status hfx_build_2e_noalloc_dev(hfx_ctx* c, const double* dD, double cj, double ck, double* dG,
                                               void* stream, hfx_fock_stats* stats) {
    if (!c) return HFX_ERR_INVALID_ARG;
    if (!dD || !dG) return hfx_fail(c, HFX_ERR_INVALID_ARG, "null pointer");
    if (!std::isfinite(cj) || !std::isfinite(ck)) return hfx_fail(c, HFX_ERR_INVALID_ARG, "non-finite cj/ck");
    if (!c->loaded) return hfx_fail(c, HFX_ERR_STATE, "hfx_build_2e_noalloc_dev: nothing loaded");
    const int dev = c->opt.device;
    if (dev < 0 || dev >= kMaxDevices) return hfx_fail(c, HFX_ERR_DEVICE, "device ordinal out of range");
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        base = g_scratch[dev];
    }
    if (!base) return hfx_fail(c, HFX_ERR_STATE, "no-alloc scratch not initialised on this device");
    const size_t mat = align256(c->nelem * sizeof(double));
    if (c->plans.size() > kMaxPlans || kMatOff + 2 * mat > HFX_NOALLOC_BYTES)
        return hfx_fail(c, HFX_ERR_INVALID_ARG,
                        "hfx_build_2e_noalloc_dev: system too large for the fixed scratch (" +
                            std::to_string(c->plans.size()) + " launch plans, max " + std::to_string(kMaxPlans) +
                            "; " + std::to_string(kMatOff + 2 * mat) + " bytes, max " +
                            std::to_string(HFX_NOALLOC_BYTES) + ")");
    const hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) return hfx_hip_check(c, e, "hipSetDevice");
    BuildBufs b;
    b.counters = reinterpret_cast<unsigned long long*>(base + kCountersOff);
    b.bad = reinterpret_cast<int*>(b.counters + HFX_CNT_WORDS);
    b.dmax = reinterpret_cast<unsigned long long*>(base + kDmaxOff);
    b.work = reinterpret_cast<unsigned long long*>(base + kWorkOff);
    b.Dp = reinterpret_cast<double*>(base + kMatOff);
    b.W = reinterpret_cast<double*>(base + kMatOff + mat);
    // every word the build accumulates into (W, counters, flag, max|D|, queue
    // counters) is cleared by fill kernels inside the build
    return hfx_build_with(c, b, dD, cj, ck, nullptr, dG, (hipStream_t)stream, stats, 0, 1);
}
