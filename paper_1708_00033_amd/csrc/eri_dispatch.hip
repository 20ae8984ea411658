// Launch helpers for the per-class kernels (one translation unit per class).
#include "hfx_internal.h"
#include "generated/eri_classes.h"

#define HFX_DECL(cid)                                        \
    extern "C" const void* hfx_class_kernel_##cid(int);      \
    extern "C" const void* hfx_class_kernel_kr_##cid(int);   \
    extern "C" const void* hfx_class_kernel_multi_##cid(int); \
    extern "C" const void* hfx_schwarz_kernel_##cid(void);
HFX_FOR_EACH_CID(HFX_DECL)

#define HFX_KPTR(cid) hfx_class_kernel_##cid,
#define HFX_RPTR(cid) hfx_class_kernel_kr_##cid,
#define HFX_SPTR(cid) hfx_schwarz_kernel_##cid,
#define HFX_MPTR(cid) hfx_class_kernel_multi_##cid,
static const void* (*const kMultiLookup[21])(int) = {HFX_FOR_EACH_CID(HFX_MPTR)};
static const void* (*const kClassLookup[21])(int) = {HFX_FOR_EACH_CID(HFX_KPTR)};
static const void* (*const kClassLookupKr[21])(int) = {HFX_FOR_EACH_CID(HFX_RPTR)};
static const void* (*const kSchwarzLookup[21])(void) = {HFX_FOR_EACH_CID(HFX_SPTR)};

extern "C" int hfx_class_wgs(int cid, int alt);

// Register-tiled kernels: variant index of (digestion mode, ket primitive
// count, bras per block), or -1 when the class has none for that count.
static int kr_variant(int cid, int mode, int kp, int nbl) {
    const int kpi = kp == 1 ? 0 : (kp == 3 ? 1 : (kp == 9 ? 2 : -1));
    if (kpi < 0 || nbl < 1 || nbl > 2) return -1;
    const int v = mode + 2 * kpi + 6 * (nbl - 1);
    return kClassLookupKr[cid](v) ? v : -1;
}

extern "C" int hfx_class_has_kr(int cid, int kp) { return kr_variant(cid, 0, kp, 1) >= 0; }

extern "C" hipError_t hfx_launch_class_kr(int cid, int mode, int kp, int nbl, int nblocks, size_t lds_bytes,
                                          hipStream_t stream, const ClassArgs* args) {
    if (nblocks <= 0) return hipSuccess;
    const int v = kr_variant(cid, mode, kp, nbl);
    if (v < 0 || !args->work) return hipErrorInvalidValue;
    const void* fn = kClassLookupKr[cid](v);
    if (lds_bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    void* kargs[] = {(void*)args};
    return hipLaunchKernel(fn, dim3(nblocks), dim3(hfx_class_wgs(cid, 1)), kargs, lds_bytes, stream);
}

extern "C" int hfx_class_resident_blocks_kr(int cid, int mode, int kp, int nbl, size_t lds_bytes) {
    const int v = kr_variant(cid, mode, kp, nbl);
    if (v < 0) return 0;
    const void* fn = kClassLookupKr[cid](v);
    if (lds_bytes > 64 * 1024 &&
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) != hipSuccess)
        return 0;
    int per_cu = 0, dev = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, hfx_class_wgs(cid, 1), lds_bytes) != hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * ncu;
}

#define HFX_WG 256

// nblocks workgroups: the task count (static launch) or the resident grid
// (persistent launch, args->work set).
extern "C" int hfx_class_wgs(int cid, int alt) { return alt ? kEriClassInfo[cid].wgs_alt : kEriClassInfo[cid].wgs; }

// alt: the class's alternative workgroup size (kEriClassInfo.wgs_alt);
// wave: one task per wave (a persistent launch, args->work set); dstage:
// ClassArgs::dstage (0, 1 or 3), the kernel variant with staged D' rows.
static int class_variant(int alt, int persistent, int wave, int mode, int mixed, int dstage) {
    const int ds = dstage == 3 ? 2 : dstage == 1 ? 1 : 0;
    return ds * 32 + (wave ? 16 : 0) + (alt ? 8 : 0) + (persistent ? 4 : 0) + mode * 2 + mixed;
}

extern "C" hipError_t hfx_launch_class(int cid, int alt, int wave, int mode, int mixed, int nblocks,
                                       size_t lds_bytes, hipStream_t stream, const ClassArgs* args) {
    if (nblocks <= 0) return hipSuccess;
    if (wave && !args->work) return hipErrorInvalidValue;
    if (args->dstage != 0 && args->dstage != 1 && args->dstage != 3) return hipErrorInvalidValue;
    const void* fn = kClassLookup[cid](class_variant(alt, args->work != nullptr, wave, mode, mixed, args->dstage));
    if (!fn) return hipErrorInvalidValue;
    if (lds_bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    void* kargs[] = {(void*)args};
    return hipLaunchKernel(fn, dim3(nblocks), dim3(hfx_class_wgs(cid, alt)), kargs, lds_bytes, stream);
}

// Workgroups of one class kernel that fit on the device at once.
extern "C" int hfx_class_resident_blocks(int cid, int alt, int wave, int mode, int mixed, int dstage,
                                         size_t lds_bytes) {
    const void* fn = kClassLookup[cid](class_variant(alt, 1, wave, mode, mixed, dstage));
    if (!fn) return 0;
    if (lds_bytes > 64 * 1024 &&
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) != hipSuccess)
        return 0;
    int per_cu = 0, dev = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, hfx_class_wgs(cid, alt), lds_bytes) != hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * ncu;
}


// Multi-density kernel of class cid (persistent; args->work set), digestion
// mode 0 (LDS rows per density) or 1 (global atomics): nblocks workgroups.
extern "C" hipError_t hfx_launch_class_multi(int cid, int mode, int nblocks, size_t lds_bytes, hipStream_t stream,
                                             const ClassArgs* args) {
    if (nblocks <= 0) return hipSuccess;
    if (!args->work) return hipErrorInvalidValue;
    const void* fn = kMultiLookup[cid](mode);
    if (lds_bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    void* kargs[] = {(void*)args};
    return hipLaunchKernel(fn, dim3(nblocks), dim3(kEriClassInfo[cid].wgs), kargs, lds_bytes, stream);
}

// Largest per-lane private segment (scratch) in bytes and largest register
// count over every kernel variant of class cid (launch form, digestion,
// staged D' rows, precision, workgroup size), read from the code object's
// metadata without a launch.
extern "C" hipError_t hfx_class_kernel_resources(int cid, long long* scratch_bytes, int* regs) {
    long long sc = 0;
    int rg = 0;
    for (int v = 0; v < 128 + 12 + 2; ++v) {
        const void* fn = v < 128   ? kClassLookup[cid](v)
                         : v < 140 ? kClassLookupKr[cid](v - 128)
                                   : kMultiLookup[cid](v - 140);
        if (!fn) continue;
        hipFuncAttributes fa;
        const hipError_t e = hipFuncGetAttributes(&fa, fn);
        if (e != hipSuccess) return e;
        sc = fa.localSizeBytes > (size_t)sc ? (long long)fa.localSizeBytes : sc;
        rg = fa.numRegs > rg ? fa.numRegs : rg;
    }
    *scratch_bytes = sc;
    *regs = rg;
    return hipSuccess;
}

extern "C" hipError_t hfx_launch_schwarz(int cid, const PairInfo* pairs, int npairs, const PrimPair* prim,
                                         const double* boys, double* Q, hipStream_t stream) {
    if (npairs <= 0) return hipSuccess;
    const void* fn = kSchwarzLookup[cid]();
    void* kargs[] = {(void*)&pairs, (void*)&npairs, (void*)&prim, (void*)&boys, (void*)&Q};
    return hipLaunchKernel(fn, dim3((npairs + HFX_WG - 1) / HFX_WG), dim3(HFX_WG), kargs, 0, stream);
}
