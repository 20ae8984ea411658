// Launch helpers for the per-class kernels (one translation unit per class).
#include "hfx_internal.h"
#include "generated/eri_classes.h"

#define HFX_DECL(cid)                                        \
    extern "C" const void* hfx_class_kernel_##cid(int);      \
    extern "C" const void* hfx_schwarz_kernel_##cid(void);
HFX_FOR_EACH_CID(HFX_DECL)

#define HFX_KPTR(cid) hfx_class_kernel_##cid,
#define HFX_SPTR(cid) hfx_schwarz_kernel_##cid,
static const void* (*const kClassLookup[21])(int) = {HFX_FOR_EACH_CID(HFX_KPTR)};
static const void* (*const kSchwarzLookup[21])(void) = {HFX_FOR_EACH_CID(HFX_SPTR)};

#define HFX_WG 256

// nblocks workgroups: the task count (static launch) or the resident grid
// (persistent launch, args->work set).
extern "C" int hfx_class_wgs(int cid, int alt) { return alt ? kEriClassInfo[cid].wgs_alt : kEriClassInfo[cid].wgs; }

// alt: the class's alternative workgroup size (kEriClassInfo.wgs_alt);
// wave: one task per wave (a persistent launch, args->work set).
static int class_variant(int alt, int persistent, int wave, int mode, int mixed) {
    return (wave ? 16 : 0) + (alt ? 8 : 0) + (persistent ? 4 : 0) + mode * 2 + mixed;
}

extern "C" hipError_t hfx_launch_class(int cid, int alt, int wave, int mode, int mixed, int nblocks,
                                       size_t lds_bytes, hipStream_t stream, const ClassArgs* args) {
    if (nblocks <= 0) return hipSuccess;
    if (wave && !args->work) return hipErrorInvalidValue;
    const void* fn = kClassLookup[cid](class_variant(alt, args->work != nullptr, wave, mode, mixed));
    if (lds_bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    void* kargs[] = {(void*)args};
    return hipLaunchKernel(fn, dim3(nblocks), dim3(hfx_class_wgs(cid, alt)), kargs, lds_bytes, stream);
}

// Workgroups of one class kernel that fit on the device at once.
extern "C" int hfx_class_resident_blocks(int cid, int alt, int wave, int mode, int mixed, size_t lds_bytes) {
    const void* fn = kClassLookup[cid](class_variant(alt, 1, wave, mode, mixed));
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


// Largest per-lane private segment (scratch) in bytes and largest register
// count over every kernel variant of class cid (launch form, digestion,
// precision, workgroup size), read from the code object's metadata without a
// launch.
extern "C" hipError_t hfx_class_kernel_resources(int cid, long long* scratch_bytes, int* regs) {
    long long sc = 0;
    int rg = 0;
    for (int v = 0; v < 32; ++v) {
        hipFuncAttributes fa;
        const hipError_t e = hipFuncGetAttributes(&fa, kClassLookup[cid](v));
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
