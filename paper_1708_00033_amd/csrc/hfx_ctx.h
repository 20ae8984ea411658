// Host-side context of the library (shared by the API and SCF sources).
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <map>
#include <string>
#include <vector>

#include "hfx.h"
#include "hfx_internal.h"

struct ShellHost {
    double x, y, z;
    int l, nprim, prim_off, bf;
};

// Significant pairs of one pair class that share one primitive count, sorted
// by Schwarz bound (descending); ket primitives as a structure of arrays.
struct KetList {
    int K = 0, kp = 0, n = 0;
    PairInfo* d_pairs = nullptr;
    double* d_q = nullptr;
    double* d_soa = nullptr;
    float* d_soa32 = nullptr;   // its FP32 copy (the FP32 evaluation of mixed builds)
    double* d_wket = nullptr;   // ket-block J accumulator, ncart(l_c) ncart(l_d) x n
    double* d_dket = nullptr;   // D'_cd of every ket, gathered per build, same layout
    double* d_dket_multi = nullptr;   // the same for each density of a multi-density build
    double* d_wket_multi = nullptr;   // and the ket-block J accumulators
    int dket_multi_cap = 0;           // densities they hold
    int4* d_kbf = nullptr;      // per ket: (bfa, bfb, a, b)
    int* d_kpos = nullptr;      // per ket: position in its pair class's Q-sorted list
    int ncd = 1;
};

// One launch: class (B, K) against one ket list.
struct SubPlan {
    int cid = 0, B = 0, K = 0, list = 0;
    int nbra = 0;             // bras with at least one ket
    int ntask = 0;
    int* d_split = nullptr;   // per task: first ket evaluated in FP32 (mixed builds)
    int4* d_tasks = nullptr;
    long long quartets = 0, integrals = 0, prim = 0;
    size_t lds_bytes = 0;     // bra rows F_I, F_J (LDS digestion)
    size_t lds_dst = 0;       // the bra's staged D' rows (LDS digestion with D rows)
    int dstage = 0;           // ClassArgs::dstage: bit 0 shell a's D' rows staged, bit 1 shell b's
    size_t lds_tab = 0;       // the class's FP64 Boys rows in LDS
    int mode = 0;             // digestion actually used (LDS may fall back to global)
    // timing (when enabled): events around this launch, summed milliseconds
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool pending = false;
    double ms = 0.0;
    long long launches = 0;
    bool fp64_only = false;   // class built only in FP64 (mixed requests run FP64)
    // LDS of a workgroup: bra rows (one set per wave with one task per wave) and Boys rows
    size_t lds() const { return (mode == 0 ? (lds_bytes + lds_dst) * (wave ? wave : nbl) : 0) + lds_tab; }
    bool persist = false;     // persistent launch through per-XCD work counters
    int wave = 0;             // > 0: one task per wave (persistent), this many waves per workgroup
    bool kr = false;          // register-tiled persistent kernel (ket primitives in registers), FP64
    bool priv = false;        // private digestion: global atomics into the per-XCD copies of W
    int nbl = 1;              // bras per task (register-tiled blocks of Q-adjacent bras)
    int alt = 0;              // 1: the class's alternative workgroup size
    int nblocks[2] = {0, 0};  // resident grid (multiple of 8) for the FP64 / the mixed kernel
};

struct ClassTotals {
    long long quartets = 0, integrals = 0, prim = 0, ntask = 0;
};

// One molecule of a batch (a single system is a batch of one).  Its
// matrices are the ragged block at element offset moff, nbf x nbf row-major.
struct MolInfo {
    int natom = 0, aoff = 0, nshell = 0, soff = 0;
    int nbf = 0, boff = 0, nelec = 0, nocc = 0;
    long long moff = 0;
    double enuc = 0.0;
};

struct GuessPairsDev;   // learned-guess pair data (guess.hip)

struct hfx_ctx {
    hfx_options opt{};
    std::string err;
    bool loaded = false;
    // system
    int natom = 0, nshell = 0, nbf = 0, nelec = 0, nocc = 0;   // totals over the batch
    double enuc = 0.0;
    int nmol = 0, max_ld = 0;
    size_t nelem = 0;                   // sum of nbf_m^2 (ragged matrix storage)
    std::vector<MolInfo> mol;
    long long* d_moff = nullptr;
    int* d_mdim = nullptr;
    int* d_mboff = nullptr;
    // Per ket list, groups of kets sharing (molecule, column window of shell c,
    // column window of shell d), Q descending within a group: group starts
    // (ngroup + 1), each molecule's first group (nmol + 1), window code per
    // group (wc | wd << 16).  Without windows a group is a molecule.
    std::vector<std::vector<int>> kgroup, kmolg, kwcode;
    int win = 0;                          // column window (0: whole rows, no windows)
    int rs = 0;                           // LDS row length of the bra rows (doubles)
    std::vector<int> Z;
    std::vector<double> axyz;
    std::vector<ShellHost> shells;
    std::vector<double> exps, coefs;   // normalised coefficients
    std::vector<double> cscale;        // per basis function component factor
    std::vector<int> shell_exps_l;     // shell angular momenta (input order)
    std::vector<std::vector<double>> raw_exps, raw_coefs;  // input copies (for SAD)
    std::vector<int> shell_atom;
    // device data
    PrimPair* d_prim = nullptr;
    float* d_prim32 = nullptr;          // FP32 copy (HFX_PRIM_FIELDS floats per primitive pair)
    PairInfo* d_pairs[6] = {nullptr};   // significant pairs per pair class, Q descending (bras)
    int npair[6] = {0};
    std::vector<KetList> ketlists;      // per pair class and primitive count (kets)
    std::vector<SubPlan> plans;         // launches, grouped by class id
    ClassTotals totals[21];
    // host copies of the Q-sorted lists (for re-planning) and per-class tuning
    std::vector<std::vector<PairInfo>> host_bra, host_ket;
    std::vector<std::vector<double>> host_pos, host_kpos;
    int tune_tq[21] = {0};                       // 0: opt.task_quartets
    int tune_stripe[21] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1,
                           -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};  // -1: default (striped)
    int tune_persist[21] = {0};                  // 1: persistent launch
    int tune_fp32[21] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1,
                         1, 1, 1, 1, 1, 1, 1, 1, 1, 1};   // mixed builds: FP32 kernel for eligible quartets
    int tune_digest[21] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1,
                           -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};  // -1: opt.digest
    unsigned long long* d_work = nullptr;        // 8 queue counters per plan (16 apart)
    std::vector<double> Qshell;         // nshell x nshell Schwarz bounds (host)
    double* d_boys64 = nullptr;
    double* d_cscale = nullptr;
    double* d_S = nullptr;
    double* d_H = nullptr;
    double* d_W = nullptr;
    double* d_Wrep = nullptr;   // private digestion: 8 per-XCD copies of W (allocated by plans that use it)
    // multi-density builds: D' and the J and K accumulators of each density
    double* d_multi = nullptr;
    int multi_cap = 0;
    unsigned long long* d_multi_work = nullptr;   // queue counters: 8 per (plan, density group)
    size_t multi_work_cap = 0;
    double* d_Dp = nullptr;
    double* d_tmpD = nullptr;   // host-variant staging
    double* d_tmpF = nullptr;
    unsigned long long* d_dmax = nullptr;
    unsigned long long* d_counters = nullptr;  // HFX_CNT_WORDS quartet-counter words, then the non-finite flag
    int* d_bad = nullptr;
    rocblas_handle blas = nullptr;
    hipGraphExec_t graph_exec = nullptr;   // captured build (hfx_graph_capture)
    GuessPairsDev* guess = nullptr;        // hfx_guess_setup
    // SAD: atomic densities by element and basis (kept across loads)
    std::map<std::string, std::vector<double>> sad_cache;
    // timing
    bool timing = false;
    hipStream_t last_stream = nullptr;
    // class launches of a build spread over the caller's stream and
    // nstreams - 1 side streams (created with the context, default
    // priority), forked from and joined back into the caller's stream
    static constexpr int kMaxStreams = 4;
    int nstreams = 2;
    hipStream_t side[kMaxStreams - 1] = {};
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join[kMaxStreams - 1] = {};
};

// Per-build scratch of one Fock build: the accumulator W and the
// component-scaled density D' (ragged, nelem doubles each), the max|D| word,
// the quartet counters (HFX_CNT_WORDS) followed by the non-finite flag, and 16 queue counters
// per launch plan.  Context memory by default (hfx_ctx_bufs); the no-alloc
// entry point passes a static device array instead.
struct BuildBufs {
    double* W = nullptr;
    double* Dp = nullptr;
    unsigned long long* dmax = nullptr;
    unsigned long long* counters = nullptr;
    int* bad = nullptr;
    unsigned long long* work = nullptr;
};

// implemented in guess.hip
void hfx_guess_release(hfx_ctx* c);

// implemented in noalloc.hip
hipError_t hfx_noalloc_init(int device);

// implemented in hfx_api.cpp
hfx_status hfx_fail(hfx_ctx* c, hfx_status s, const std::string& msg);
hfx_status hfx_hip_check(hfx_ctx* c, hipError_t e, const char* what);
hfx_status hfx_build_internal(hfx_ctx* c, const double* dD, double cj, double ck, const double* dH, double* dOut,
                              hipStream_t st, hfx_fock_stats* stats, int shard, int nshards);
hfx_status hfx_build_with(hfx_ctx* c, const BuildBufs& b, const double* dD, double cj, double ck, const double* dH,
                          double* dOut, hipStream_t st, hfx_fock_stats* stats, int shard, int nshards);

// implemented in misc_kernels.hip
extern "C" {
hipError_t hfx_prepare_density(const double* D, const double* cs, int nmol, const long long* moff, const int* mdim,
                               const int* mboff, int max_ld, double* Dp, unsigned long long* dmax_bits, hipStream_t st);
hipError_t hfx_fill(double* p, size_t n, double v, hipStream_t st);
hipError_t hfx_reduce_replicas(const double* rep, int nrep, size_t n, double* W, hipStream_t st);
hipError_t hfx_fill_u64(unsigned long long* p, int n, hipStream_t st);
hipError_t hfx_split(const PairInfo* bra, const double* ketq, const int4* tasks, int ntask, double fp32_tau,
                     const unsigned long long* dmax_bits, int* split, hipStream_t st);
hipError_t hfx_gather_ket(const PairInfo* kets, int n, int nc, int nd, const double* D, const long long* moff,
                          double* dket, hipStream_t st);
hipError_t hfx_scatter_ket(const PairInfo* kets, int n, int nc, int nd, const double* wket, const long long* moff,
                           double* W, hipStream_t st);
hipError_t hfx_assemble(const double* H, const double* W, const double* cs, int nmol, const long long* moff,
                        const int* mdim, const int* mboff, int max_ld, double* F, int* bad, hipStream_t st);
hipError_t hfx_one_electron(const void* sh, int nshell, const double* exps, const double* coefs, const double* atoms,
                            int natom, const double* cs, const double* boys, int n, double* S, double* T, double* V,
                            hipStream_t st);
hipError_t hfx_antisym(const double* A, int n, double* out, hipStream_t st);
int hfx_dot_partial(const double* a, const double* b, size_t n, int mode, double* out, hipStream_t st);
int hfx_energy_partial(const double* D, const double* H, const double* F, size_t n, double* out, hipStream_t st);
hipError_t hfx_lincomb(const double* const* M, const double* c, int m, size_t n, double* out, hipStream_t st);
hipError_t hfx_scale_cols(const double* U, const double* w, const int* keep, int n, int nk, double* out,
                          hipStream_t st);
hipError_t hfx_weight_cols(const double* C, const double* occ, int n, int nk, double* out, hipStream_t st);
hipError_t hfx_pad_blocks(const double* src, const long long* moff, const int* dim, int nmol, int NP, double pad,
                          double* dst, hipStream_t st);
hipError_t hfx_pad_rest(const int* dim, int nmol, int NP, double pad, double* dst, hipStream_t st);
// eri_dispatch.hip
hipError_t hfx_launch_class(int cid, int alt, int wave, int mode, int mixed, int nblocks, size_t lds_bytes,
                            hipStream_t stream, const ClassArgs* args);
int hfx_class_resident_blocks(int cid, int alt, int wave, int mode, int mixed, int dstage, size_t lds_bytes);
int hfx_class_wgs(int cid, int alt);
hipError_t hfx_class_kernel_resources(int cid, long long* scratch_bytes, int* regs);
int hfx_class_has_kr(int cid, int kp);
hipError_t hfx_launch_class_kr(int cid, int mode, int kp, int nbl, int nblocks, size_t lds_bytes, hipStream_t stream,
                               const ClassArgs* args);
int hfx_class_resident_blocks_kr(int cid, int mode, int kp, int nbl, size_t lds_bytes);
hipError_t hfx_launch_class_multi(int cid, int mode, int nblocks, size_t lds_bytes, hipStream_t stream,
                                  const ClassArgs* args);
hipError_t hfx_launch_schwarz(int cid, const PairInfo* pairs, int npairs, const PrimPair* prim, const double* boys,
                              double* Q, hipStream_t stream);
}
