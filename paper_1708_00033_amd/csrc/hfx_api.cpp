// C ABI of the library: context, system loading (normalisation, shell pairs,
// Schwarz bounds, screened quartet plan, one-electron integrals) and the
// direct Fock build.  The SCF driver lives in scf.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "hfx_ctx.h"

// ---- errors ---------------------------------------------------------------------

hfx_status hfx_fail(hfx_ctx* c, hfx_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

hfx_status hfx_hip_check(hfx_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return HFX_OK;
    return hfx_fail(c, e == hipErrorOutOfMemory ? HFX_ERR_OOM : HFX_ERR_DEVICE,
                    std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCK(call)                                                      \
    do {                                                                 \
        hfx_status _s = hfx_hip_check(c, (call), #call);                 \
        if (_s != HFX_OK) return _s;                                     \
    } while (0)

template <typename T>
static hipError_t dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void**)p, count * sizeof(T));
}

template <typename T>
static void dfree(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }
static int pair_class(int la, int lb) { return la * (la + 1) / 2 + lb; }   // la >= lb
static int class_id(int B, int K) { return B * (B + 1) / 2 + K; }           // B >= K

static const int kPairL[6][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};

static hfx_status replan(hfx_ctx* c);

constexpr int kXcds = 8;   // XCDs of an MI355X: private digestion keeps one copy of W per XCD

// A captured build replays the launch arguments (plans, task buffers,
// precision split) of the moment it was captured: drop it whenever those
// change, so that hfx_graph_launch reports HFX_ERR_STATE instead of replaying
// freed buffers or a stale precision choice.
static void drop_graph(hfx_ctx* c) {
    if (c->graph_exec) {
        (void)hipGraphExecDestroy(c->graph_exec);
        c->graph_exec = nullptr;
    }
}

// ---- options -----------------------------------------------------------------------

extern "C" hfx_status hfx_default_options(hfx_options* o) {
    if (!o) return HFX_ERR_INVALID_ARG;
    o->device = 0;
    o->schwarz_tau = 1e-10;
    o->precision = HFX_PREC_FP64;
    o->fp32_tau = 1e-7;
    o->digest = HFX_DIGEST_LDS_D;
    o->task_quartets = 8192;
    o->log_level = 0;
    return HFX_OK;
}

extern "C" hfx_status hfx_default_scf_options(hfx_scf_options* o) {
    if (!o) return HFX_ERR_INVALID_ARG;
    o->max_iter = 100;
    o->e_tol = 1e-8;
    o->d_rms_tol = 1e-7;
    o->diis_max = 8;
    o->guess = HFX_GUESS_SAD;
    o->D0 = nullptr;
    o->lindep = 1e-7;
    o->model = nullptr;
    o->graph = 0;
    return HFX_OK;
}

static hfx_status check_options(hfx_ctx* c, const hfx_options* o) {
    if (!(o->schwarz_tau >= 0.0) || !std::isfinite(o->schwarz_tau))
        return hfx_fail(c, HFX_ERR_INVALID_ARG, "schwarz_tau must be finite and >= 0");
    if (o->precision != HFX_PREC_FP64 && o->precision != HFX_PREC_MIXED)
        return hfx_fail(c, HFX_ERR_INVALID_ARG, "precision must be HFX_PREC_FP64 or HFX_PREC_MIXED");
    if (!(o->fp32_tau >= 0.0) || !std::isfinite(o->fp32_tau))
        return hfx_fail(c, HFX_ERR_INVALID_ARG, "fp32_tau must be finite and >= 0");
    if (o->digest != HFX_DIGEST_LDS && o->digest != HFX_DIGEST_GLOBAL && o->digest != HFX_DIGEST_PRIVATE &&
        o->digest != HFX_DIGEST_LDS_D)
        return hfx_fail(c, HFX_ERR_INVALID_ARG,
                        "digest must be HFX_DIGEST_LDS, HFX_DIGEST_GLOBAL, HFX_DIGEST_PRIVATE or HFX_DIGEST_LDS_D");
    if (o->task_quartets < 256 || o->task_quartets % 256 != 0 || o->task_quartets > (1 << 24))
        return hfx_fail(c, HFX_ERR_INVALID_ARG, "task_quartets must be a multiple of 256 in [256, 2^24]");
    return HFX_OK;
}

// ---- lifetime ------------------------------------------------------------------------

static void release_system(hfx_ctx* c) {
    hfx_guess_release(c);
    dfree(c->d_work);
    drop_graph(c);
    dfree(c->d_prim);
    dfree(c->d_prim32);
    for (int k = 0; k < 6; ++k) {
        dfree(c->d_pairs[k]);
        c->npair[k] = 0;
    }
    for (auto& L : c->ketlists) {
        dfree(L.d_pairs);
        dfree(L.d_q);
        dfree(L.d_soa);
        dfree(L.d_soa32);
        dfree(L.d_wket);
        dfree(L.d_kbf);
        dfree(L.d_kpos);
        dfree(L.d_dket);
        dfree(L.d_dket_multi);
        dfree(L.d_wket_multi);
        L.dket_multi_cap = 0;
    }
    c->ketlists.clear();
    c->host_bra.clear();
    c->host_pos.clear();
    c->host_ket.clear();
    c->host_kpos.clear();
    for (auto& p : c->plans) {
        dfree(p.d_split);
        dfree(p.d_tasks);
        if (p.ev0) (void)hipEventDestroy(p.ev0);
        if (p.ev1) (void)hipEventDestroy(p.ev1);
    }
    c->plans.clear();
    for (auto& t : c->totals) t = ClassTotals();
    dfree(c->d_cscale);
    dfree(c->d_moff);
    dfree(c->d_mdim);
    dfree(c->d_mboff);
    c->kgroup.clear();
    c->kmolg.clear();
    c->kwcode.clear();
    dfree(c->d_S);
    dfree(c->d_H);
    dfree(c->d_W);
    dfree(c->d_Wrep);
    dfree(c->d_multi);
    c->multi_cap = 0;
    dfree(c->d_multi_work);
    c->multi_work_cap = 0;
    dfree(c->d_Dp);
    dfree(c->d_tmpD);
    dfree(c->d_tmpF);
    c->loaded = false;
}

// Per-lane scratch (private segment) that a class kernel may need.  The
// runtime reserves scratch for every wave slot the kernel can occupy; a
// (dd|dd) kernel variant with 25,200 bytes per lane made a queue fail with
// HSA_STATUS_ERROR_OUT_OF_RESOURCES, while every current variant needs under
// 8 KiB.  Checked once per process from the code objects' metadata.
constexpr long long kScratchBudget = 16384;

struct KernelResources {
    hipError_t err = hipSuccess;
    long long scratch[21] = {0};
    int regs[21] = {0};
};

static const KernelResources& kernel_resources() {
    static const KernelResources r = [] {
        KernelResources k;
        for (int cid = 0; cid < 21 && k.err == hipSuccess; ++cid)
            k.err = hfx_class_kernel_resources(cid, &k.scratch[cid], &k.regs[cid]);
        return k;
    }();
    return r;
}

extern "C" hfx_status hfx_kernel_resources(int device, long long* out) {
    if (!out) return HFX_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HFX_ERR_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return HFX_ERR_DEVICE;
    const KernelResources& r = kernel_resources();
    if (r.err != hipSuccess) return HFX_ERR_DEVICE;
    for (int k = 0; k < 21; ++k) {
        out[3 * k] = r.scratch[k];
        out[3 * k + 1] = r.regs[k];
        out[3 * k + 2] = kScratchBudget;
    }
    return HFX_OK;
}

extern "C" hfx_status hfx_create(const hfx_options* opt, hfx_ctx** out) {
    if (!out) return HFX_ERR_INVALID_ARG;
    hfx_ctx* c = new (std::nothrow) hfx_ctx();
    if (!c) return HFX_ERR_OOM;
    if (opt) c->opt = *opt; else hfx_default_options(&c->opt);
    hfx_status s = check_options(c, &c->opt);
    if (s != HFX_OK) { delete c; return s; }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0 || c->opt.device < 0 || c->opt.device >= ndev) {
        delete c;
        return HFX_ERR_DEVICE;
    }
    if (hipSetDevice(c->opt.device) != hipSuccess) { delete c; return HFX_ERR_DEVICE; }
    {
        const KernelResources& r = kernel_resources();
        bool ok = r.err == hipSuccess;
        for (int k = 0; k < 21 && ok; ++k) ok = r.scratch[k] <= kScratchBudget;
        if (!ok) { delete c; return HFX_ERR_DEVICE; }
    }
    std::vector<double> tab((size_t)BOYS_TAB_ENTRIES);
    hfx_boys_table(tab.data());
    if (dalloc(&c->d_boys64, tab.size()) != hipSuccess || dalloc(&c->d_dmax, 1) != hipSuccess ||
        dalloc(&c->d_counters, HFX_CNT_WORDS + 1) != hipSuccess) {
        hfx_destroy(c);
        return HFX_ERR_OOM;
    }
    if (hipMemcpy(c->d_boys64, tab.data(), tab.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
        hfx_destroy(c);
        return HFX_ERR_DEVICE;
    }
    if (hfx_noalloc_init(c->opt.device) != hipSuccess) {   // device address of the no-alloc scratch
        hfx_destroy(c);
        return HFX_ERR_DEVICE;
    }
    if (rocblas_create_handle(&c->blas) != rocblas_status_success) {
        hfx_destroy(c);
        return HFX_ERR_DEVICE;
    }
    bool ev_ok = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) == hipSuccess;
    for (int s = 0; s < hfx_ctx::kMaxStreams - 1 && ev_ok; ++s)
        ev_ok = hipStreamCreateWithFlags(&c->side[s], hipStreamNonBlocking) == hipSuccess &&
                hipEventCreateWithFlags(&c->ev_join[s], hipEventDisableTiming) == hipSuccess;
    if (!ev_ok) {
        hfx_destroy(c);
        return HFX_ERR_DEVICE;
    }
    c->d_bad = (int*)(c->d_counters + HFX_CNT_WORDS);
    *out = c;
    return HFX_OK;
}

extern "C" void hfx_destroy(hfx_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->opt.device);
    release_system(c);
    dfree(c->d_boys64);
    dfree(c->d_dmax);
    dfree(c->d_counters);
    c->d_bad = nullptr;
    if (c->blas) rocblas_destroy_handle(c->blas);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    for (int s = 0; s < hfx_ctx::kMaxStreams - 1; ++s) {
        if (c->side[s]) (void)hipStreamDestroy(c->side[s]);
        if (c->ev_join[s]) (void)hipEventDestroy(c->ev_join[s]);
    }
    delete c;
}

extern "C" const char* hfx_last_error(const hfx_ctx* c) { return c ? c->err.c_str() : "null context"; }

extern "C" hfx_status hfx_configure(hfx_ctx* c, const hfx_options* o) {
    if (!c || !o) return HFX_ERR_INVALID_ARG;
    hfx_status s = check_options(c, o);
    if (s != HFX_OK) return s;
    if (o->device != c->opt.device || o->schwarz_tau != c->opt.schwarz_tau)
        return hfx_fail(c, HFX_ERR_INVALID_ARG, "device and schwarz_tau cannot change after hfx_create");
    const bool new_plan = o->task_quartets != c->opt.task_quartets || o->digest != c->opt.digest;
    if (new_plan || o->precision != c->opt.precision || o->fp32_tau != c->opt.fp32_tau) drop_graph(c);
    c->opt = *o;
    if (new_plan && c->loaded) {
        HIPCK(hipSetDevice(c->opt.device));
        return replan(c);
    }
    return HFX_OK;
}

// ---- loading ----------------------------------------------------------------------------

static double dfact_odd(int n) {   // (2n-1)!!
    double r = 1.0;
    for (int k = 2 * n - 1; k > 1; k -= 2) r *= k;
    return r;
}

// Plan one launch (class (B, K) against ket list li): per-bra screened ket
// counts, workgroup tasks, counts.  Bras are the whole Q-sorted list of pair
// class B; for B == K an unordered pair {bra, ket} is taken once, with the
// ket not after the bra in that order (Q descending, then pair index).
static hfx_status plan_sub(hfx_ctx* c, int B, int li, const std::vector<PairInfo>& bras,
                           const std::vector<double>& bra_pos, const std::vector<PairInfo>& kets,
                           const std::vector<double>& ket_pos) {
    const KetList& KL = c->ketlists[li];
    const int K = KL.K;
    SubPlan P;
    P.cid = class_id(B, K);
    P.B = B;
    P.K = K;
    P.list = li;
    const double tau = c->opt.schwarz_tau;
    const int TQ = c->tune_tq[P.cid] > 0 ? c->tune_tq[P.cid] : c->opt.task_quartets;
    const bool stripe = c->tune_stripe[P.cid] >= 0 ? c->tune_stripe[P.cid] != 0 : true;
    // bra r (molecule m) meets the kets of its own molecule's groups; in
    // each group the kets with Q_s Q_r >= tau are a prefix (Q descending),
    // and for B == K so are the kets not after the bra in the class order
    const std::vector<int>& gs = c->kgroup[li];
    const std::vector<int>& mg = c->kmolg[li];
    const std::vector<int>& wcode = c->kwcode[li];
    const int nbra = (int)bras.size();
    struct Run { int r, g, n; };
    std::vector<Run> runs;
    for (int r = 0; r < nbra; ++r) {
        const double qr = bras[r].Q;
        for (int g = mg[bras[r].mol]; g < mg[bras[r].mol + 1]; ++g) {
            const int kb = gs[g], ke = gs[g + 1];
            int lo = kb, hi = ke;
            while (lo < hi) {
                const int mid = (lo + hi) / 2;
                if (kets[mid].Q * qr >= tau) lo = mid + 1; else hi = mid;
            }
            int n = lo - kb;
            if (B == K) {
                int l2 = kb, h2 = ke;
                while (l2 < h2) {
                    const int mid = (l2 + h2) / 2;
                    if (ket_pos[mid] <= bra_pos[r]) l2 = mid + 1; else h2 = mid;
                }
                n = std::min(n, l2 - kb);
            }
            if (n <= 0) continue;
            runs.push_back(Run{r, g, n});
            P.quartets += (long long)n;
            P.prim += (long long)bras[r].nprim * (long long)KL.kp * (long long)n;
        }
    }
    const int nint = ncart(kPairL[B][0]) * ncart(kPairL[B][1]) * ncart(kPairL[K][0]) * ncart(kPairL[K][1]);
    P.integrals = P.quartets * nint;
    // Tasks, striped over the 8 XCDs (workgroup i runs on XCD i mod 8, each
    // with its own L2): a long ket prefix is cut into chunks and chunk j of
    // every bra goes to the XCD queue j mod 8, so an XCD streams only its
    // share of each ket list; short prefixes fill the least loaded queue.
    // Queues are interleaved (task 8k + j = queue j's k-th entry) and padded
    // with empty tasks (r = -1).
    P.lds_bytes = (size_t)(ncart(kPairL[B][0]) + ncart(kPairL[B][1])) * c->rs * sizeof(double);
    P.fp64_only = nint >= 600;   // see ClassKernels in eri_impl.h
    P.lds_tab = (size_t)boys_lds_bytes();   // FP64 rows (the mixed kernels' FP32 part reads them too)
    const int digest = c->tune_digest[P.cid] >= 0 ? c->tune_digest[P.cid] : c->opt.digest;
    // 160 KiB of LDS per workgroup, less room for the persistent kernel's static counter
    constexpr size_t kLdsBudget = 160 * 1024 - 256;
    const bool lds_digest = digest == HFX_DIGEST_LDS || digest == HFX_DIGEST_LDS_D;
    P.mode = (lds_digest && P.lds_bytes + P.lds_tab <= kLdsBudget) ? 0 : 1;
    P.priv = digest == HFX_DIGEST_PRIVATE;   // global-atomic kernels into the per-XCD copies
    // D' rows staged too: both shells' rows when they fit, else shell a's
    // (the larger set); only for classes with small integral blocks and
    // whole rows (with column windows a task covers one pair of windows, and
    // copying its rows cost more than the gathers it saved on 512 waters)
    P.dstage = 0;
    P.lds_dst = 0;
    if (digest == HFX_DIGEST_LDS_D && P.mode == 0 && nint <= HFX_STAGE_D_MAX_NI && c->win == 0) {
        const size_t rows_a = (size_t)ncart(kPairL[B][0]) * c->rs * sizeof(double);
        if (2 * P.lds_bytes + P.lds_tab <= kLdsBudget) {
            P.dstage = 3;
            P.lds_dst = P.lds_bytes;
        } else if (P.lds_bytes + rows_a + P.lds_tab <= kLdsBudget) {
            P.dstage = 1;
            P.lds_dst = rows_a;
        }
    }
    // workgroup size: the class's alternative (smaller) size when two such
    // workgroups fit in LDS, else its default (a large group keeps the waves
    // per CU up when LDS admits one workgroup per CU)
    P.alt = hfx_class_wgs(P.cid, 1) != hfx_class_wgs(P.cid, 0) && 2 * P.lds() <= 160 * 1024 - 512;
    // register-tiled persistent form (launch form 3): blocks of two
    // Q-adjacent bras of one molecule when their rows fit in LDS, else one
    const int form = c->tune_persist[P.cid];
    if ((form == 3 || form == 4) && hfx_class_has_kr(P.cid, KL.kp) && nbra < (1 << 28)) {
        P.kr = true;
        P.alt = 1;   // the register-tiled kernels use the class's alternative workgroup size
        P.dstage = 0;   // their digestion reads D' from global memory
        P.lds_dst = 0;
        P.nbl = form == 3 ? 2 : 1;
        if (P.mode == 0 && P.lds() > 160 * 1024 - 256) P.nbl = 1;
    }
    // one task per block of bras: the block's ket range in a group is the
    // longest of its bras' screened prefixes; the kernel keeps, per bra, only
    // the kets of its own prefix (the same test as above, per lane)
    struct BRun { int r0, nb, g, n; };
    std::vector<BRun> bruns;
    if (P.nbl > 1) {
        std::vector<int> first(nbra), size(nbra);
        for (int r = 0; r < nbra;) {
            int e = r;
            while (e < nbra && bras[e].mol == bras[r].mol) ++e;
            for (int b = r; b < e; b += P.nbl)
                for (int k = b; k < std::min(e, b + P.nbl); ++k) {
                    first[k] = b;
                    size[k] = std::min(P.nbl, e - b);
                }
            r = e;
        }
        std::map<int, int> cur;   // group -> longest prefix of the current block
        int cur_first = -1, cur_nb = 0;
        auto flush = [&]() {
            for (const auto& x : cur) bruns.push_back(BRun{cur_first, cur_nb, x.first, x.second});
            cur.clear();
        };
        for (const Run& ru : runs) {
            if (first[ru.r] != cur_first) {
                flush();
                cur_first = first[ru.r];
                cur_nb = size[ru.r];
            }
            int& x = cur[ru.g];
            x = std::max(x, ru.n);
        }
        flush();
    } else {
        bruns.reserve(runs.size());
        for (const Run& ru : runs) bruns.push_back(BRun{ru.r, 1, ru.g, ru.n});
    }
    const int NX = 8, WGS = hfx_class_wgs(P.cid, P.alt);
    std::vector<std::vector<int4>> queue(NX);
    std::vector<long long> load(NX, 0);
    for (const BRun& ru : bruns) {
        const int r = ru.r0 | ((ru.nb - 1) << 28), n = ru.n, kb = gs[ru.g], w = wcode[ru.g];
        if (stripe && n >= 2 * NX * WGS) {
            int nch = (n + TQ - 1) / TQ;
            nch = ((nch + NX - 1) / NX) * NX;
            int len = (n + nch - 1) / nch;
            len = ((len + WGS - 1) / WGS) * WGS;
            for (int j = 0, s0 = 0; s0 < n; ++j, s0 += len) {
                queue[j % NX].push_back(make_int4(r, kb + s0, kb + std::min(n, s0 + len), w));
                load[j % NX] += std::min(len, n - s0);
            }
        } else {
            for (int s0 = 0; s0 < n; s0 += TQ) {
                const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                queue[q].push_back(make_int4(r, kb + s0, kb + std::min(n, s0 + TQ), w));
                load[q] += std::min(TQ, n - s0);
            }
        }
    }
    size_t qmax = 0;
    for (auto& q : queue) qmax = std::max(qmax, q.size());
    std::vector<int4> tasks;
    tasks.reserve(qmax * NX);
    for (size_t k = 0; k < qmax; ++k)
        for (int j = 0; j < NX; ++j) tasks.push_back(k < queue[j].size() ? queue[j][k] : make_int4(-1, 0, 0, 0));
    if (tasks.size() > (size_t)0x7fffffff) return hfx_fail(c, HFX_ERR_INVALID_ARG, "too many tasks for one launch");
    P.nbra = nbra;
    P.ntask = (int)tasks.size();
    if (P.ntask == 0) return HFX_OK;
    P.persist = c->tune_persist[P.cid] > 0;
    // one task per wave: each wave of the workgroup needs its own bra rows
    P.wave = 0;
    if (c->tune_persist[P.cid] == 2) {
        P.wave = WGS / 64;
        if (P.lds() > 160 * 1024 - 256) P.wave = 0;   // does not fit: one task per workgroup
    }
    if (P.kr) {
        int nb = hfx_class_resident_blocks_kr(P.cid, P.mode, KL.kp, P.nbl, P.lds());
        if (nb <= 0) return hfx_fail(c, HFX_ERR_DEVICE, "occupancy query of a register-tiled class kernel failed");
        nb = std::min(nb, P.ntask);
        P.nblocks[0] = P.nblocks[1] = ((nb + 7) / 8) * 8;
    }
    for (int mx = 0; mx < (P.kr ? 0 : (P.fp64_only ? 1 : 2)); ++mx) {
        int nb = hfx_class_resident_blocks(P.cid, P.alt, P.wave > 0, P.mode, mx, P.dstage, P.lds());
        if (nb <= 0) return hfx_fail(c, HFX_ERR_DEVICE, "occupancy query of a class kernel failed");
        nb = std::min(nb, P.ntask);
        P.nblocks[mx] = ((nb + 7) / 8) * 8;   // whole rounds over the 8 XCDs
    }
    HIPCK(dalloc(&P.d_split, tasks.size()));
    HIPCK(dalloc(&P.d_tasks, tasks.size()));
    HIPCK(hipMemcpy(P.d_tasks, tasks.data(), tasks.size() * sizeof(int4), hipMemcpyHostToDevice));
    ClassTotals& T = c->totals[P.cid];
    T.quartets += P.quartets;
    T.integrals += P.integrals;
    T.prim += P.prim;
    T.ntask += P.ntask;
    c->plans.push_back(P);
    return HFX_OK;
}

// (Re)build every launch plan from the stored Q-sorted lists with the
// current per-class tuning.
static hfx_status replan(hfx_ctx* c) {
    drop_graph(c);
    dfree(c->d_work);
    for (auto& p : c->plans) {
        dfree(p.d_split);
        dfree(p.d_tasks);
        if (p.ev0) (void)hipEventDestroy(p.ev0);
        if (p.ev1) (void)hipEventDestroy(p.ev1);
    }
    c->plans.clear();
    for (auto& t : c->totals) t = ClassTotals();
    for (int B = 0; B < 6; ++B)
        for (size_t li = 0; li < c->ketlists.size(); ++li) {
            if (c->ketlists[li].K > B) continue;
            hfx_status s = plan_sub(c, B, (int)li, c->host_bra[B], c->host_pos[B], c->host_ket[li], c->host_kpos[li]);
            if (s != HFX_OK) return s;
        }
    // launch order: largest classes first (sub-launches of a class stay together)
    static const int order[21] = {0, 1, 2, 6, 7, 3, 8, 9, 4, 10, 11, 13, 12, 5, 15, 16, 14, 18, 17, 19, 20};
    int rank[21];
    for (int i = 0; i < 21; ++i) rank[order[i]] = i;
    std::stable_sort(c->plans.begin(), c->plans.end(),
                     [&](const SubPlan& x, const SubPlan& y) { return rank[x.cid] < rank[y.cid]; });
    HIPCK(dalloc(&c->d_work, 16 * std::max<size_t>(c->plans.size(), 1)));   // 8 queue counters per plan, 16 apart
    bool any_priv = false;
    for (const auto& p : c->plans) any_priv |= p.priv;
    if (any_priv && !c->d_Wrep) HIPCK(dalloc(&c->d_Wrep, kXcds * c->nelem));
    if (!any_priv) dfree(c->d_Wrep);
    if (c->timing)
        for (auto& p : c->plans) {
            HIPCK(hipEventCreate(&p.ev0));
            HIPCK(hipEventCreate(&p.ev1));
        }
    return HFX_OK;
}

extern "C" hfx_status hfx_set_class_tuning(hfx_ctx* c, int cid, int task_quartets, int xcd_stripe,
                                           int persistent, int digest) {
    if (!c) return HFX_ERR_INVALID_ARG;
    if (cid < -1 || cid >= 21) return hfx_fail(c, HFX_ERR_INVALID_ARG, "class index out of range");
    if (task_quartets != 0 && (task_quartets < 256 || task_quartets % 256 != 0 || task_quartets > (1 << 24)))
        return hfx_fail(c, HFX_ERR_INVALID_ARG, "task_quartets must be 0 or a multiple of 256 in [256, 2^24]");
    if (xcd_stripe < -1 || xcd_stripe > 1) return hfx_fail(c, HFX_ERR_INVALID_ARG, "xcd_stripe must be -1, 0 or 1");
    if (persistent < 0 || persistent > 4)
        return hfx_fail(c, HFX_ERR_INVALID_ARG, "persistent must be 0, 1, 2, 3 or 4");
    if (digest < -1 || digest > 3) return hfx_fail(c, HFX_ERR_INVALID_ARG, "digest must be -1, 0, 1, 2 or 3");
    for (int k = 0; k < 21; ++k)
        if (cid == -1 || cid == k) {
            c->tune_tq[k] = task_quartets;
            c->tune_stripe[k] = xcd_stripe;
            c->tune_persist[k] = persistent;
            c->tune_digest[k] = digest;
        }
    if (!c->loaded) return HFX_OK;
    HIPCK(hipSetDevice(c->opt.device));
    return replan(c);
}

extern "C" hfx_status hfx_set_class_precision(hfx_ctx* c, int cid, int fp32) {
    if (!c) return HFX_ERR_INVALID_ARG;
    if (cid < -1 || cid >= 21) return hfx_fail(c, HFX_ERR_INVALID_ARG, "class index out of range");
    if (fp32 < 0 || fp32 > 1) return hfx_fail(c, HFX_ERR_INVALID_ARG, "fp32 must be 0 or 1");
    for (int k = 0; k < 21; ++k)
        if (cid == -1 || cid == k) {
            if (c->tune_fp32[k] != fp32) drop_graph(c);
            c->tune_fp32[k] = fp32;
        }
    return HFX_OK;
}

static hfx_status load_batch(hfx_ctx* c, int nmol, const int* natom_m, const int* Z, const double* xyz,
                             const int* nshell_m, const hfx_shell* sh, const int* charge_m);

// SP (L) shells are written out as an s shell and a p shell sharing the
// exponents (s coefficients, then p coefficients), then loaded as usual.
extern "C" hfx_status hfx_load_batch(hfx_ctx* c, int nmol, const int* natom_m, const int* Z, const double* xyz,
                                     const int* nshell_m, const hfx_shell* sh, const int* charge_m) {
    if (!c) return HFX_ERR_INVALID_ARG;
    if (nmol <= 0 || !natom_m || !Z || !xyz || !nshell_m || !sh)
        return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_load: empty system or null pointer");
    long long ntot = 0;
    for (int m = 0; m < nmol; ++m) {
        if (nshell_m[m] <= 0) return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_load: every molecule needs atoms and shells");
        ntot += nshell_m[m];
    }
    bool any_sp = false;
    for (long long s = 0; s < ntot; ++s) any_sp |= sh[s].l == HFX_SHELL_SP;
    if (!any_sp) return load_batch(c, nmol, natom_m, Z, xyz, nshell_m, sh, charge_m);
    std::vector<hfx_shell> ex;
    std::vector<int> nsh(nmol, 0);
    for (int m = 0, s = 0; m < nmol; ++m)
        for (int k = 0; k < nshell_m[m]; ++k, ++s) {
            hfx_shell q = sh[s];
            if (q.l == HFX_SHELL_SP) {
                if (!q.coefs_p) return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_load: SP shell without p coefficients");
                q.l = 0;
                ex.push_back(q);
                q.l = 1;
                q.coefs = q.coefs_p;
                ex.push_back(q);
                nsh[m] += 2;
            } else {
                ex.push_back(q);
                nsh[m] += 1;
            }
        }
    return load_batch(c, nmol, natom_m, Z, xyz, nsh.data(), ex.data(), charge_m);
}

static hfx_status load_batch(hfx_ctx* c, int nmol, const int* natom_m, const int* Z, const double* xyz,
                             const int* nshell_m, const hfx_shell* sh, const int* charge_m) {
    // ---- validation ----
    long long natom = 0, nshell = 0;
    for (int m = 0; m < nmol; ++m) {
        if (natom_m[m] <= 0 || nshell_m[m] <= 0)
            return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_load: every molecule needs atoms and shells");
        long long nel = -(charge_m ? charge_m[m] : 0);
        for (int a = 0; a < natom_m[m]; ++a) {
            const long long ga = natom + a;
            if (Z[ga] < 0 || Z[ga] > 118) return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_load: nuclear charge out of range");
            for (int x = 0; x < 3; ++x)
                if (!std::isfinite(xyz[3 * ga + x]))
                    return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_load: non-finite coordinate");
            nel += Z[ga];
        }
        if (nel < 0 || nel % 2)
            return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_load: closed shell needs an even electron count");
        for (int s = 0; s < nshell_m[m]; ++s) {
            const hfx_shell& q = sh[nshell + s];
            if (q.atom < 0 || q.atom >= natom_m[m]) return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_load: shell atom index");
            if (q.l < 0 || q.l > 2)
                return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_load: only s, p, d and SP shells (l in -1..2)");
            if (q.nprim < 1 || q.nprim > 16 || !q.exps || !q.coefs)
                return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_load: nprim must be in [1, 16]");
            for (int k = 0; k < q.nprim; ++k)
                if (!(q.exps[k] > 0.0) || !std::isfinite(q.exps[k]) || !std::isfinite(q.coefs[k]))
                    return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_load: exponents must be finite and > 0");
        }
        natom += natom_m[m];
        nshell += nshell_m[m];
    }
    if (nshell > 0x7fffffff / 2) return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_load: too many shells");
    HIPCK(hipSetDevice(c->opt.device));
    release_system(c);

    c->nmol = nmol;
    c->natom = (int)natom;
    c->nshell = (int)nshell;
    c->Z.assign(Z, Z + natom);
    c->axyz.assign(xyz, xyz + 3 * natom);
    c->shells.clear();
    c->exps.clear();
    c->coefs.clear();
    c->cscale.clear();
    c->raw_exps.clear();
    c->raw_coefs.clear();
    c->shell_atom.clear();
    c->shell_exps_l.clear();
    c->mol.assign(nmol, MolInfo());
    int nbf_tot = 0, nocc_tot = 0, nelec_tot = 0;
    long long nelem = 0;
    for (int m = 0, a0 = 0, s0 = 0; m < nmol; a0 += natom_m[m], s0 += nshell_m[m], ++m) {
        MolInfo& M = c->mol[m];
        M.natom = natom_m[m];
        M.aoff = a0;
        M.nshell = nshell_m[m];
        M.soff = s0;
        int nbf = 0;
        for (int s = s0; s < s0 + nshell_m[m]; ++s) {
            const int l = sh[s].l, np = sh[s].nprim;
            const int ga = a0 + sh[s].atom;
            ShellHost h;
            h.x = xyz[3 * ga];
            h.y = xyz[3 * ga + 1];
            h.z = xyz[3 * ga + 2];
            h.l = l;
            h.nprim = np;
            h.prim_off = (int)c->exps.size();
            h.bf = nbf;   // local to the molecule
            // unit-normalised primitives: (2a/pi)^{3/4} (4a)^{l/2} for the x^l
            // component; contraction renormalised to unit self-overlap.
            std::vector<double> nc(np);
            for (int k = 0; k < np; ++k)
                nc[k] = sh[s].coefs[k] * std::pow(2.0 * sh[s].exps[k] / M_PI, 0.75) * std::pow(4.0 * sh[s].exps[k], 0.5 * l);
            double self = 0.0;
            for (int i = 0; i < np; ++i)
                for (int j = 0; j < np; ++j) {
                    const double p = sh[s].exps[i] + sh[s].exps[j];
                    self += nc[i] * nc[j] * std::pow(M_PI / p, 1.5) / std::pow(2.0 * p, l);
                }
            const double rn = 1.0 / std::sqrt(self);
            for (int k = 0; k < np; ++k) {
                c->exps.push_back(sh[s].exps[k]);
                c->coefs.push_back(nc[k] * rn);
            }
            for (int x = l; x >= 0; --x)
                for (int y = l - x; y >= 0; --y) {
                    const int z = l - x - y;
                    c->cscale.push_back(1.0 / std::sqrt(dfact_odd(x) * dfact_odd(y) * dfact_odd(z)));
                }
            nbf += ncart(l);
            c->shells.push_back(h);
            c->raw_exps.emplace_back(sh[s].exps, sh[s].exps + np);
            c->raw_coefs.emplace_back(sh[s].coefs, sh[s].coefs + np);
            c->shell_atom.push_back(ga);
            c->shell_exps_l.push_back(l);
        }
        int nel = -(charge_m ? charge_m[m] : 0);
        double e = 0.0;
        for (int a = a0; a < a0 + natom_m[m]; ++a) {
            nel += Z[a];
            for (int b = a0; b < a; ++b) {
                const double dx = xyz[3 * a] - xyz[3 * b], dy = xyz[3 * a + 1] - xyz[3 * b + 1],
                             dz = xyz[3 * a + 2] - xyz[3 * b + 2];
                const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
                if (r == 0.0 && Z[a] * Z[b] != 0) return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_load: coincident nuclei");
                if (r > 0.0) e += (double)Z[a] * Z[b] / r;
            }
        }
        M.nbf = nbf;
        M.boff = nbf_tot;
        M.moff = nelem;
        M.nelec = nel;
        M.nocc = nel / 2;
        M.enuc = e;
        nbf_tot += nbf;
        nocc_tot += M.nocc;
        nelec_tot += nel;
        nelem += (long long)nbf * nbf;
    }
    c->nbf = nbf_tot;
    c->nocc = nocc_tot;
    c->nelec = nelec_tot;
    c->nelem = (size_t)nelem;
    c->enuc = 0.0;
    c->max_ld = 0;
    for (auto& M : c->mol) {
        c->enuc += M.enuc;
        c->max_ld = std::max(c->max_ld, M.nbf);
    }
    {
        std::vector<long long> moff(nmol);
        std::vector<int> mdim(nmol), mboff(nmol);
        for (int m = 0; m < nmol; ++m) {
            moff[m] = c->mol[m].moff;
            mdim[m] = c->mol[m].nbf;
            mboff[m] = c->mol[m].boff;
        }
        HIPCK(dalloc(&c->d_moff, nmol));
        HIPCK(dalloc(&c->d_mdim, nmol));
        HIPCK(dalloc(&c->d_mboff, nmol));
        HIPCK(hipMemcpy(c->d_moff, moff.data(), nmol * sizeof(long long), hipMemcpyHostToDevice));
        HIPCK(hipMemcpy(c->d_mdim, mdim.data(), nmol * sizeof(int), hipMemcpyHostToDevice));
        HIPCK(hipMemcpy(c->d_mboff, mboff.data(), nmol * sizeof(int), hipMemcpyHostToDevice));
    }
    HIPCK(dalloc(&c->d_cscale, nbf_tot));
    HIPCK(hipMemcpy(c->d_cscale, c->cscale.data(), nbf_tot * sizeof(double), hipMemcpyHostToDevice));

    // ---- shell pairs within each molecule, canonical orientation ----
    std::vector<PrimPair> prim;
    std::vector<std::vector<PairInfo>> all(6);
    for (int m = 0; m < nmol; ++m) {
        const MolInfo& M = c->mol[m];
        for (int a = M.soff; a < M.soff + M.nshell; ++a)
            for (int b = M.soff; b <= a; ++b) {
                int A = a, Bs = b;
                if (c->shells[b].l > c->shells[a].l) std::swap(A, Bs);
                const ShellHost& SA = c->shells[A];
                const ShellHost& SB = c->shells[Bs];
                PairInfo pi;
                pi.a = A;
                pi.b = Bs;
                pi.bfa = SA.bf;
                pi.bfb = SB.bf;
                pi.AB[0] = SA.x - SB.x;
                pi.AB[1] = SA.y - SB.y;
                pi.AB[2] = SA.z - SB.z;
                pi.Q = 0.0;
                pi.mol = m;
                pi.ld = M.nbf;
                const double ab2 = pi.AB[0] * pi.AB[0] + pi.AB[1] * pi.AB[1] + pi.AB[2] * pi.AB[2];
                pi.prim_off = (int)prim.size();
                int np = 0;
                double kmax = 0.0;
                for (int i = 0; i < SA.nprim; ++i)
                    for (int j = 0; j < SB.nprim; ++j) {
                        const double al = c->exps[SA.prim_off + i], be = c->exps[SB.prim_off + j];
                        const double p = al + be, mu = al * be / p;
                        PrimPair pp;
                        pp.p = p;
                        pp.inv2p = 0.5 / p;
                        pp.P[0] = (al * SA.x + be * SB.x) / p;
                        pp.P[1] = (al * SA.y + be * SB.y) / p;
                        pp.P[2] = (al * SA.z + be * SB.z) / p;
                        pp.PA[0] = pp.P[0] - SA.x;
                        pp.PA[1] = pp.P[1] - SA.y;
                        pp.PA[2] = pp.P[2] - SA.z;
                        const double ek = std::exp(-mu * ab2);
                        // sqrt(2 pi^{5/2}) = sqrt(2) pi^{5/4}
                        pp.K = c->coefs[SA.prim_off + i] * c->coefs[SB.prim_off + j] * ek * 1.4142135623730951 *
                               std::pow(M_PI, 1.25) / p;
                        pp.pad = 0.0;
                        kmax = std::max(kmax, ek);
                        prim.push_back(pp);
                        ++np;
                    }
                pi.nprim = np;
                // Gaussian overlap exp(-mu R^2) < 1e-40 for every primitive pair:
                // the pair vanishes.  (Dropping single negligible primitive pairs
                // would split the ket lists by primitive count into more, shorter
                // lists: more tasks and LDS row flushes than the primitive work saved.)
                if (kmax < 1e-40) {
                    prim.resize(pi.prim_off);
                    continue;
                }
                if (prim.size() > (size_t)0x7fffffff) return hfx_fail(c, HFX_ERR_INVALID_ARG, "too many primitive pairs");
                all[pair_class(SA.l, SB.l)].push_back(pi);
            }
    }
    HIPCK(dalloc(&c->d_prim, prim.size()));
    HIPCK(hipMemcpy(c->d_prim, prim.data(), prim.size() * sizeof(PrimPair), hipMemcpyHostToDevice));
    {   // FP32 copy, same layout, for the FP32 evaluation of mixed builds
        std::vector<float> p32(prim.size() * HFX_PRIM_FIELDS);
        const double* src = reinterpret_cast<const double*>(prim.data());
        for (size_t i = 0; i < p32.size(); ++i) p32[i] = (float)src[i];
        HIPCK(dalloc(&c->d_prim32, p32.size()));
        HIPCK(hipMemcpy(c->d_prim32, p32.data(), p32.size() * sizeof(float), hipMemcpyHostToDevice));
    }

    // ---- Schwarz bounds on the GPU (FP64 class kernels on (ab|ab)) ----
    const bool keep_qshell = nmol == 1;
    c->Qshell.assign(keep_qshell ? (size_t)nshell * nshell : 0, 0.0);
    double qmax = 0.0;
    for (int B = 0; B < 6; ++B) {
        auto& L = all[B];
        if (L.empty()) continue;
        PairInfo* dp = nullptr;
        double* dq = nullptr;
        HIPCK(dalloc(&dp, L.size()));
        HIPCK(dalloc(&dq, L.size()));
        HIPCK(hipMemcpy(dp, L.data(), L.size() * sizeof(PairInfo), hipMemcpyHostToDevice));
        HIPCK(hfx_launch_schwarz(class_id(B, B), dp, (int)L.size(), c->d_prim, c->d_boys64, dq, 0));
        std::vector<double> q(L.size());
        HIPCK(hipMemcpy(q.data(), dq, q.size() * sizeof(double), hipMemcpyDeviceToHost));
        dfree(dp);
        dfree(dq);
        for (size_t i = 0; i < L.size(); ++i) {
            if (!std::isfinite(q[i])) return hfx_fail(c, HFX_ERR_NUMERICAL, "non-finite Schwarz bound");
            L[i].Q = q[i];
            qmax = std::max(qmax, q[i]);
            if (keep_qshell) {
                c->Qshell[(size_t)L[i].a * nshell + L[i].b] = q[i];
                c->Qshell[(size_t)L[i].b * nshell + L[i].a] = q[i];
            }
        }
    }
    // ---- significant pairs, sorted by molecule then Q descending (ties: pair order) ----
    const double tau = c->opt.schwarz_tau;
    std::vector<std::vector<double>> pos(6);
    for (int B = 0; B < 6; ++B) {
        auto& L = all[B];
        std::vector<PairInfo> keep;
        keep.reserve(L.size());
        for (auto& p : L)
            if (p.Q * qmax >= tau) keep.push_back(p);
        std::stable_sort(keep.begin(), keep.end(), [](const PairInfo& x, const PairInfo& y) {
            return x.mol < y.mol || (x.mol == y.mol && x.Q > y.Q);
        });
        L.swap(keep);
        c->npair[B] = (int)L.size();
        pos[B].resize(L.size());
        for (size_t i = 0; i < L.size(); ++i) pos[B][i] = (double)i;
        HIPCK(dalloc(&c->d_pairs[B], L.size()));
        if (!L.empty()) HIPCK(hipMemcpy(c->d_pairs[B], L.data(), L.size() * sizeof(PairInfo), hipMemcpyHostToDevice));
    }
    // ---- ket lists: one per pair class and primitive count, in groups ----
    // Large molecules: the bra rows staged in LDS cover two column windows
    // of kWindow basis functions (shell c's and shell d's), so kets are
    // grouped by (molecule, window of c, window of d), Q descending within
    // a group; small ones stage whole rows (one group per molecule).
    constexpr int kWindowAbove = 2048, kWindow = 768, kWindowPad = 8;   // pad: a shell's extent past its window
    c->win = c->max_ld > kWindowAbove ? kWindow : 0;
    c->rs = c->win ? 2 * (c->win + kWindowPad) : c->max_ld;
    std::vector<std::vector<PairInfo>> klist;
    std::vector<std::vector<double>> kpos;
    c->kgroup.clear();
    c->kmolg.clear();
    c->kwcode.clear();
    for (int K = 0; K < 6; ++K) {
        std::vector<int> nps;
        for (auto& p : all[K])
            if (std::find(nps.begin(), nps.end(), p.nprim) == nps.end()) nps.push_back(p.nprim);
        std::sort(nps.begin(), nps.end());
        for (int kp : nps) {
            KetList KL;
            KL.K = K;
            KL.kp = kp;
            std::vector<PairInfo> sub;
            std::vector<double> sp;
            for (size_t i = 0; i < all[K].size(); ++i)
                if (all[K][i].nprim == kp) {
                    sub.push_back(all[K][i]);
                    sp.push_back(pos[K][i]);
                }
            KL.n = (int)sub.size();
            const size_t n = sub.size();
            auto wc_of = [&](const PairInfo& p) { return c->win ? p.bfa / c->win : 0; };
            auto wd_of = [&](const PairInfo& p) { return c->win ? p.bfb / c->win : 0; };
            if (c->win) {   // stable: Q order kept within (molecule, wc, wd)
                std::vector<size_t> idx(n);
                for (size_t i = 0; i < n; ++i) idx[i] = i;
                std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
                    const PairInfo &u = sub[x], &v = sub[y];
                    if (u.mol != v.mol) return u.mol < v.mol;
                    if (wc_of(u) != wc_of(v)) return wc_of(u) < wc_of(v);
                    return wd_of(u) < wd_of(v);
                });
                std::vector<PairInfo> s2(n);
                std::vector<double> p2(n);
                for (size_t i = 0; i < n; ++i) {
                    s2[i] = sub[idx[i]];
                    p2[i] = sp[idx[i]];
                }
                sub.swap(s2);
                sp.swap(p2);
            }
            std::vector<int> gstart, molg(nmol + 1, 0), wcode;
            for (size_t s = 0; s < n; ++s) {
                const int w = wc_of(sub[s]) | (wd_of(sub[s]) << 16);
                if (s == 0 || sub[s].mol != sub[s - 1].mol || w != wcode.back()) {
                    gstart.push_back((int)s);
                    wcode.push_back(w);
                    molg[sub[s].mol + 1] = (int)gstart.size();
                }
            }
            gstart.push_back((int)n);
            for (int m = 0; m < nmol; ++m) molg[m + 1] = std::max(molg[m + 1], molg[m]);   // molecules without kets
            std::vector<double> q(n), soa((size_t)9 * kp * n);
            std::vector<int4> kbf(n);
            for (size_t s = 0; s < n; ++s) {
                q[s] = sub[s].Q;
                kbf[s] = make_int4(sub[s].bfa, sub[s].bfb, sub[s].a, sub[s].b);
                for (int k = 0; k < kp; ++k) {
                    const PrimPair& pp = prim[sub[s].prim_off + k];
                    const double f[9] = {pp.p, pp.inv2p, pp.P[0], pp.P[1], pp.P[2], pp.PA[0], pp.PA[1], pp.PA[2], pp.K};
                    for (int fi = 0; fi < 9; ++fi) soa[((size_t)fi * kp + k) * n + s] = f[fi];
                }
            }
            HIPCK(dalloc(&KL.d_pairs, n));
            HIPCK(dalloc(&KL.d_q, n));
            HIPCK(dalloc(&KL.d_soa, soa.size()));
            KL.ncd = ncart(kPairL[K][0]) * ncart(kPairL[K][1]);
            HIPCK(dalloc(&KL.d_wket, (size_t)KL.ncd * n));
            HIPCK(dalloc(&KL.d_dket, (size_t)KL.ncd * n));
            HIPCK(dalloc(&KL.d_kbf, n));
            HIPCK(hipMemcpy(KL.d_kbf, kbf.data(), n * sizeof(int4), hipMemcpyHostToDevice));
            {
                std::vector<int> kp_int(n);
                for (size_t i = 0; i < n; ++i) kp_int[i] = (int)sp[i];
                HIPCK(dalloc(&KL.d_kpos, n));
                HIPCK(hipMemcpy(KL.d_kpos, kp_int.data(), n * sizeof(int), hipMemcpyHostToDevice));
            }
            HIPCK(hipMemcpy(KL.d_pairs, sub.data(), n * sizeof(PairInfo), hipMemcpyHostToDevice));
            HIPCK(hipMemcpy(KL.d_q, q.data(), n * sizeof(double), hipMemcpyHostToDevice));
            HIPCK(hipMemcpy(KL.d_soa, soa.data(), soa.size() * sizeof(double), hipMemcpyHostToDevice));
            {
                const std::vector<float> soa32(soa.begin(), soa.end());
                HIPCK(dalloc(&KL.d_soa32, soa32.size()));
                HIPCK(hipMemcpy(KL.d_soa32, soa32.data(), soa32.size() * sizeof(float), hipMemcpyHostToDevice));
            }
            c->ketlists.push_back(KL);
            klist.push_back(std::move(sub));
            kpos.push_back(std::move(sp));
            c->kgroup.push_back(std::move(gstart));
            c->kmolg.push_back(std::move(molg));
            c->kwcode.push_back(std::move(wcode));
        }
    }
    c->host_bra.assign(all.begin(), all.end());
    c->host_pos = pos;
    c->host_ket = std::move(klist);
    c->host_kpos = std::move(kpos);
    {
        hfx_status s = replan(c);
        if (s != HFX_OK) return s;
    }

    // ---- one-electron integrals, one launch per molecule (its own nuclei) ----
    std::vector<double> atoms(4 * (size_t)natom);
    for (long long a = 0; a < natom; ++a) {
        atoms[4 * a] = xyz[3 * a];
        atoms[4 * a + 1] = xyz[3 * a + 1];
        atoms[4 * a + 2] = xyz[3 * a + 2];
        atoms[4 * a + 3] = Z[a];
    }
    const size_t ne = c->nelem;
    ShellHost* dsh = nullptr;
    double *dexp = nullptr, *dcoef = nullptr, *datoms = nullptr, *dT = nullptr, *dV = nullptr;
    HIPCK(dalloc(&dsh, nshell));
    HIPCK(dalloc(&dexp, c->exps.size()));
    HIPCK(dalloc(&dcoef, c->coefs.size()));
    HIPCK(dalloc(&datoms, atoms.size()));
    HIPCK(dalloc(&c->d_S, ne));
    HIPCK(dalloc(&dT, ne));
    HIPCK(dalloc(&dV, ne));
    HIPCK(hipMemcpy(dsh, c->shells.data(), nshell * sizeof(ShellHost), hipMemcpyHostToDevice));
    HIPCK(hipMemcpy(dexp, c->exps.data(), c->exps.size() * 8, hipMemcpyHostToDevice));
    HIPCK(hipMemcpy(dcoef, c->coefs.data(), c->coefs.size() * 8, hipMemcpyHostToDevice));
    HIPCK(hipMemcpy(datoms, atoms.data(), atoms.size() * 8, hipMemcpyHostToDevice));
    for (int m = 0; m < nmol; ++m) {
        const MolInfo& M = c->mol[m];
        HIPCK(hfx_one_electron(dsh + M.soff, M.nshell, dexp, dcoef, datoms + 4 * (size_t)M.aoff, M.natom,
                               c->d_cscale + M.boff, c->d_boys64, M.nbf, c->d_S + M.moff, dT + M.moff, dV + M.moff,
                               0));
    }
    HIPCK(dalloc(&c->d_H, ne));
    HIPCK(hipMemcpy(c->d_H, dT, ne * 8, hipMemcpyDeviceToDevice));
    {
        const double one = 1.0;
        rocblas_set_pointer_mode(c->blas, rocblas_pointer_mode_host);
        rocblas_set_stream(c->blas, 0);
        if (rocblas_daxpy(c->blas, (rocblas_int)ne, &one, dV, 1, c->d_H, 1) != rocblas_status_success)
            return hfx_fail(c, HFX_ERR_DEVICE, "rocblas_daxpy failed");
    }
    HIPCK(hipDeviceSynchronize());
    dfree(dsh);
    dfree(dexp);
    dfree(dcoef);
    dfree(datoms);
    dfree(dT);
    dfree(dV);
    HIPCK(dalloc(&c->d_W, ne));
    HIPCK(dalloc(&c->d_Dp, ne));
    c->loaded = true;
    return HFX_OK;
}

extern "C" hfx_status hfx_load(hfx_ctx* c, int natom, const int* Z, const double* xyz, int nshell,
                               const hfx_shell* sh, int charge) {
    return hfx_load_batch(c, 1, &natom, Z, xyz, &nshell, sh, &charge);
}

extern "C" hfx_status hfx_batch_layout(const hfx_ctx* c, int* nmol, int* nbf, int* nocc, long long* offset,
                                       long long* total) {
    if (!c) return HFX_ERR_INVALID_ARG;
    if (!c->loaded) return HFX_ERR_STATE;
    if (nmol) *nmol = c->nmol;
    for (int m = 0; m < c->nmol; ++m) {
        if (nbf) nbf[m] = c->mol[m].nbf;
        if (nocc) nocc[m] = c->mol[m].nocc;
        if (offset) offset[m] = c->mol[m].moff;
    }
    if (total) *total = (long long)c->nelem;
    return HFX_OK;
}

extern "C" hfx_status hfx_dims(const hfx_ctx* c, int* nbf, int* nocc, int* nshell) {
    if (!c) return HFX_ERR_INVALID_ARG;
    if (!c->loaded) return HFX_ERR_STATE;
    if (nbf) *nbf = c->nbf;
    if (nocc) *nocc = c->nocc;
    if (nshell) *nshell = c->nshell;
    return HFX_OK;
}

extern "C" hfx_status hfx_core(hfx_ctx* c, double* S, double* H, double* enuc) {
    if (!c) return HFX_ERR_INVALID_ARG;
    if (!c->loaded) return hfx_fail(c, HFX_ERR_STATE, "hfx_core: nothing loaded");
    HIPCK(hipSetDevice(c->opt.device));
    const size_t nn = c->nelem;
    if (S) HIPCK(hipMemcpy(S, c->d_S, nn * 8, hipMemcpyDeviceToHost));
    if (H) HIPCK(hipMemcpy(H, c->d_H, nn * 8, hipMemcpyDeviceToHost));
    if (enuc) *enuc = c->enuc;
    return HFX_OK;
}

extern "C" hfx_status hfx_schwarz(hfx_ctx* c, double* Q) {
    if (!c || !Q) return HFX_ERR_INVALID_ARG;
    if (!c->loaded) return hfx_fail(c, HFX_ERR_STATE, "hfx_schwarz: nothing loaded");
    if (c->nmol != 1) return hfx_fail(c, HFX_ERR_STATE, "hfx_schwarz: single-molecule contexts only");
    std::memcpy(Q, c->Qshell.data(), c->Qshell.size() * sizeof(double));
    return HFX_OK;
}

extern "C" hfx_status hfx_class_counts(const hfx_ctx* c, long long* counts) {
    if (!c || !counts) return HFX_ERR_INVALID_ARG;
    if (!c->loaded) return HFX_ERR_STATE;
    for (int k = 0; k < 21; ++k) {
        counts[4 * k] = c->totals[k].quartets;
        counts[4 * k + 1] = c->totals[k].integrals;
        counts[4 * k + 2] = c->totals[k].prim;
        counts[4 * k + 3] = c->totals[k].ntask;
    }
    return HFX_OK;
}

// ---- kernel timing ---------------------------------------------------------------------

static void collect_timing(hfx_ctx* c) {
    for (auto& p : c->plans)
        if (p.pending) {
            (void)hipEventSynchronize(p.ev1);
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, p.ev0, p.ev1) == hipSuccess) {
                p.ms += ms;
                p.launches += 1;
            }
            p.pending = false;
        }
}

extern "C" hfx_status hfx_kernel_timing(hfx_ctx* c, int enable) {
    if (!c) return HFX_ERR_INVALID_ARG;
    collect_timing(c);
    c->timing = enable != 0;
    for (auto& p : c->plans) {
        p.ms = 0.0;
        p.launches = 0;
        if (c->timing && !p.ev0) {
            HIPCK(hipEventCreate(&p.ev0));
            HIPCK(hipEventCreate(&p.ev1));
        }
    }
    return HFX_OK;
}

extern "C" hfx_status hfx_set_streams(hfx_ctx* c, int n) {
    if (!c) return HFX_ERR_INVALID_ARG;
    if (n < 1 || n > hfx_ctx::kMaxStreams)
        return hfx_fail(c, HFX_ERR_INVALID_ARG, "set_streams: between 1 and 4 streams");
    c->nstreams = n;
    return HFX_OK;
}

extern "C" hfx_status hfx_kernel_times(hfx_ctx* c, double* ms, long long* launches) {
    if (!c) return HFX_ERR_INVALID_ARG;
    collect_timing(c);
    double m[21] = {0};
    long long l[21] = {0};
    for (auto& p : c->plans) {
        m[p.cid] += p.ms;
        l[p.cid] = std::max(l[p.cid], p.launches);
    }
    for (int k = 0; k < 21; ++k) {
        if (ms) ms[k] = m[k];
        if (launches) launches[k] = l[k];
    }
    return HFX_OK;
}

extern "C" hfx_status hfx_plan_count(const hfx_ctx* c, int* n) {
    if (!c || !n) return HFX_ERR_INVALID_ARG;
    *n = (int)c->plans.size();
    return HFX_OK;
}

extern "C" hfx_status hfx_plan_info(hfx_ctx* c, int i, long long* info, double* ms) {
    if (!c || !info || i < 0 || i >= (int)c->plans.size()) return HFX_ERR_INVALID_ARG;
    collect_timing(c);
    const SubPlan& p = c->plans[i];
    const KetList& KL = c->ketlists[p.list];
    info[0] = p.cid;
    info[1] = KL.kp;
    info[2] = p.ntask;
    info[3] = p.quartets;
    info[4] = p.prim;
    info[5] = p.integrals;
    info[6] = p.launches;
    info[7] = p.priv ? HFX_DIGEST_PRIVATE : p.mode == 1 ? HFX_DIGEST_GLOBAL : p.dstage ? HFX_DIGEST_LDS_D : HFX_DIGEST_LDS;
    info[8] = hfx_class_wgs(p.cid, p.alt);
    info[9] = p.kr ? c->tune_persist[p.cid] : (p.persist ? (p.wave ? 2 : 1) : 0);
    info[10] = p.persist ? p.nblocks[0] : p.ntask;   // the FP64 kernel's grid
    info[11] = p.nbl;
    info[12] = p.dstage;
    if (ms) *ms = p.ms;
    return HFX_OK;
}

// ---- the Fock build -------------------------------------------------------------------

// Per class, FP64 and FP32 evaluated-quartet counts: the sums of their slots.
static hipError_t read_counters(const unsigned long long* d, long long* cnt) {
    std::vector<unsigned long long> w(HFX_CNT_WORDS);
    const hipError_t e = hipMemcpy(w.data(), d, w.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    for (int k = 0; k < 42; ++k) {
        unsigned long long t = 0;
        for (int j = 0; j < HFX_CNT_SLOTS; ++j) t += w[(size_t)k * HFX_CNT_SLOTS * HFX_CNT_STRIDE + j * HFX_CNT_STRIDE];
        cnt[k] = (long long)t;
    }
    return hipSuccess;
}

hfx_status hfx_build_internal(hfx_ctx* c, const double* dD, double cj, double ck, const double* dH, double* dOut,
                              hipStream_t st, hfx_fock_stats* stats, int shard, int nshards) {
    BuildBufs b;
    b.W = c->d_W;
    b.Dp = c->d_Dp;
    b.dmax = c->d_dmax;
    b.counters = c->d_counters;
    b.bad = c->d_bad;
    b.work = c->d_work;
    return hfx_build_with(c, b, dD, cj, ck, dH, dOut, st, stats, shard, nshards);
}

// Streams of a build's class launches: the launch plans are dealt
// round-robin over the caller's stream and ns - 1 side streams, so a launch
// on one stream fills the CUs that the previous launch on another stream
// frees while its last tasks finish (every class kernel accumulates with
// atomics, so concurrent launches need no ordering).  Per-launch timing keeps
// every launch on the caller's stream: its events then bracket only its own
// kernel.
static int build_streams(const hfx_ctx* c) {
    return c->timing ? 1 : std::min<int>(c->nstreams, (int)c->plans.size());
}

static hipError_t fork_streams(hfx_ctx* c, int ns, hipStream_t st) {
    if (ns <= 1) return hipSuccess;
    hipError_t e = hipEventRecord(c->ev_fork, st);   // after all earlier work on the caller's stream
    for (int s = 0; s < ns - 1 && e == hipSuccess; ++s) e = hipStreamWaitEvent(c->side[s], c->ev_fork, 0);
    return e;
}

static hipError_t join_streams(hfx_ctx* c, int ns, hipStream_t st) {
    hipError_t e = hipSuccess;
    for (int s = 0; s < ns - 1 && e == hipSuccess; ++s) {
        e = hipEventRecord(c->ev_join[s], c->side[s]);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, c->ev_join[s], 0);
    }
    return e;
}

static hipStream_t plan_stream(const hfx_ctx* c, int ns, size_t pi, hipStream_t st) {
    const int k = (int)(pi % (size_t)ns);
    return k ? c->side[k - 1] : st;
}

hfx_status hfx_build_with(hfx_ctx* c, const BuildBufs& bufs, const double* dD, double cj, double ck,
                          const double* dH, double* dOut, hipStream_t st, hfx_fock_stats* stats, int shard,
                          int nshards) {
    if (!c->loaded) return hfx_fail(c, HFX_ERR_STATE, "build: nothing loaded");
    const size_t nn = c->nelem;
    const bool mixed = c->opt.precision == HFX_PREC_MIXED;
    auto t0 = std::chrono::steady_clock::now();
    if (c->timing) collect_timing(c);
    HIPCK(hfx_fill_u64(bufs.dmax, 1, st));
    HIPCK(hfx_fill_u64(bufs.counters, HFX_CNT_WORDS + 1, st));   // quartet counters + the non-finite flag
    HIPCK(hfx_prepare_density(dD, c->d_cscale, c->nmol, c->d_moff, c->d_mdim, c->d_mboff, c->max_ld, bufs.Dp,
                              bufs.dmax, st));
    HIPCK(hfx_fill(bufs.W, nn, 0.0, st));
    for (auto& KL : c->ketlists) {
        HIPCK(hfx_fill(KL.d_wket, (size_t)KL.ncd * KL.n, 0.0, st));
        HIPCK(hfx_gather_ket(KL.d_pairs, KL.n, ncart(kPairL[KL.K][0]), ncart(kPairL[KL.K][1]), bufs.Dp, c->d_moff,
                             KL.d_dket, st));
    }
    bool any_persist = false, any_priv = false;
    for (const auto& P : c->plans) {
        any_persist |= P.persist;
        any_priv |= P.priv;
    }
    if (any_persist) HIPCK(hfx_fill_u64(bufs.work, 16 * (int)c->plans.size(), st));
    if (any_priv) {
        if (!c->d_Wrep) return hfx_fail(c, HFX_ERR_STATE, "build: private digestion without its copies of W");
        HIPCK(hfx_fill(c->d_Wrep, kXcds * nn, 0.0, st));
    }
    const int ns = build_streams(c);
    HIPCK(fork_streams(c, ns, st));
    for (size_t pi = 0; pi < c->plans.size(); ++pi) {
        SubPlan& P = c->plans[pi];
        const KetList& KL = c->ketlists[P.list];
        const int cid = P.cid;
        const bool mx = mixed && !P.fp64_only && c->tune_fp32[cid] && !P.kr;
        const hipStream_t ps = plan_stream(c, ns, pi, st);
        if (mx)
            HIPCK(hfx_split(c->d_pairs[P.B], KL.d_q, P.d_tasks, P.ntask, c->opt.fp32_tau, bufs.dmax, P.d_split,
                            ps));
        ClassArgs a;
        a.bra = c->d_pairs[P.B];
        a.ket = KL.d_pairs;
        a.kbf = KL.d_kbf;
        a.dket = KL.d_dket;
        a.prim = c->d_prim;
        a.kprim = KL.d_soa;
        a.prim32 = c->d_prim32;
        a.kprim32 = KL.d_soa32;
        a.nket_list = KL.n;
        a.knprim = KL.kp;
        a.split = mx ? P.d_split : nullptr;
        a.win = c->win;
        a.rs = c->rs;
        a.dstage = P.dstage;
        a.moff = c->d_moff;
        a.tasks = P.d_tasks;
        a.boys64 = c->d_boys64;
        a.D = bufs.Dp;
        a.W = P.priv ? c->d_Wrep : bufs.W;
        a.wrep = P.priv ? (long long)nn : 0;
        a.wket = KL.d_wket;
        a.counters = bufs.counters + (size_t)cid * HFX_CNT_CLASS;
        a.cj = cj;
        a.ck = ck;
        a.shard = shard;
        a.nshards = nshards;
        a.work = P.persist ? bufs.work + 16 * pi : nullptr;
        a.ketq = KL.d_q;
        a.kpos = KL.d_kpos;
        a.tau = c->opt.schwarz_tau;
        a.same = P.B == P.K;
        a.qlen = P.ntask / 8;
        a.task_off = 0;
        // a static grid of ntask workgroups is cut into launches of at most
        // kMaxGroups (2^20 x 1024 lanes < 2^32 work-items; a multiple of 8
        // keeps workgroup i on XCD i mod 8 in step with the task queues)
        constexpr int kMaxGroups = 1 << 20;
        if (c->timing && P.ev0) HIPCK(hipEventRecord(P.ev0, ps));
        // one launch per plan; a mixed build's kernel evaluates each task's
        // kets before its split in FP64 and the rest in FP32
        const int m = mx ? 1 : 0;
        if (P.kr) {
            HIPCK(hfx_launch_class_kr(cid, P.mode, KL.kp, P.nbl, P.nblocks[0], P.lds(), ps, &a));
        } else if (P.persist) {
            HIPCK(hfx_launch_class(cid, P.alt, P.wave > 0, P.mode, m, P.nblocks[m], P.lds(), ps, &a));
        } else {
            for (int off = 0; off < P.ntask; off += kMaxGroups) {
                a.task_off = off;
                HIPCK(hfx_launch_class(cid, P.alt, 0, P.mode, m, std::min(kMaxGroups, P.ntask - off), P.lds(), ps,
                                       &a));
            }
        }
        if (c->timing && P.ev1) {
            HIPCK(hipEventRecord(P.ev1, ps));
            P.pending = true;
        }
    }
    HIPCK(join_streams(c, ns, st));
    if (any_priv) HIPCK(hfx_reduce_replicas(c->d_Wrep, kXcds, nn, bufs.W, st));
    for (auto& KL : c->ketlists)
        HIPCK(hfx_scatter_ket(KL.d_pairs, KL.n, ncart(kPairL[KL.K][0]), ncart(kPairL[KL.K][1]), KL.d_wket, c->d_moff, bufs.W,
                              st));
    HIPCK(hfx_assemble(dH, bufs.W, c->d_cscale, c->nmol, c->d_moff, c->d_mdim, c->d_mboff, c->max_ld, dOut, bufs.bad,
                       st));
    c->last_stream = st;
    if (stats) {
        HIPCK(hipStreamSynchronize(st));
        long long cnt[42];
        int bad = 0;
        HIPCK(read_counters(bufs.counters, cnt));
        HIPCK(hipMemcpy(&bad, bufs.bad, sizeof(int), hipMemcpyDeviceToHost));
        stats->quartets_fp64 = stats->quartets_fp32 = stats->integrals = stats->prim_quartets = 0;
        for (int k = 0; k < 21; ++k) {
            stats->quartets_fp64 += cnt[2 * k];
            stats->quartets_fp32 += cnt[2 * k + 1];
            stats->integrals += c->totals[k].integrals;
            stats->prim_quartets += c->totals[k].prim;
        }
        stats->t_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (bad) return hfx_fail(c, HFX_ERR_NUMERICAL, "non-finite value in the Fock matrix");
    }
    return HFX_OK;
}

static bool finite_host(const double* p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

extern "C" hfx_status hfx_build_fock_dev(hfx_ctx* c, const double* dD, double* dF, void* stream,
                                         hfx_fock_stats* stats) {
    if (!c || !dD || !dF) return c ? hfx_fail(c, HFX_ERR_INVALID_ARG, "null pointer") : HFX_ERR_INVALID_ARG;
    HIPCK(hipSetDevice(c->opt.device));
    return hfx_build_internal(c, dD, 2.0, 1.0, c->d_H, dF, (hipStream_t)stream, stats, 0, 1);
}

extern "C" hfx_status hfx_build_2e_dev(hfx_ctx* c, const double* dD, double cj, double ck, double* dG, void* stream,
                                       hfx_fock_stats* stats) {
    if (!c || !dD || !dG) return c ? hfx_fail(c, HFX_ERR_INVALID_ARG, "null pointer") : HFX_ERR_INVALID_ARG;
    if (!std::isfinite(cj) || !std::isfinite(ck)) return hfx_fail(c, HFX_ERR_INVALID_ARG, "non-finite cj/ck");
    HIPCK(hipSetDevice(c->opt.device));
    return hfx_build_internal(c, dD, cj, ck, nullptr, dG, (hipStream_t)stream, stats, 0, 1);
}

extern "C" hfx_status hfx_build_2e_shard_dev(hfx_ctx* c, const double* dD, double cj, double ck, int shard,
                                             int nshards, double* dG, void* stream, hfx_fock_stats* stats) {
    if (!c || !dD || !dG) return c ? hfx_fail(c, HFX_ERR_INVALID_ARG, "null pointer") : HFX_ERR_INVALID_ARG;
    if (nshards < 1 || shard < 0 || shard >= nshards) return hfx_fail(c, HFX_ERR_INVALID_ARG, "bad shard");
    if (!std::isfinite(cj) || !std::isfinite(ck)) return hfx_fail(c, HFX_ERR_INVALID_ARG, "non-finite cj/ck");
    HIPCK(hipSetDevice(c->opt.device));
    return hfx_build_internal(c, dD, cj, ck, nullptr, dG, (hipStream_t)stream, stats, shard, nshards);
}

// ---- several densities in one pass ------------------------------------------------
// Every screened quartet is evaluated once and digested for each density
// (section 7 of the paper names UHF, GVB, DFT and CPHF as sharing this loop
// structure: an alpha and a beta density, or one density per perturbation).

extern "C" hfx_status hfx_build_jk_multi_dev(hfx_ctx* c, int ndens, const double* dD, double* dJ, double* dK,
                                             void* stream, hfx_fock_stats* stats) {
    if (!c) return HFX_ERR_INVALID_ARG;
    if (ndens < 1 || ndens > 64 || !dD || (!dJ && !dK))
        return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_build_jk_multi_dev: ndens in [1, 64], dD and dJ or dK needed");
    if (!c->loaded) return hfx_fail(c, HFX_ERR_STATE, "hfx_build_jk_multi_dev: nothing loaded");
    HIPCK(hipSetDevice(c->opt.device));
    hipStream_t st = (hipStream_t)stream;
    const size_t nn = c->nelem;
    auto t0 = std::chrono::steady_clock::now();
    if (c->multi_cap < ndens) {
        dfree(c->d_multi);
        c->multi_cap = 0;
        HIPCK(dalloc(&c->d_multi, 3 * (size_t)ndens * nn));
        c->multi_cap = ndens;
    }
    for (auto& KL : c->ketlists)
        if (KL.dket_multi_cap < ndens) {
            dfree(KL.d_dket_multi);
            dfree(KL.d_wket_multi);
            KL.dket_multi_cap = 0;
            HIPCK(dalloc(&KL.d_dket_multi, (size_t)ndens * KL.ncd * KL.n));
            HIPCK(dalloc(&KL.d_wket_multi, (size_t)ndens * KL.ncd * KL.n));
            KL.dket_multi_cap = ndens;
        }
    // densities per launch of a plan: as many LDS row sets as fit beside the
    // Boys rows (MODE 0), else all of them with global atomics (MODE 1)
    std::vector<int> group(c->plans.size()), gmode(c->plans.size());
    size_t nwork = 0;
    for (size_t pi = 0; pi < c->plans.size(); ++pi) {
        const SubPlan& P = c->plans[pi];
        const size_t budget = 160 * 1024 - 256;
        const size_t fit = P.lds_tab < budget ? (budget - P.lds_tab) / std::max<size_t>(1, P.lds_bytes) : 0;
        const bool lds = P.mode == 0 && !P.priv && fit >= 1;
        gmode[pi] = lds ? 0 : 1;
        group[pi] = lds ? (int)std::min<size_t>(fit, (size_t)ndens) : ndens;
        nwork += 8 * (size_t)((ndens + group[pi] - 1) / group[pi]);
    }
    if (c->multi_work_cap < nwork) {
        dfree(c->d_multi_work);
        c->multi_work_cap = 0;
        HIPCK(dalloc(&c->d_multi_work, nwork));
        c->multi_work_cap = nwork;
    }
    double* Dp = c->d_multi;
    double* WJ = Dp + (size_t)ndens * nn;
    double* WK = WJ + (size_t)ndens * nn;
    HIPCK(hfx_fill_u64(c->d_dmax, 1, st));
    HIPCK(hfx_fill_u64(c->d_counters, HFX_CNT_WORDS + 1, st));
    for (int d = 0; d < ndens; ++d)
        HIPCK(hfx_prepare_density(dD + (size_t)d * nn, c->d_cscale, c->nmol, c->d_moff, c->d_mdim, c->d_mboff,
                                  c->max_ld, Dp + (size_t)d * nn, c->d_dmax, st));
    HIPCK(hfx_fill(WJ, 2 * (size_t)ndens * nn, 0.0, st));
    for (auto& KL : c->ketlists) {
        HIPCK(hfx_fill(KL.d_wket_multi, (size_t)ndens * KL.ncd * KL.n, 0.0, st));
        for (int d = 0; d < ndens; ++d)
            HIPCK(hfx_gather_ket(KL.d_pairs, KL.n, ncart(kPairL[KL.K][0]), ncart(kPairL[KL.K][1]),
                                 Dp + (size_t)d * nn, c->d_moff, KL.d_dket_multi + (size_t)d * KL.ncd * KL.n, st));
    }
    HIPCK(hfx_fill_u64(c->d_multi_work, (int)nwork, st));
    size_t wofs = 0;
    const int ns = build_streams(c);
    HIPCK(fork_streams(c, ns, st));
    for (size_t pi = 0; pi < c->plans.size(); ++pi) {
        const SubPlan& P = c->plans[pi];
        const KetList& KL = c->ketlists[P.list];
        const hipStream_t ps = plan_stream(c, ns, pi, st);
        ClassArgs a;
        std::memset(&a, 0, sizeof(a));
        a.bra = c->d_pairs[P.B];
        a.ket = KL.d_pairs;
        a.kbf = KL.d_kbf;
        a.prim = c->d_prim;
        a.kprim = KL.d_soa;
        a.nket_list = KL.n;
        a.knprim = KL.kp;
        a.tasks = P.d_tasks;
        a.moff = c->d_moff;
        a.boys64 = c->d_boys64;
        a.D = Dp;
        a.W = WJ;
        a.WK = WK;
        a.dket = KL.d_dket_multi;
        a.counters = c->d_counters + (size_t)P.cid * HFX_CNT_CLASS;
        a.cj = 1.0;    // J updates into W: (W + W^T)/8 = J
        a.ck = -1.0;   // K updates into WK: (WK + WK^T)/8 = K
        a.nshards = 1;
        a.qlen = P.ntask / 8;
        a.ketq = KL.d_q;
        a.kpos = KL.d_kpos;
        a.tau = c->opt.schwarz_tau;
        a.same = P.B == P.K;
        a.win = c->win;
        a.rs = c->rs;
        a.dstride = (long long)nn;
        a.kstride = (long long)KL.ncd * KL.n;
        const int nblocks = ((std::min(P.ntask, 2048) + 7) / 8) * 8;   // resident or queued: queues drain either way
        for (int d0 = 0; d0 < ndens; d0 += group[pi]) {
            ClassArgs b = a;
            b.ndens = std::min(group[pi], ndens - d0);
            b.D = Dp + (size_t)d0 * nn;
            b.W = WJ + (size_t)d0 * nn;
            b.WK = WK + (size_t)d0 * nn;
            b.dket = KL.d_dket_multi + (size_t)d0 * a.kstride;
            b.wket = KL.d_wket_multi + (size_t)d0 * a.kstride;
            b.work = c->d_multi_work + wofs;
            wofs += 8;
            const size_t lds = P.lds_tab + (gmode[pi] == 0 ? (size_t)b.ndens * P.lds_bytes : 0);
            HIPCK(hfx_launch_class_multi(P.cid, gmode[pi], nblocks, lds, ps, &b));
        }
    }
    HIPCK(join_streams(c, ns, st));
    for (auto& KL : c->ketlists)   // each density's ket-block J sums into its J accumulator
        for (int d = 0; d < ndens; ++d)
            HIPCK(hfx_scatter_ket(KL.d_pairs, KL.n, ncart(kPairL[KL.K][0]), ncart(kPairL[KL.K][1]),
                                  KL.d_wket_multi + (size_t)d * KL.ncd * KL.n, c->d_moff, WJ + (size_t)d * nn, st));
    for (int d = 0; d < ndens; ++d) {
        if (dJ)
            HIPCK(hfx_assemble(nullptr, WJ + (size_t)d * nn, c->d_cscale, c->nmol, c->d_moff, c->d_mdim, c->d_mboff,
                               c->max_ld, dJ + (size_t)d * nn, c->d_bad, st));
        if (dK)
            HIPCK(hfx_assemble(nullptr, WK + (size_t)d * nn, c->d_cscale, c->nmol, c->d_moff, c->d_mdim, c->d_mboff,
                               c->max_ld, dK + (size_t)d * nn, c->d_bad, st));
    }
    c->last_stream = st;
    if (stats) {
        HIPCK(hipStreamSynchronize(st));
        long long cnt[42];
        int bad = 0;
        HIPCK(read_counters(c->d_counters, cnt));
        HIPCK(hipMemcpy(&bad, c->d_bad, sizeof(int), hipMemcpyDeviceToHost));
        stats->quartets_fp64 = stats->quartets_fp32 = stats->integrals = stats->prim_quartets = 0;
        for (int k = 0; k < 21; ++k) {
            stats->quartets_fp64 += cnt[2 * k];
            stats->integrals += c->totals[k].integrals;
            stats->prim_quartets += c->totals[k].prim;
        }
        stats->t_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (bad) return hfx_fail(c, HFX_ERR_NUMERICAL, "non-finite value in J or K");
    }
    return HFX_OK;
}

// ---- HIP graph of one build -------------------------------------------------------
// One eager build first (kernel attributes, first-touch), then the same
// launch sequence is captured on the caller's stream and instantiated.  Every
// node is a kernel (fills are kernels too: no memset nodes).

extern "C" hfx_status hfx_graph_capture(hfx_ctx* c, const double* dD, double* dF, void* stream) {
    if (!c || !dD || !dF || !stream)
        return c ? hfx_fail(c, HFX_ERR_INVALID_ARG, "graph capture needs device pointers and a non-null stream")
                 : HFX_ERR_INVALID_ARG;
    if (!c->loaded) return hfx_fail(c, HFX_ERR_STATE, "hfx_graph_capture: nothing loaded");
    HIPCK(hipSetDevice(c->opt.device));
    hipStream_t st = (hipStream_t)stream;
    drop_graph(c);
    const bool timing = c->timing;
    c->timing = false;
    hfx_status s = hfx_build_internal(c, dD, 2.0, 1.0, c->d_H, dF, st, nullptr, 0, 1);
    if (s != HFX_OK) {
        c->timing = timing;
        return s;
    }
    HIPCK(hipStreamSynchronize(st));
    HIPCK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    s = hfx_build_internal(c, dD, 2.0, 1.0, c->d_H, dF, st, nullptr, 0, 1);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    c->timing = timing;
    if (s != HFX_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    HIPCK(e);
    const hipError_t ei = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCK(ei);
    return HFX_OK;
}

extern "C" hfx_status hfx_graph_launch(hfx_ctx* c, void* stream) {
    if (!c) return HFX_ERR_INVALID_ARG;
    if (!c->graph_exec) return hfx_fail(c, HFX_ERR_STATE, "hfx_graph_launch: no captured graph");
    HIPCK(hipSetDevice(c->opt.device));
    HIPCK(hipGraphLaunch(c->graph_exec, (hipStream_t)stream));
    return HFX_OK;
}

extern "C" hfx_status hfx_build_fock(hfx_ctx* c, const double* D, double* F, hfx_fock_stats* stats) {
    if (!c || !D || !F) return c ? hfx_fail(c, HFX_ERR_INVALID_ARG, "null pointer") : HFX_ERR_INVALID_ARG;
    if (!c->loaded) return hfx_fail(c, HFX_ERR_STATE, "hfx_build_fock: nothing loaded");
    const size_t nn = c->nelem;
    if (!finite_host(D, nn)) return hfx_fail(c, HFX_ERR_NUMERICAL, "non-finite density");
    HIPCK(hipSetDevice(c->opt.device));
    if (!c->d_tmpD) HIPCK(dalloc(&c->d_tmpD, nn));
    if (!c->d_tmpF) HIPCK(dalloc(&c->d_tmpF, nn));
    HIPCK(hipMemcpy(c->d_tmpD, D, nn * 8, hipMemcpyHostToDevice));
    hfx_fock_stats local;
    hfx_status s = hfx_build_internal(c, c->d_tmpD, 2.0, 1.0, c->d_H, c->d_tmpF, 0, stats ? stats : &local, 0, 1);
    if (s != HFX_OK) return s;
    HIPCK(hipMemcpy(F, c->d_tmpF, nn * 8, hipMemcpyDeviceToHost));
    return HFX_OK;
}
