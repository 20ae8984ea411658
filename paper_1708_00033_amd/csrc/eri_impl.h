// Direct J/K digestion kernels: one launch per canonical quartet class.
//
// Work decomposition (the paper's algorithm 3 re-expressed for one GPU):
// pairs of a class are sorted by Schwarz bound Q, so for a bra pair r the
// kets that survive screening Q_r Q_s >= tau are a prefix of the ket list
// (for bra and ket of the same class, additionally s <= r keeps each
// unordered quartet once).  A workgroup task is one bra pair and up to
// consecutive kets of its prefix (at most task_quartets); lanes take one
// quartet each.
//
// Digestion (section 4.1, eq. 2) accumulates W with
//   W_ab += 2 cj g D_cd,  W_cd += 2 cj g D_ab,
//   W_ac -= ck g D_bd,    W_bd -= ck g D_ac,  W_ad -= ck g D_bc,  W_bc -= ck g D_ad,
// g = s (ab|cd), s the number of distinct permutations of the unique quartet,
// and the two-electron Fock part is (W + W^T)/8 = cj J - ck K.
//
// MODE 0 (LDS-staged): like algorithm 3's private F_I / F_J buffers, the two
// bra rows a and b of W live in LDS for the whole task: the bra block W_ab
// is summed in registers, W_ac/W_ad/W_bc/W_bd go to LDS with ds_add_f64, and
// only the ket block W_cd goes straight to HBM with global atomics.  At the
// end of the task the LDS rows are flushed with one atomic per touched
// element.  MODE 1 (global): every update is a global atomic, into one
// shared W or (private digestion, ClassArgs::wrep) into the copy of W of the
// XCD the wave runs on; the copies are summed after the class launches.
#pragma once
#include "hfx_internal.h"

#define HFX_WG 256
// integral blocks at least this large are digested with rolled loops
#define HFX_ROLLED_DIGEST_MIN 600



// K update of W[grow][gcol]: MODE 0 into the task's LDS bra row at column
// lcol (gcol less the column base of its window), MODE 1 straight into W.
template <int MODE>
__device__ __forceinline__ void row_add(double* lds_row, double* W, int grow, int gcol, int N, int lcol, double v) {
    if constexpr (MODE == 0) {
        atomicAdd(lds_row + lcol, v);
    } else {
        atomicAdd(W + (size_t)grow * N + gcol, v);
    }
}

// dket: the gathered D'_cd of the ket list ([component][ket position]); W
// receives the J updates and WK the K updates of MODE 1 (one matrix for a
// Fock build, separate J and K accumulators for a multi-density build).
// DST (LDS digestion): bit 0, the bra's D' rows of shell a come from their
// LDS copy DI (same columns as FI); bit 1, those of shell b from DJ.
template <int NA, int NB, int NC, int ND, int MODE, int DST = 0>
__device__ __forceinline__ void digest(const double* I, double g, const ClassArgs& a, const PairInfo& bra,
                                       int fc, int fd, int spos, const double* dab, double* jab, double* FI,
                                       double* FJ, const double* __restrict__ D, double* W, int N,
                                       int RS, int cb, int db, const double* __restrict__ dket, double* WK,
                                       double* wket, const double* DI = nullptr, const double* DJ = nullptr) {
    const int fa = bra.bfa, fb = bra.bfb;
    const double cj2 = 2.0 * a.cj * g, ckg = -a.ck * g;
    // J, bra block: per-lane running sums over the task (reduced at the end)
    {
        // D_cd gathered in ket-list order before the build (coalesced across lanes)
        double dcd[NC * ND];
#pragma unroll
        for (int ls = 0; ls < NC * ND; ++ls) dcd[ls] = dket[(size_t)ls * a.nket_list + spos];
#pragma unroll
        for (int mn = 0; mn < NA * NB; ++mn) {
            double v = 0.0;
#pragma unroll
            for (int ls = 0; ls < NC * ND; ++ls) v += I[mn * NC * ND + ls] * dcd[ls];
            jab[mn] += g * v;
        }
    }
    // J, ket block.  MODE 0: into the ket list's own accumulator, indexed by
    // ket position so that a wave's atomics fall in a few 64-byte lines
    // (scattered into W once per build); MODE 1: straight into W.
#pragma unroll
    for (int l = 0; l < NC; ++l)
#pragma unroll
        for (int s = 0; s < ND; ++s) {
            double v = 0.0;
#pragma unroll
            for (int mn = 0; mn < NA * NB; ++mn) v += I[mn * NC * ND + l * ND + s] * dab[mn];
            if constexpr (MODE == 0)
                atomicAdd(wket + (size_t)(l * ND + s) * a.nket_list + spos, cj2 * v);
            else
                atomicAdd(W + (size_t)(fc + l) * N + fd + s, cj2 * v);
        }
    // K: W_ac -= ck g sum_{nu sigma} I D_bd
    {
        double dbd[NB * ND];
#pragma unroll
        for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int s = 0; s < ND; ++s)
                dbd[n * ND + s] = (DST & 2) ? DJ[n * RS + fd + s - db] : D[(size_t)(fb + n) * N + fd + s];
#pragma unroll
        for (int m = 0; m < NA; ++m)
#pragma unroll
            for (int l = 0; l < NC; ++l) {
                double v = 0.0;
#pragma unroll
                for (int n = 0; n < NB; ++n)
#pragma unroll
                    for (int s = 0; s < ND; ++s) v += I[((m * NB + n) * NC + l) * ND + s] * dbd[n * ND + s];
                row_add<MODE>(FI + m * RS, WK, fa + m, fc + l, N, fc + l - cb, ckg * v);
            }
    }
    // K: W_bd -= ck g sum_{mu lambda} I D_ac
    {
        double dac[NA * NC];
#pragma unroll
        for (int m = 0; m < NA; ++m)
#pragma unroll
            for (int l = 0; l < NC; ++l)
                dac[m * NC + l] = (DST & 1) ? DI[m * RS + fc + l - cb] : D[(size_t)(fa + m) * N + fc + l];
#pragma unroll
        for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int s = 0; s < ND; ++s) {
                double v = 0.0;
#pragma unroll
                for (int m = 0; m < NA; ++m)
#pragma unroll
                    for (int l = 0; l < NC; ++l) v += I[((m * NB + n) * NC + l) * ND + s] * dac[m * NC + l];
                row_add<MODE>(FJ + n * RS, WK, fb + n, fd + s, N, fd + s - db, ckg * v);
            }
    }
    // K: W_ad -= ck g sum_{nu lambda} I D_bc
    {
        double dbc[NB * NC];
#pragma unroll
        for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int l = 0; l < NC; ++l)
                dbc[n * NC + l] = (DST & 2) ? DJ[n * RS + fc + l - cb] : D[(size_t)(fb + n) * N + fc + l];
#pragma unroll
        for (int m = 0; m < NA; ++m)
#pragma unroll
            for (int s = 0; s < ND; ++s) {
                double v = 0.0;
#pragma unroll
                for (int n = 0; n < NB; ++n)
#pragma unroll
                    for (int l = 0; l < NC; ++l) v += I[((m * NB + n) * NC + l) * ND + s] * dbc[n * NC + l];
                row_add<MODE>(FI + m * RS, WK, fa + m, fd + s, N, fd + s - db, ckg * v);
            }
    }
    // K: W_bc -= ck g sum_{mu sigma} I D_ad
    {
        double dad[NA * ND];
#pragma unroll
        for (int m = 0; m < NA; ++m)
#pragma unroll
            for (int s = 0; s < ND; ++s)
                dad[m * ND + s] = (DST & 1) ? DI[m * RS + fd + s - db] : D[(size_t)(fa + m) * N + fd + s];
#pragma unroll
        for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int l = 0; l < NC; ++l) {
                double v = 0.0;
#pragma unroll
                for (int m = 0; m < NA; ++m)
#pragma unroll
                    for (int s = 0; s < ND; ++s) v += I[((m * NB + n) * NC + l) * ND + s] * dad[m * ND + s];
                row_add<MODE>(FJ + n * RS, WK, fb + n, fc + l, N, fc + l - cb, ckg * v);
            }
    }
}

// The updates of digest() for the register-tiled kernels: D_cd comes in
// registers (read once per ket) and the ket block's J contribution is summed
// into jcd over the bras of a block (one atomic per ket and component after
// the block) instead of one atomic per quartet.
template <int NA, int NB, int NC, int ND, int MODE>
__device__ __forceinline__ void digest_kr(const double* I, double g, double ck, const PairInfo& bra, int fc, int fd,
                                          const double* dcd, const double* dab, double* jab, double* jcd,
                                          double* FI, double* FJ, const double* __restrict__ D,
                                          double* __restrict__ W, int N, int RS, int cb, int db) {
    const int fa = bra.bfa, fb = bra.bfb;
    const double ckg = -ck * g;
#pragma unroll
    for (int mn = 0; mn < NA * NB; ++mn) {
        double v = 0.0;
#pragma unroll
        for (int ls = 0; ls < NC * ND; ++ls) v += I[mn * NC * ND + ls] * dcd[ls];
        jab[mn] += g * v;
    }
#pragma unroll
    for (int ls = 0; ls < NC * ND; ++ls) {
        double v = 0.0;
#pragma unroll
        for (int mn = 0; mn < NA * NB; ++mn) v += I[mn * NC * ND + ls] * dab[mn];
        jcd[ls] += g * v;
    }
    {   // K: W_ac -= ck g sum I D_bd
        double dbd[NB * ND];
#pragma unroll
        for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int s = 0; s < ND; ++s) dbd[n * ND + s] = D[(size_t)(fb + n) * N + fd + s];
#pragma unroll
        for (int m = 0; m < NA; ++m)
#pragma unroll
            for (int l = 0; l < NC; ++l) {
                double v = 0.0;
#pragma unroll
                for (int n = 0; n < NB; ++n)
#pragma unroll
                    for (int s = 0; s < ND; ++s) v += I[((m * NB + n) * NC + l) * ND + s] * dbd[n * ND + s];
                row_add<MODE>(FI + m * RS, W, fa + m, fc + l, N, fc + l - cb, ckg * v);
            }
    }
    {   // K: W_bd -= ck g sum I D_ac
        double dac[NA * NC];
#pragma unroll
        for (int m = 0; m < NA; ++m)
#pragma unroll
            for (int l = 0; l < NC; ++l) dac[m * NC + l] = D[(size_t)(fa + m) * N + fc + l];
#pragma unroll
        for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int s = 0; s < ND; ++s) {
                double v = 0.0;
#pragma unroll
                for (int m = 0; m < NA; ++m)
#pragma unroll
                    for (int l = 0; l < NC; ++l) v += I[((m * NB + n) * NC + l) * ND + s] * dac[m * NC + l];
                row_add<MODE>(FJ + n * RS, W, fb + n, fd + s, N, fd + s - db, ckg * v);
            }
    }
    {   // K: W_ad -= ck g sum I D_bc
        double dbc[NB * NC];
#pragma unroll
        for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int l = 0; l < NC; ++l) dbc[n * NC + l] = D[(size_t)(fb + n) * N + fc + l];
#pragma unroll
        for (int m = 0; m < NA; ++m)
#pragma unroll
            for (int s = 0; s < ND; ++s) {
                double v = 0.0;
#pragma unroll
                for (int n = 0; n < NB; ++n)
#pragma unroll
                    for (int l = 0; l < NC; ++l) v += I[((m * NB + n) * NC + l) * ND + s] * dbc[n * NC + l];
                row_add<MODE>(FI + m * RS, W, fa + m, fd + s, N, fd + s - db, ckg * v);
            }
    }
    {   // K: W_bc -= ck g sum I D_ad
        double dad[NA * ND];
#pragma unroll
        for (int m = 0; m < NA; ++m)
#pragma unroll
            for (int s = 0; s < ND; ++s) dad[m * ND + s] = D[(size_t)(fa + m) * N + fd + s];
#pragma unroll
        for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int l = 0; l < NC; ++l) {
                double v = 0.0;
#pragma unroll
                for (int m = 0; m < NA; ++m)
#pragma unroll
                    for (int s = 0; s < ND; ++s) v += I[((m * NB + n) * NC + l) * ND + s] * dad[m * ND + s];
                row_add<MODE>(FJ + n * RS, W, fb + n, fc + l, N, fc + l - cb, ckg * v);
            }
    }
}

// Same updates with rolled loops, for classes whose integral block is too
// large to keep in registers (the block then lives in scratch).
template <int NA, int NB, int NC, int ND, int MODE>
__device__ __forceinline__ void digest_rolled(const double* I, double g, const ClassArgs& a, const PairInfo& bra,
                                              int fc, int fd, int spos, const double* dab, double* jab,
                                              double* FI, double* FJ, const double* __restrict__ D,
                                              double* W, int N, int RS, int cb, int db,
                                              const double* __restrict__ dket, double* WK, double* wket) {
    const int fa = bra.bfa, fb = bra.bfb;
    const double cj2 = 2.0 * a.cj * g, ckg = -a.ck * g;
    (void)wket;   // the ket block's J goes straight into W (rolled digestion)
#pragma unroll 1
    for (int mn = 0; mn < NA * NB; ++mn) {
        double v = 0.0;
#pragma unroll 1
        for (int ls = 0; ls < NC * ND; ++ls) v += I[mn * NC * ND + ls] * dket[(size_t)ls * a.nket_list + spos];
        jab[mn] += g * v;
    }
#pragma unroll 1
    for (int ls = 0; ls < NC * ND; ++ls) {
        double v = 0.0;
#pragma unroll 1
        for (int mn = 0; mn < NA * NB; ++mn) v += I[mn * NC * ND + ls] * dab[mn];
        atomicAdd(W + (size_t)(fc + ls / ND) * N + fd + ls % ND, cj2 * v);
    }
#pragma unroll 1
    for (int m = 0; m < NA; ++m)
#pragma unroll 1
        for (int l = 0; l < NC; ++l) {
            double v1 = 0.0;
#pragma unroll 1
            for (int n = 0; n < NB; ++n)
#pragma unroll 1
                for (int s = 0; s < ND; ++s)
                    v1 += I[((m * NB + n) * NC + l) * ND + s] * D[(size_t)(fb + n) * N + fd + s];
            row_add<MODE>(FI + m * RS, WK, fa + m, fc + l, N, fc + l - cb, ckg * v1);
        }
#pragma unroll 1
    for (int n = 0; n < NB; ++n)
#pragma unroll 1
        for (int s = 0; s < ND; ++s) {
            double v2 = 0.0;
#pragma unroll 1
            for (int m = 0; m < NA; ++m)
#pragma unroll 1
                for (int l = 0; l < NC; ++l)
                    v2 += I[((m * NB + n) * NC + l) * ND + s] * D[(size_t)(fa + m) * N + fc + l];
            row_add<MODE>(FJ + n * RS, WK, fb + n, fd + s, N, fd + s - db, ckg * v2);
        }
#pragma unroll 1
    for (int m = 0; m < NA; ++m)
#pragma unroll 1
        for (int s = 0; s < ND; ++s) {
            double v3 = 0.0;
#pragma unroll 1
            for (int n = 0; n < NB; ++n)
#pragma unroll 1
                for (int l = 0; l < NC; ++l)
                    v3 += I[((m * NB + n) * NC + l) * ND + s] * D[(size_t)(fb + n) * N + fc + l];
            row_add<MODE>(FI + m * RS, WK, fa + m, fd + s, N, fd + s - db, ckg * v3);
        }
#pragma unroll 1
    for (int n = 0; n < NB; ++n)
#pragma unroll 1
        for (int l = 0; l < NC; ++l) {
            double v4 = 0.0;
#pragma unroll 1
            for (int m = 0; m < NA; ++m)
#pragma unroll 1
                for (int s = 0; s < ND; ++s)
                    v4 += I[((m * NB + n) * NC + l) * ND + s] * D[(size_t)(fa + m) * N + fd + s];
            row_add<MODE>(FJ + n * RS, WK, fb + n, fc + l, N, fc + l - cb, ckg * v4);
        }
}

// Digestion of one pass of a large class: the integrals (a_k b | c d) of the
// k-th Cartesian component of shell a, all b, c, d (I laid out [b][c][d]).
// Same updates as digest(), restricted to mu = k; rolled loops (the block
// lives in scratch, 8 NB NC ND bytes per lane).
template <int NA, int NB, int NC, int ND, int MODE>
__device__ __forceinline__ void digest_pass(int k, const double* I, double g, const ClassArgs& a,
                                            const PairInfo& bra, int fc, int fd, int spos, const double* dab,
                                            double* jab, double* FI, double* FJ, const double* __restrict__ D,
                                            double* W, int N, int RS, int cb, int db,
                                            const double* __restrict__ dket, double* WK, double* wket) {
    const int fa = bra.bfa, fb = bra.bfb;
    const double cj2 = 2.0 * a.cj * g, ckg = -a.ck * g;
    constexpr int NCD = NC * ND;
#pragma unroll 1
    for (int n = 0; n < NB; ++n) {   // J, bra block (mu = k)
        double v = 0.0;
#pragma unroll 1
        for (int ls = 0; ls < NCD; ++ls) v += I[n * NCD + ls] * dket[(size_t)ls * a.nket_list + spos];
        jab[k * NB + n] += g * v;
    }
#pragma unroll 1
    for (int ls = 0; ls < NCD; ++ls) {   // J, ket block
        double v = 0.0;
#pragma unroll 1
        for (int n = 0; n < NB; ++n) v += I[n * NCD + ls] * dab[k * NB + n];
        if constexpr (MODE == 0)
            atomicAdd(wket + (size_t)ls * a.nket_list + spos, cj2 * v);
        else
            atomicAdd(W + (size_t)(fc + ls / ND) * N + fd + ls % ND, cj2 * v);
    }
#pragma unroll 1
    for (int l = 0; l < NC; ++l) {   // K: (k, c_l) -= sum_{n s} I D_bd
        double v = 0.0;
#pragma unroll 1
        for (int n = 0; n < NB; ++n)
#pragma unroll 1
            for (int s = 0; s < ND; ++s) v += I[(n * NC + l) * ND + s] * D[(size_t)(fb + n) * N + fd + s];
        row_add<MODE>(FI + k * RS, WK, fa + k, fc + l, N, fc + l - cb, ckg * v);
    }
#pragma unroll 1
    for (int s = 0; s < ND; ++s) {   // K: (k, d_s) -= sum_{n l} I D_bc
        double v = 0.0;
#pragma unroll 1
        for (int n = 0; n < NB; ++n)
#pragma unroll 1
            for (int l = 0; l < NC; ++l) v += I[(n * NC + l) * ND + s] * D[(size_t)(fb + n) * N + fc + l];
        row_add<MODE>(FI + k * RS, WK, fa + k, fd + s, N, fd + s - db, ckg * v);
    }
#pragma unroll 1
    for (int n = 0; n < NB; ++n) {
#pragma unroll 1
        for (int s = 0; s < ND; ++s) {   // K: (b_n, d_s) -= sum_l I D_ac
            double v = 0.0;
#pragma unroll 1
            for (int l = 0; l < NC; ++l) v += I[(n * NC + l) * ND + s] * D[(size_t)(fa + k) * N + fc + l];
            row_add<MODE>(FJ + n * RS, WK, fb + n, fd + s, N, fd + s - db, ckg * v);
        }
#pragma unroll 1
        for (int l = 0; l < NC; ++l) {   // K: (b_n, c_l) -= sum_s I D_ad
            double v = 0.0;
#pragma unroll 1
            for (int s = 0; s < ND; ++s) v += I[(n * NC + l) * ND + s] * D[(size_t)(fa + k) * N + fd + s];
            row_add<MODE>(FJ + n * RS, WK, fb + n, fc + l, N, fc + l - cb, ckg * v);
        }
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// A wave's evaluated-quartet counts (per-lane running counts) into the
// class's counter slot of this workgroup.  All lanes of the wave call it.
__device__ __forceinline__ void flush_counts(const ClassArgs& a, unsigned c64, unsigned c32) {
    const unsigned long long s64 = (unsigned long long)wave_sum((double)c64);
    const unsigned long long s32 = (unsigned long long)wave_sum((double)c32);
    if ((threadIdx.x & 63) == 0 && a.counters) {
        const int slot = (int)(blockIdx.x % HFX_CNT_SLOTS);
        if (s64) atomicAdd(a.counters + slot * HFX_CNT_STRIDE, s64);
        if (s32) atomicAdd(a.counters + (HFX_CNT_SLOTS + slot) * HFX_CNT_STRIDE, s32);
    }
}

// One class, one digestion mode, one precision scheme (FP32 = 0: FP64
// evaluation; FP32 = 1, a mixed build: every task's kets below split[task]
// in FP64, the rest, a suffix of its Q-sorted range, in FP32 widened to FP64
// before digestion, both in the same launch and into the same LDS rows).
//
// LDS of a class kernel: the class's FP64 Boys rows (padded rows,
// BOYS_LROW64 apart; the FP32 evaluation rounds their coefficients), then
// (MODE 0) the bra rows F_I, F_J of the current task.
template <class E>
struct LdsLayout {
    static constexpr int L = E::LA + E::LB + E::LC + E::LD;
    static constexpr int ROWS = BOYS_NT * BOYS_LROW64;   // offset of the bra rows, doubles
};

// Uniform per workgroup: padding tasks (XCD striping) and other shards' bras do nothing.
__device__ __forceinline__ bool task_active(const ClassArgs& a, const int4 task) {
    return task.x >= 0 && (a.nshards <= 1 || task.x % a.nshards == a.shard);
}

template <class E>
__device__ __forceinline__ void load_boys_lds(const ClassArgs& a, double* t64) {
    using LL = LdsLayout<E>;
    const double* __restrict__ g64 = a.boys64 + (size_t)boys_block(LL::L) * BOYS_NT * BOYS_ROW;
    for (int i = threadIdx.x; i < boys_entries(); i += E::WGS)
        t64[(i / BOYS_ROW) * BOYS_LROW64 + i % BOYS_ROW] = g64[i];
    for (int k = threadIdx.x; k < BOYS_NT; k += E::WGS) t64[k * BOYS_LROW64 + BOYS_EXP_SLOT] = a.boys64[BOYS_EXP_OFF + k];
    __syncthreads();
}

// LDS ordering point of the lanes that run one task: the workgroup, or (WAVE)
// the single wave, whose LDS operations are processed in order.
template <bool WAVE>
__device__ __forceinline__ void task_sync() {
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    } else {
        __syncthreads();
    }
}

// One task (one bra, a range of its kets) on the lanes of the workgroup or
// (WAVE) of one wave, whose bra rows are the wave's own LDS region.
// Evaluated quartets go to the lane's running counts cnt64 / cnt32.
// DST: the bra's D' rows staged in LDS for the LDS digestion (bit 0 shell
// a's, bit 1 shell b's), a kernel variant of the classes with small blocks.
template <class E, int MODE, int FP32, bool WAVE = false, int DST = 0>
__device__ __forceinline__ void class_task(const ClassArgs& a, const int ti, const double* t64, unsigned& cnt64,
                                           unsigned& cnt32) {
    static_assert(!(FP32 && E::PASSES), "classes evaluated in passes are FP64 only");
    constexpr int NA = hfx_ncart(E::LA), NB = hfx_ncart(E::LB), NC = hfx_ncart(E::LC), ND = hfx_ncart(E::LD);
    constexpr int NAB = NA * NB, NI = NA * NB * NC * ND;
    constexpr int NT = WAVE ? 64 : E::WGS;   // lanes of the task
    const int tid = WAVE ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
    extern __shared__ __align__(16) double lds[];
    const int4 task = a.tasks[ti];
    const int r = task.x;
    if (!task_active(a, task)) return;
    // kets [s0, send) of the list: [s0, split) in FP64, [split, send) in FP32
    const int s0 = task.y, send = task.z;
    const int split = FP32 ? min(max(a.split[ti], s0), send) : send;
    const PairInfo bra = a.bra[r];
    // the bra's molecule: its blocks of D' and W, leading dimension ld
    const int N = bra.ld;
    const double* __restrict__ Dm = a.D + a.moff[bra.mol];
    // private digestion: this XCD's own copy of W (algorithm 2's private
    // Fock matrix, one per XCD instead of one per thread)
    double* __restrict__ Wm = a.W + a.moff[bra.mol] + (a.wrep ? (size_t)hfx_xcc_id() * a.wrep : 0);
    // LDS bra rows of length RS: whole rows, or (column windows) the task's
    // window of shell c at [0, RS/2) and of shell d at [RS/2, RS) (one region
    // when both windows coincide); column col sits at col - cb (c) / col - db (d)
    int RS = N, cb = 0, db = 0, half = N;
    if (a.win) {
        RS = a.rs;
        half = RS / 2;
        const int wc = task.w & 0xffff, wd = task.w >> 16;
        cb = wc * a.win;
        db = wd == wc ? cb : wd * a.win - half;
    }
    // LDS digestion with staged D' rows: DI, the bra's rows of shell a (DST
    // bit 0), then DJ, those of shell b (bit 1), after F_I and F_J
    static_assert(DST == 0 || (MODE == 0 && NI <= HFX_STAGE_D_MAX_NI && !E::PASSES), "no staged D' rows");
    constexpr int nda = (DST & 1) ? NA : 0, ndb = (DST & 2) ? NB : 0;
    // a wave's region is (NA + NB + nda + ndb) a.rs doubles (a.rs >= RS for every molecule of a batch)
    double* FI = lds + LdsLayout<E>::ROWS + (WAVE ? (int)(threadIdx.x >> 6) * (NA + NB + nda + ndb) * a.rs : 0);
    double* FJ = FI + NA * RS;
    double* DI = FJ + NB * RS;
    double* DJ = DI + nda * RS;
    if constexpr (MODE == 0) {
        for (int i = tid; i < (NA + NB) * RS; i += NT) FI[i] = 0.0;
        // staged rows over the same columns as F_I / F_J (zero past the molecule's last column)
        for (int i = tid; i < (nda + ndb) * RS; i += NT) {
            const bool ra = i < nda * RS;
            const int ii = ra ? i : i - nda * RS;
            const int row = (ra ? bra.bfa : bra.bfb) + ii / RS;
            const int lc = ii % RS;
            const int col = lc + (lc < half ? cb : db);
            DI[i] = col < N ? Dm[(size_t)row * N + col] : 0.0;
        }
        task_sync<WAVE>();
    }
    double dab[NAB], jab[NAB];
#pragma unroll
    for (int m = 0; m < NA; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            dab[m * NB + n] = Dm[(size_t)(bra.bfa + m) * N + bra.bfb + n];
            jab[m * NB + n] = 0.0;
        }
    const double sbra = bra.a != bra.b ? 2.0 : 1.0;
    const int kps = a.nket_list, kfs = a.nket_list * a.knprim;
    unsigned n64 = 0, n32 = 0;
    if constexpr (E::PASSES) {
        // one Cartesian component of shell a per pass, and the passes of a
        // quartet on different lanes: work item it = k * nq + (s - s0), so a
        // short task (few kets) still fills NA times as many lanes, and the
        // lanes of a wave share k
        const int nq = send - s0;
        for (int it = tid; it < NA * nq; it += NT) {
            const int k = it / nq, s = s0 + it % nq;
            const int4 kb = a.kbf[s];
            const double g = sbra * (kb.z != kb.w ? 2.0 : 1.0) * ((kb.z == bra.a && kb.w == bra.b) ? 1.0 : 2.0);
            double Ik[NB * NC * ND];
            E::template run_pass<double, BOYS_LROW64>(k, (const double*)(a.prim + bra.prim_off), bra.nprim,
                                                      a.kprim + s, kfs, kps, a.knprim, bra.AB, a.ket[s].AB, t64, Ik);
            digest_pass<NA, NB, NC, ND, MODE>(k, Ik, g, a, bra, kb.x, kb.y, s, dab, jab, FI, FJ, Dm, Wm, N, RS, cb,
                                              db, a.dket, Wm, a.wket);
            if (k == 0) ++n64;
        }
    }
    // The task's kets in slots of 64 consecutive kets, dealt to the task's
    // waves in turn (wave w takes slots w, w + nw, ...): the FP64 part
    // [s0, split) fills the first slots and the FP32 part [split, send) the
    // rest, so every slot is uniform in precision and the two parts cost at
    // most one partial slot more than one part (a per-lane choice, or one
    // loop per part over the whole workgroup, costs a full workgroup
    // iteration per task, which short tasks cannot hide).  With one part this
    // is the plain interleaving s = s0 + tid + i NT.
    const int nw = NT / 64, wv = tid >> 6, ln = tid & 63;
    const int slots64 = (split - s0 + 63) >> 6;
    const int slots = slots64 + ((send - split + 63) >> 6);
    for (int j = wv; j < slots && !E::PASSES; j += nw) {
        const bool lo = j < slots64;   // wave-uniform
        const int s = lo ? s0 + (j << 6) + ln : split + ((j - slots64) << 6) + ln;
        if (s >= (lo ? split : send)) continue;   // the part's last, partial slot
        double I[NI];
        if (!FP32 || lo) {
            E::template run<double, BOYS_LROW64>((const double*)(a.prim + bra.prim_off), bra.nprim, a.kprim + s,
                                                 kfs, kps, a.knprim, bra.AB, a.ket[s].AB, t64, I);
            ++n64;
        } else if constexpr (FP32) {
            // FP32 primitive copies, the FP64 Boys rows rounded
            float If[NI];
            E::template run<float, BOYS_LROW64>(a.prim32 + (size_t)bra.prim_off * HFX_PRIM_FIELDS, bra.nprim,
                                                a.kprim32 + s, kfs, kps, a.knprim, bra.AB, a.ket[s].AB, t64, If);
#pragma unroll
            for (int i = 0; i < NI; ++i) I[i] = (double)If[i];
            ++n32;
        }
        // the block (either precision) digested in FP64
        const int4 kb = a.kbf[s];   // ket's first basis functions and shells
        const double g = sbra * (kb.z != kb.w ? 2.0 : 1.0) * ((kb.z == bra.a && kb.w == bra.b) ? 1.0 : 2.0);
        if constexpr (NI >= HFX_ROLLED_DIGEST_MIN)
            digest_rolled<NA, NB, NC, ND, MODE>(I, g, a, bra, kb.x, kb.y, s, dab, jab, FI, FJ, Dm, Wm, N, RS, cb, db,
                                                a.dket, Wm, a.wket);
        else
            digest<NA, NB, NC, ND, MODE, DST>(I, g, a, bra, kb.x, kb.y, s, dab, jab, FI, FJ, Dm, Wm, N, RS, cb, db,
                                              a.dket, Wm, a.wket, DI, DJ);
    }
    // bra J block: wave reduction, one global add per wave (column bfb may lie
    // outside the task's windows)
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int mn = 0; mn < NAB; ++mn) {
        const double v = wave_sum(jab[mn]);
        if (lane == 0) {
            const int m = mn / NB, n = mn % NB;
            atomicAdd(Wm + (size_t)(bra.bfa + m) * N + bra.bfb + n, 2.0 * a.cj * v);
        }
    }
    cnt64 += n64;
    cnt32 += n32;
    if constexpr (MODE == 0) {
        task_sync<WAVE>();
        for (int i = tid; i < (NA + NB) * RS; i += NT) {
            const double v = FI[i];
            if (v != 0.0) {
                const int row = i < NA * RS ? bra.bfa + i / RS : bra.bfb + (i - NA * RS) / RS;
                const int lc = i < NA * RS ? i % RS : (i - NA * RS) % RS;
                const int col = lc + (lc < half ? cb : db);
                if (col < N) atomicAdd(Wm + (size_t)row * N + col, v);
            }
        }
    }
}

// Register-tiled task: a block of nb <= NBL consecutive bras of the class's
// Q-sorted list (one molecule) against one range of kets whose primitive
// count KP is a compile-time constant.  Each lane takes kets of the range; a
// ket's primitives, D'_cd and record are read once into registers and
// serve every bra of the block, whose screened prefixes differ: bra r takes
// ket s iff Q_r Q_s >= tau (and, for bra and ket of one pair class, the ket's
// class position <= r), the same test that sizes the plan's prefixes.  The
// ket block's J sum over the block goes out in one atomic per component; each
// bra has its own LDS rows F_I, F_J (MODE 0).  FP64 only.
template <class E, int MODE, int KP, int NBL>
__device__ __forceinline__ void class_task_kr(const ClassArgs& a, const int ti, const double* t64, unsigned& cnt64) {
    constexpr int NA = hfx_ncart(E::LA), NB = hfx_ncart(E::LB), NC = hfx_ncart(E::LC), ND = hfx_ncart(E::LD);
    constexpr int NAB = NA * NB, NCD = NC * ND, NI = NAB * NCD;
    constexpr int NT = E::WGS;
    const int tid = (int)threadIdx.x;
    extern __shared__ __align__(16) double lds[];
    const int4 task = a.tasks[ti];
    if (task.x < 0) return;
    const int r0 = task.x & 0x0fffffff;
    const int nb = (task.x >> 28) + 1;
    const int s0 = task.y, send = task.z;
    PairInfo bra[NBL];
    bool on[NBL];
#pragma unroll
    for (int i = 0; i < NBL; ++i) {
        on[i] = i < nb && (a.nshards <= 1 || (r0 + i) % a.nshards == a.shard);
        bra[i] = a.bra[r0 + (i < nb ? i : 0)];
    }
    bool any = false;
#pragma unroll
    for (int i = 0; i < NBL; ++i) any |= on[i];
    if (!any) return;   // uniform: another shard's block
    // the block's molecule (shared by its bras): blocks of D', W, leading dimension
    const int N = bra[0].ld;
    const double* __restrict__ Dm = a.D + a.moff[bra[0].mol];
    double* __restrict__ Wm = a.W + a.moff[bra[0].mol] + (a.wrep ? (size_t)hfx_xcc_id() * a.wrep : 0);
    int RS = N, cb = 0, db = 0, half = N;
    if (a.win) {
        RS = a.rs;
        half = RS / 2;
        const int wc = task.w & 0xffff, wd = task.w >> 16;
        cb = wc * a.win;
        db = wd == wc ? cb : wd * a.win - half;
    }
    constexpr int ROWS = (NA + NB);
    double* F0 = lds + LdsLayout<E>::ROWS;   // bra i's rows at F0 + i ROWS a.rs
    if constexpr (MODE == 0) {
        for (int i = tid; i < nb * ROWS * a.rs; i += NT) F0[i] = 0.0;
        __syncthreads();
    }
    double dab[NBL][NAB], jab[NBL][NAB], sbra[NBL];
#pragma unroll
    for (int i = 0; i < NBL; ++i) {
        sbra[i] = bra[i].a != bra[i].b ? 2.0 : 1.0;
#pragma unroll
        for (int m = 0; m < NA; ++m)
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                dab[i][m * NB + n] = Dm[(size_t)(bra[i].bfa + m) * N + bra[i].bfb + n];
                jab[i][m * NB + n] = 0.0;
            }
    }
    const int nl = a.nket_list;
    unsigned n64 = 0;
    for (int s = s0 + tid; s < send; s += NT) {
        const int4 kb = a.kbf[s];
        const int fc = kb.x, fd = kb.y;
        double kv[KP][9];
#pragma unroll
        for (int k = 0; k < KP; ++k)
#pragma unroll
            for (int f = 0; f < 9; ++f) kv[k][f] = a.kprim[(size_t)(f * KP + k) * nl + s];
        double dcd[NCD], jcd[NCD];
#pragma unroll
        for (int ls = 0; ls < NCD; ++ls) {
            dcd[ls] = a.dket[(size_t)ls * nl + s];
            jcd[ls] = 0.0;
        }
        const double qs = a.ketq[s];
        const int ks = a.same ? a.kpos[s] : 0;
        const double* kab = a.ket[s].AB;   // read only by classes with a p or d ket
        const double gk = kb.z != kb.w ? 2.0 : 1.0;
        bool hit = false;
#pragma unroll
        for (int i = 0; i < NBL; ++i) {
            if (!on[i]) continue;
            if (!(qs * bra[i].Q >= a.tau) || ks > r0 + i) continue;
            const double g = sbra[i] * gk * ((kb.z == bra[i].a && kb.w == bra[i].b) ? 1.0 : 2.0);
            double I[NI];
            E::template run_kr<double, BOYS_LROW64, KP>(a.prim + bra[i].prim_off, bra[i].nprim, kv, bra[i].AB, kab,
                                                        t64, I);
            ++n64;
            hit = true;
            double* FI = F0 + i * ROWS * a.rs;
            digest_kr<NA, NB, NC, ND, MODE>(I, g, a.ck, bra[i], fc, fd, dcd, dab[i], jab[i], jcd, FI, FI + NA * RS,
                                            Dm, Wm, N, RS, cb, db);
        }
        if (hit) {
            const double cj2 = 2.0 * a.cj;
#pragma unroll
            for (int l = 0; l < NC; ++l)
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    if constexpr (MODE == 0)
                        atomicAdd(a.wket + (size_t)(l * ND + d) * nl + s, cj2 * jcd[l * ND + d]);
                    else
                        atomicAdd(Wm + (size_t)(fc + l) * N + fd + d, cj2 * jcd[l * ND + d]);
                }
        }
    }
    const int lane = tid & 63;
#pragma unroll
    for (int i = 0; i < NBL; ++i) {
        if (!on[i]) continue;
#pragma unroll
        for (int mn = 0; mn < NAB; ++mn) {
            const double v = wave_sum(jab[i][mn]);
            if (lane == 0) atomicAdd(Wm + (size_t)(bra[i].bfa + mn / NB) * N + bra[i].bfb + mn % NB, 2.0 * a.cj * v);
        }
    }
    cnt64 += n64;
    if constexpr (MODE == 0) {
        __syncthreads();
        for (int i = tid; i < nb * ROWS * a.rs; i += NT) {
            const double v = F0[i];
            if (v != 0.0) {
                const int bi = i / (ROWS * a.rs), j = i - bi * ROWS * a.rs;
                int bfa = bra[0].bfa, bfb = bra[0].bfb;
#pragma unroll
                for (int k = 1; k < NBL; ++k)
                    if (bi == k) {
                        bfa = bra[k].bfa;
                        bfb = bra[k].bfb;
                    }
                const int row = j < NA * RS ? bfa + j / RS : bfb + (j - NA * RS) / RS;
                const int lc = j < NA * RS ? j % RS : (j - NA * RS) % RS;
                const int col = lc + (lc < half ? cb : db);
                if (col < N) atomicAdd(Wm + (size_t)row * N + col, v);
            }
        }
    }
}

// Persistent register-tiled launch (same queues as k_class_persist).
template <class E, int MODE, int KP, int NBL>
__global__ __launch_bounds__(E::WGS) void k_class_kr(const ClassArgs a) {
    extern __shared__ __align__(16) double lds[];
    __shared__ int next_entry;
    double* t64 = lds;
    load_boys_lds<E>(a, t64);
    unsigned cnt64 = 0;
    const int x0 = blockIdx.x & 7;
    for (int q = 0; q < 8;) {
        const int x = (x0 + q) & 7;
        if (threadIdx.x == 0) next_entry = (int)atomicAdd(a.work + x, 1ull);
        __syncthreads();
        const int k = next_entry;
        __syncthreads();
        if (k >= a.qlen) {
            ++q;
            continue;
        }
        class_task_kr<E, MODE, KP, NBL>(a, 8 * k + x, t64, cnt64);
    }
    flush_counts(a, cnt64, 0);
}

// Several densities in one pass over the integrals (FP64): every quartet of
// the task is evaluated once and digested for each density d < a.ndens
// (D'_d, its gathered D'_cd, its J and K accumulators and its ket-block J
// accumulator at offsets d dstride / d kstride), the J updates into a.W (the
// ket block's via a.wket in MODE 0) and the K updates into a.WK.  MODE 0
// stages each density's bra rows of K in LDS (a.ndens row sets; the host
// groups the densities so that they fit), MODE 1 uses global atomics.  The
// bra block's J sums are reduced over each wave per ket iteration (all lanes
// of a wave iterate together).  Tasks may be blocks of bras (register-tiled
// plans): each bra keeps the kets of its own screened prefix, the test the
// planner used.
template <class E, int MODE>
__device__ __forceinline__ void class_task_multi(const ClassArgs& a, const int ti, const double* t64,
                                                 unsigned& cnt64) {
    constexpr int NA = hfx_ncart(E::LA), NB = hfx_ncart(E::LB), NC = hfx_ncart(E::LC), ND = hfx_ncart(E::LD);
    constexpr int NAB = NA * NB, NI = NAB * NC * ND;
    constexpr int NT = E::WGS;
    extern __shared__ __align__(16) double lds[];
    const int tid = (int)threadIdx.x, lane = tid & 63;
    const int4 task = a.tasks[ti];
    if (task.x < 0) return;
    const int r0 = task.x & 0x0fffffff, nb = (task.x >> 28) + 1;
    const int s0 = task.y, nq = task.z - task.y;
    const int nwork = E::PASSES ? NA * nq : nq;
    unsigned n64 = 0;
    for (int i = 0; i < nb; ++i) {
        const int r = r0 + i;
        if (a.nshards > 1 && r % a.nshards != a.shard) continue;   // uniform
        const PairInfo bra = a.bra[r];
        const int N = bra.ld;
        const size_t moff = (size_t)a.moff[bra.mol];
        const double sbra = bra.a != bra.b ? 2.0 : 1.0;
        // LDS rows of density d at F0 + d (NA + NB) a.rs, windows as in class_task
        int RS = N, cb = 0, db = 0, half = N;
        if (a.win) {
            RS = a.rs;
            half = RS / 2;
            const int wc = task.w & 0xffff, wd = task.w >> 16;
            cb = wc * a.win;
            db = wd == wc ? cb : wd * a.win - half;
        }
        double* F0 = lds + LdsLayout<E>::ROWS;
        const int rowset = (NA + NB) * a.rs;
        if constexpr (MODE == 0) {
            for (int x = tid; x < a.ndens * rowset; x += NT) F0[x] = 0.0;
            __syncthreads();
        }
        for (int base = 0; base < nwork; base += NT) {
            const int it = base + tid;
            bool valid = it < nwork;
            const int k = E::PASSES ? (valid ? it / nq : 0) : 0;
            const int s = s0 + (valid ? (E::PASSES ? it % nq : it) : 0);
            if (valid) valid = a.ketq[s] * bra.Q >= a.tau && !(a.same && a.kpos[s] > r);
            const int4 kb = a.kbf[s];
            const double g = sbra * (kb.z != kb.w ? 2.0 : 1.0) * ((kb.z == bra.a && kb.w == bra.b) ? 1.0 : 2.0);
            double I[E::PASSES ? NB * NC * ND : NI];
            if (valid) {
                const double* bp = (const double*)(a.prim + bra.prim_off);
                if constexpr (E::PASSES)
                    E::template run_pass<double, BOYS_LROW64>(k, bp, bra.nprim, a.kprim + s, a.nket_list * a.knprim,
                                                              a.nket_list, a.knprim, bra.AB, a.ket[s].AB, t64, I);
                else
                    E::template run<double, BOYS_LROW64>(bp, bra.nprim, a.kprim + s, a.nket_list * a.knprim,
                                                         a.nket_list, a.knprim, bra.AB, a.ket[s].AB, t64, I);
                if (k == 0) ++n64;
            }
            for (int d = 0; d < a.ndens; ++d) {
                const double* __restrict__ Dd = a.D + (size_t)d * a.dstride + moff;
                double* WJ = a.W + (size_t)d * a.dstride + moff;
                double* WKd = a.WK + (size_t)d * a.dstride + moff;
                const double* dket = a.dket + (size_t)d * a.kstride;
                double* wket = a.wket + (size_t)d * a.kstride;
                double* FI = F0 + d * rowset;
                double dab[NAB], jt[NAB];
#pragma unroll
                for (int mn = 0; mn < NAB; ++mn) {
                    dab[mn] = Dd[(size_t)(bra.bfa + mn / NB) * N + bra.bfb + mn % NB];
                    jt[mn] = 0.0;
                }
                if (valid) {
                    if constexpr (E::PASSES)
                        digest_pass<NA, NB, NC, ND, MODE>(k, I, g, a, bra, kb.x, kb.y, s, dab, jt, FI, FI + NA * RS,
                                                          Dd, WJ, N, RS, cb, db, dket, WKd, wket);
                    else if constexpr (NI >= HFX_ROLLED_DIGEST_MIN)
                        digest_rolled<NA, NB, NC, ND, MODE>(I, g, a, bra, kb.x, kb.y, s, dab, jt, FI, FI + NA * RS,
                                                            Dd, WJ, N, RS, cb, db, dket, WKd, wket);
                    else
                        digest<NA, NB, NC, ND, MODE>(I, g, a, bra, kb.x, kb.y, s, dab, jt, FI, FI + NA * RS, Dd, WJ,
                                                     N, RS, cb, db, dket, WKd, wket);
                }
#pragma unroll
                for (int mn = 0; mn < NAB; ++mn) {
                    const double v = wave_sum(jt[mn]);
                    if (lane == 0 && v != 0.0)
                        atomicAdd(WJ + (size_t)(bra.bfa + mn / NB) * N + bra.bfb + mn % NB, 2.0 * a.cj * v);
                }
            }
        }
        if constexpr (MODE == 0) {   // each density's K rows into its K accumulator
            __syncthreads();
            for (int x = tid; x < a.ndens * rowset; x += NT) {
                const double v = F0[x];
                if (v != 0.0) {
                    const int d = x / rowset, j = x - d * rowset;
                    const int row = j < NA * RS ? bra.bfa + j / RS : bra.bfb + (j - NA * RS) / RS;
                    const int lc = j < NA * RS ? j % RS : (j - NA * RS) % RS;
                    const int col = lc + (lc < half ? cb : db);
                    if (col < N && j < (NA + NB) * RS)
                        atomicAdd(a.WK + (size_t)d * a.dstride + moff + (size_t)row * N + col, v);
                }
            }
            __syncthreads();
        }
    }
    cnt64 += n64;
}

template <class E, int MODE>
__global__ __launch_bounds__(E::WGS) void k_class_multi(const ClassArgs a) {
    extern __shared__ __align__(16) double lds[];
    __shared__ int next_entry;
    load_boys_lds<E>(a, lds);
    unsigned cnt64 = 0;
    const int x0 = blockIdx.x & 7;
    for (int q = 0; q < 8;) {
        const int x = (x0 + q) & 7;
        if (threadIdx.x == 0) next_entry = (int)atomicAdd(a.work + x, 1ull);
        __syncthreads();
        const int k = next_entry;
        __syncthreads();
        if (k >= a.qlen) {
            ++q;
            continue;
        }
        class_task_multi<E, MODE>(a, 8 * k + x, lds, cnt64);
    }
    flush_counts(a, cnt64, 0);
}

// Static launch: workgroup i runs task task_off + i (a plan's tasks may span
// several launches: a grid is limited to 2^32 work-items).
template <class E, int MODE, int FP32, int DST = 0>
__global__ __launch_bounds__(E::WGS) void k_class(const ClassArgs a) {
    extern __shared__ __align__(16) double lds[];
    __shared__ unsigned long long wg_count[2];   // the workgroup's counts: one global add each
    const int ti = a.task_off + (int)blockIdx.x;
    const int4 task = a.tasks[ti];
    if (!task_active(a, task)) return;
    if (threadIdx.x == 0) wg_count[0] = wg_count[1] = 0;
    load_boys_lds<E>(a, lds);   // ends with a barrier
    unsigned cnt64 = 0, cnt32 = 0;
    class_task<E, MODE, FP32, false, DST>(a, ti, lds, cnt64, cnt32);
    const unsigned long long s64 = (unsigned long long)wave_sum((double)cnt64);
    const unsigned long long s32 = (unsigned long long)wave_sum((double)cnt32);
    if ((threadIdx.x & 63) == 0) {
        if (s64) atomicAdd(&wg_count[0], s64);
        if (s32) atomicAdd(&wg_count[1], s32);
    }
    __syncthreads();
    if (threadIdx.x == 0 && a.counters) {
        const int slot = (int)(blockIdx.x % HFX_CNT_SLOTS);
        if (wg_count[0]) atomicAdd(a.counters + slot * HFX_CNT_STRIDE, wg_count[0]);
        if (wg_count[1]) atomicAdd(a.counters + (HFX_CNT_SLOTS + slot) * HFX_CNT_STRIDE, wg_count[1]);
    }
}

// Persistent launch: a resident grid; a workgroup on XCD x (workgroup index
// mod 8, the hardware's round-robin placement) takes entries of XCD x's
// queue through an atomic counter, then drains the other queues in turn, so
// no XCD idles while another still has work (the dynamic load balancing of
// ddi_dlbnext in algorithms 1-3).  A separate kernel so that the static
// form keeps its register allocation.
template <class E, int MODE, int FP32, int DST = 0>
__global__ __launch_bounds__(E::WGS) void k_class_persist(const ClassArgs a) {
    extern __shared__ __align__(16) double lds[];
    __shared__ int next_entry;
    load_boys_lds<E>(a, lds);   // once per resident workgroup
    unsigned cnt64 = 0, cnt32 = 0;
    const int x0 = blockIdx.x & 7;
    for (int q = 0; q < 8;) {
        const int x = (x0 + q) & 7;
        if (threadIdx.x == 0) next_entry = (int)atomicAdd(a.work + x, 1ull);
        __syncthreads();
        const int k = next_entry;
        __syncthreads();
        if (k >= a.qlen) {
            ++q;
            continue;
        }
        class_task<E, MODE, FP32, false, DST>(a, 8 * k + x, lds, cnt64, cnt32);
    }
    flush_counts(a, cnt64, cnt32);
}

// Persistent launch with one task per wave: each wave of a resident
// workgroup takes its own queue entries (same queues and order as
// k_class_persist) and digests into its own LDS bra rows, so short tasks
// (small molecules of a batch) occupy 64 lanes instead of a workgroup.  The
// Boys rows are shared by the workgroup's waves.
template <class E, int MODE, int FP32, int DST = 0>
__global__ __launch_bounds__(E::WGS) void k_class_wave(const ClassArgs a) {
    extern __shared__ __align__(16) double lds[];
    load_boys_lds<E>(a, lds);
    unsigned cnt64 = 0, cnt32 = 0;
    const int x0 = blockIdx.x & 7;
    for (int q = 0; q < 8;) {
        const int x = (x0 + q) & 7;
        int k = 0;
        if ((threadIdx.x & 63) == 0) k = (int)atomicAdd(a.work + x, 1ull);
        k = __shfl(k, 0, 64);
        if (k >= a.qlen) {
            ++q;
            continue;
        }
        class_task<E, MODE, FP32, true, DST>(a, 8 * k + x, lds, cnt64, cnt32);
    }
    flush_counts(a, cnt64, cnt32);
}

// Schwarz bound of every pair of one pair class: Q = sqrt(max (mn|mn)) with
// the component normalisation s_m s_n applied (always FP64).
// 1/sqrt((2lx-1)!!(2ly-1)!!(2lz-1)!!) of Cartesian component c of shell l.
__device__ __forceinline__ double comp_scale(int l, int c) {
    return (l == 2 && (c == 0 || c == 3 || c == 5)) ? 0.57735026918962576451 : 1.0;
}

template <class E>
__global__ __launch_bounds__(HFX_WG) void k_schwarz(const PairInfo* __restrict__ pairs, int npairs,
                                                     const PrimPair* __restrict__ prim,
                                                     const double* __restrict__ boys, double* __restrict__ Q) {
    constexpr int NA = hfx_ncart(E::LA), NB = hfx_ncart(E::LB);
    const int i = blockIdx.x * HFX_WG + threadIdx.x;
    if (i >= npairs) return;
    const PairInfo pr = pairs[i];
    double I[NA * NB * NA * NB];
    // ket read from the array-of-structures layout: field stride 1, primitive stride 10 doubles
    E::template run<double>((const double*)(prim + pr.prim_off), pr.nprim, (const double*)(prim + pr.prim_off), 1,
                            (int)(sizeof(PrimPair) / sizeof(double)), pr.nprim, pr.AB, pr.AB,
                            boys + (size_t)boys_block(E::LA + E::LB + E::LC + E::LD) * BOYS_NT * BOYS_ROW, I);
    double mx = 0.0;
#pragma unroll
    for (int m = 0; m < NA; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const double s = comp_scale(E::LA, m) * comp_scale(E::LB, n);
            const double v = I[(m * NB + n) * NA * NB + m * NB + n] * s * s;
            mx = v > mx ? v : mx;
        }
    Q[i] = sqrt(mx);
}


// Kernel variants of one class: launch form x digestion mode x precision.
// Classes with integral blocks of HFX_ROLLED_DIGEST_MIN or more (d-d bra with
// a d-d or d-p ket) exist only in FP64: their register allocation is the
// build-time bottleneck and they carry a negligible share of the quartets,
// so mixed builds evaluate them in FP64 (the more accurate choice).
template <class E>
struct ClassKernelsOne {
    static constexpr int NI = hfx_ncart(E::LA) * hfx_ncart(E::LB) * hfx_ncart(E::LC) * hfx_ncart(E::LD);
    static constexpr bool kOnlyFp64Global = NI >= HFX_ROLLED_DIGEST_MIN;
    static constexpr bool kStage = NI <= HFX_STAGE_D_MAX_NI && !E::PASSES;
    // LDS digestion with staged D' rows (DST 1: shell a's, 3: both shells'):
    // form 0 static, 1 persistent, 2 one task per wave
    template <int DST>
    static const void* staged(int form, int mixed) {
        static const void* t[6] = {(const void*)k_class<E, 0, 0, DST>,         (const void*)k_class<E, 0, 1, DST>,
                                   (const void*)k_class_persist<E, 0, 0, DST>, (const void*)k_class_persist<E, 0, 1, DST>,
                                   (const void*)k_class_wave<E, 0, 0, DST>,    (const void*)k_class_wave<E, 0, 1, DST>};
        return t[2 * form + mixed];
    }
    // variant = 4 persistent + 2 mode + mixed (FP64 prefix and FP32 suffix of
    // every task); bit 4: one task per wave (persistent); bits 5-6: staged
    // D' rows (1: shell a's, 2: both shells'; LDS digestion only)
    static const void* get(int variant) {
        if (const int ds = (variant >> 5) & 3) {
            if constexpr (kStage) {
                if (variant & 2) return nullptr;
                const int form = (variant & 16) ? 2 : (variant & 4) ? 1 : 0;
                return ds == 1 ? staged<1>(form, variant & 1) : staged<3>(form, variant & 1);
            } else {
                return nullptr;
            }
        }
        if (variant & 16) {
            if constexpr (kOnlyFp64Global) {
                return (variant & 2) ? (const void*)k_class_wave<E, 1, 0> : (const void*)k_class_wave<E, 0, 0>;
            } else {
                static const void* w[4] = {(const void*)k_class_wave<E, 0, 0>, (const void*)k_class_wave<E, 0, 1>,
                                           (const void*)k_class_wave<E, 1, 0>, (const void*)k_class_wave<E, 1, 1>};
                return w[variant & 3];
            }
        }
        if constexpr (kOnlyFp64Global) {
            static const void* t[4] = {(const void*)k_class<E, 0, 0>, (const void*)k_class<E, 1, 0>,
                                       (const void*)k_class_persist<E, 0, 0>, (const void*)k_class_persist<E, 1, 0>};
            return t[(variant >= 4 ? 2 : 0) + ((variant & 3) >= 2 ? 1 : 0)];
        } else {
            static const void* t[8] = {(const void*)k_class<E, 0, 0>,         (const void*)k_class<E, 0, 1>,
                                       (const void*)k_class<E, 1, 0>,         (const void*)k_class<E, 1, 1>,
                                       (const void*)k_class_persist<E, 0, 0>, (const void*)k_class_persist<E, 0, 1>,
                                       (const void*)k_class_persist<E, 1, 0>, (const void*)k_class_persist<E, 1, 1>};
            return t[variant];
        }
    }
};

// variant bit 3: the class's alternative workgroup size (EA; the same kernels
// when EA has E's size); bit 4: one task per wave.
template <class E, class EA>
struct ClassKernels {
    static const void* get(int variant) {
        if constexpr (EA::WGS != E::WGS) {
            if (variant & 8) return ClassKernelsOne<EA>::get(variant & 119);
        }
        return ClassKernelsOne<E>::get(variant & 119);
    }
};

// Register-tiled kernels of one class: variant = mode + 2 kpi + 6 (NBL - 1),
// ket primitive count 1, 3 or 9 (kpi 0, 1, 2), blocks of 1 or 2 bras.
template <class E>
struct ClassKernelsKr {
    static const void* get(int v) {
        static const void* t[12] = {
            (const void*)k_class_kr<E, 0, 1, 1>, (const void*)k_class_kr<E, 1, 1, 1>,
            (const void*)k_class_kr<E, 0, 3, 1>, (const void*)k_class_kr<E, 1, 3, 1>,
            (const void*)k_class_kr<E, 0, 9, 1>, (const void*)k_class_kr<E, 1, 9, 1>,
            (const void*)k_class_kr<E, 0, 1, 2>, (const void*)k_class_kr<E, 1, 1, 2>,
            (const void*)k_class_kr<E, 0, 3, 2>, (const void*)k_class_kr<E, 1, 3, 2>,
            (const void*)k_class_kr<E, 0, 9, 2>, (const void*)k_class_kr<E, 1, 9, 2>};
        return (v >= 0 && v < 12) ? t[v] : nullptr;
    }
};

// Register-tiled kernels use the class's alternative (smaller) workgroup
// size: the ket primitives in registers need more than the 128 VGPRs a
// 1024-lane workgroup leaves each lane.
#define HFX_CLASS_KR(cid) \
    extern "C" const void* hfx_class_kernel_kr_##cid(int v) { return ClassKernelsKr<Eval##cid##A>::get(v); }
#define HFX_CLASS_NO_KR(cid) \
    extern "C" const void* hfx_class_kernel_kr_##cid(int) { return nullptr; }

// Per-class translation unit: evaluator wrapper, the kernel variants, the
// Schwarz kernel and C lookups.
#define HFX_CLASS_TU(cid, fname, la_, lb_, lc_, ld_, wgs_, wgs_alt_)                                               \
    struct Eval##cid {                                                                                 \
        static constexpr int LA = la_, LB = lb_, LC = lc_, LD = ld_, WGS = wgs_;                       \
        static constexpr bool PASSES = false;                                                          \
        template <typename R, int BS = BOYS_ROW, typename SP = double, typename TT = R>                \
        __device__ __forceinline__ static void run(const SP* bp, int nbp, const SP* kq0, int kfs,      \
                                                   int kps, int nkp, const double* ab,                 \
                                                   const double* cd, const TT* tab, R* out) {          \
            fname<R, BS, SP, TT>(bp, nbp, kq0, kfs, kps, nkp, R(ab[0]), R(ab[1]), R(ab[2]), R(cd[0]),  \
                                 R(cd[1]), R(cd[2]), tab, out);                                        \
        }                                                                                              \
        template <typename R, int BS, int KP>                                                          \
        __device__ __forceinline__ static void run_kr(const PrimPair* bp, int nbp,                     \
                                                      const R (&kv)[KP][9], const double* ab,          \
                                                      const double* cd, const R* tab, R* out) {        \
            fname##_kr<R, BS, KP>(bp, nbp, kv, R(ab[0]), R(ab[1]), R(ab[2]), R(cd[0]), R(cd[1]),       \
                                  R(cd[2]), tab, out);                                                 \
        }                                                                                              \
    };                                                                                                 \
    struct Eval##cid##A : Eval##cid {                                                                   \
        static constexpr int WGS = wgs_alt_;                                                           \
    };                                                                                                 \
    extern "C" const void* hfx_class_kernel_##cid(int variant) {                                       \
        return ClassKernels<Eval##cid, Eval##cid##A>::get(variant);                                    \
    }                                                                                                  \
    extern "C" const void* hfx_class_kernel_multi_##cid(int mode) {                                   \
        return mode ? (const void*)k_class_multi<Eval##cid, 1> : (const void*)k_class_multi<Eval##cid, 0>; \
    }                                                                                                  \
    extern "C" const void* hfx_schwarz_kernel_##cid(void) { return (const void*)k_schwarz<Eval##cid>; }

// Per-class translation unit of a large class: the full evaluator (Schwarz
// bounds) plus the per-component passes used by the class kernels.
#define HFX_CLASS_TU_PASSES(cid, fname, la_, lb_, lc_, ld_, wgs_, wgs_alt_)                                        \
    struct Eval##cid {                                                                                 \
        static constexpr int LA = la_, LB = lb_, LC = lc_, LD = ld_, WGS = wgs_;                       \
        static constexpr bool PASSES = true;                                                           \
        template <typename R, int BS = BOYS_ROW, typename SP = double, typename TT = R>                \
        __device__ __forceinline__ static void run(const SP* bp, int nbp, const SP* kq0, int kfs,      \
                                                   int kps, int nkp, const double* ab,                 \
                                                   const double* cd, const TT* tab, R* out) {          \
            fname<R, BS, SP, TT>(bp, nbp, kq0, kfs, kps, nkp, R(ab[0]), R(ab[1]), R(ab[2]), R(cd[0]),  \
                                 R(cd[1]), R(cd[2]), tab, out);                                        \
        }                                                                                              \
        template <typename R, int BS = BOYS_ROW>                                                       \
        __device__ __forceinline__ static void run_pass(int k, const double* bp, int nbp,              \
                                                        const double* kq0, int kfs, int kps, int nkp,  \
                                                        const double* ab, const double* cd,            \
                                                        const R* tab, R* out) {                        \
            fname##_pass<R, BS>(k, bp, nbp, kq0, kfs, kps, nkp, R(ab[0]), R(ab[1]), R(ab[2]),          \
                                R(cd[0]), R(cd[1]), R(cd[2]), tab, out);                               \
        }                                                                                              \
    };                                                                                                 \
    struct Eval##cid##A : Eval##cid {                                                                   \
        static constexpr int WGS = wgs_alt_;                                                           \
    };                                                                                                 \
    extern "C" const void* hfx_class_kernel_##cid(int variant) {                                       \
        return ClassKernels<Eval##cid, Eval##cid##A>::get(variant);                                    \
    }                                                                                                  \
    extern "C" const void* hfx_class_kernel_multi_##cid(int mode) {                                   \
        return mode ? (const void*)k_class_multi<Eval##cid, 1> : (const void*)k_class_multi<Eval##cid, 0>; \
    }                                                                                                  \
    extern "C" const void* hfx_schwarz_kernel_##cid(void) { return (const void*)k_schwarz<Eval##cid>; }
