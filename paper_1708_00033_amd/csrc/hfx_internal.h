// Internal data layout and device helpers of the HIP Fock-build library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// ---- shell-pair data in HBM ---------------------------------------------------
// One primitive pair (alpha on the pair's first shell A, beta on B) in the
// pair's canonical orientation (l_A >= l_B):
//   p = alpha + beta, inv2p = 1/(2p), P = (alpha A + beta B)/p, PA = P - A,
//   K = c_A c_B exp(-alpha beta/p |AB|^2) sqrt(2 pi^{5/2}) / p
// so that the quartet prefactor 2 pi^{5/2}/(p q sqrt(p+q)) K_ab K_cd is
// K_bra K_ket / sqrt(p+q).  80 bytes, read per lane from L2.
struct PrimPair {
    double p, inv2p;
    double P[3];
    double PA[3];
    double K;
    double pad;
};
#define HFX_PRIM_FIELDS 10   // elements of one PrimPair (an FP32 copy has the same layout in floats)
// LDS digestion with the bra's D' rows staged in LDS: classes with at most
// this many integrals per quartet (two more kernel variants per launch form)
#define HFX_STAGE_D_MAX_NI 64

// One shell pair in canonical orientation: shells a (higher l) and b, their
// first basis functions, its primitive pairs, its Schwarz bound and A - B.
struct PairInfo {
    int a, b;          // shells (global index)
    int bfa, bfb;      // first basis functions, local to the molecule
    int prim_off, nprim;
    double Q;
    double AB[3];
    int mol;           // molecule of a batch
    int ld;            // its basis size (leading dimension of its blocks)
};

// Arguments of one class kernel launch.  The kets of a launch all have the
// same number of primitive pairs (knprim), so the primitive loop trip count
// is uniform across a wave.  Ket primitive data are a structure of arrays:
// field f (the PrimPair member order p, inv2p, P[3], PA[3], K) of primitive k
// of ket s at kprim[(f * knprim + k) * nket_list + s].
struct ClassArgs {
    const PairInfo* __restrict__ bra;   // bra pairs of the class, Q descending
    const PairInfo* __restrict__ ket;   // ket pairs (one primitive count), Q descending
    const int4* __restrict__ kbf;       // per ket: first basis functions and shells (bfa, bfb, a, b)
    const double* __restrict__ dket;    // per build: D'_cd of every ket, [component][ket position]
    const PrimPair* __restrict__ prim;  // all primitive pairs (bra access)
    const double* __restrict__ kprim;   // ket primitives, structure of arrays
    const float* __restrict__ prim32;   // FP32 copies of both (mixed builds: the FP32 evaluation reads
    const float* __restrict__ kprim32;  // them without conversions)
    int nket_list, knprim;
    const int* __restrict__ split;      // mixed builds, per task: kets below this list position use FP64,
                                        // the rest FP32 (one launch evaluates both parts)
    const int4* __restrict__ tasks;     // (bra index, first ket, end ket, window code wc | wd << 16); bra -1:
                                        // empty.  Task 8k + x is entry k of XCD x's queue.  Register-tiled
                                        // plans: bra index | (bras in the block - 1) << 28
    const double* __restrict__ ketq;    // register-tiled plans: Q of every ket (list order)
    const int* __restrict__ kpos;       // and its position in its pair class's Q-sorted list
    double tau;                         // Schwarz threshold
    int same;                           // bra and ket of the same pair class (ket position <= bra index)
    long long wrep;                     // private digestion: elements between the per-XCD replicas of W
                                        // (W is replica 0); 0: one shared W
    // multi-density builds (k_class_multi): ndens densities D' (and their J
    // accumulators W, K accumulators WK) dstride elements apart, their
    // gathered D'_cd (dket) and ket-block J accumulators (wket) kstride
    // elements apart
    int ndens;
    long long dstride, kstride;
    double* WK;
    int win, rs;                        // column window (0: whole rows) and LDS bra-row length (doubles)
    int dstage;                         // staged D' rows (0, 1: shell a's, 3: both): selects the kernel variant
    int task_off;                       // static launch: workgroup i runs task task_off + i
    unsigned long long* __restrict__ work;  // persistent launch: 8 per-XCD queue counters (zeroed before the
                                            // launch); null: one task per workgroup
    int qlen;                           // entries per XCD queue (tasks = 8 qlen)
    const long long* __restrict__ moff; // per molecule: element offset of its blocks in D', W
    const double* __restrict__ boys64;
    const double* __restrict__ D;       // component-scaled density D'
    double* __restrict__ W;             // accumulator, F_2e = s (W + W^T) s / 8
    double* __restrict__ wket;          // LDS mode: ket-block J sums, [component][ket position]
    unsigned long long* __restrict__ counters;  // the class's quartet counters (HFX_CNT_CLASS words)
    int shard, nshards;                 // only bras with r % nshards == shard (1 shard: all)
    double cj, ck;                      // W_ab += cj*2 g D_cd ; W_ac -= ck g D_bd
};

// Evaluated-quartet counters of a build: per class, FP64 then FP32, each
// spread over HFX_CNT_SLOTS words one 128-byte line apart (a workgroup adds
// into slot blockIdx mod HFX_CNT_SLOTS), summed on the host.  Kernels add once
// per wave at the end of a persistent launch, once per workgroup in the
// static form: one hot word per class taking an atomic per wave and task cost
// more than some classes' integrals.
#define HFX_CNT_SLOTS 8
#define HFX_CNT_STRIDE 16
#define HFX_CNT_CLASS (2 * HFX_CNT_SLOTS * HFX_CNT_STRIDE)
#define HFX_CNT_WORDS (21 * HFX_CNT_CLASS)   // then one word: the non-finite flag

// Index (0..7) of the accelerator complex die (XCD) the wave runs on, read
// from the hardware register.  It only selects which private copy of the
// accumulator a wave adds into: device-wide atomics keep any choice correct.
__device__ __forceinline__ int hfx_xcc_id() {
    unsigned x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    return (int)(x & 7u);
}

// Constant address space: loads through such a pointer at a wave-uniform
// address become scalar (SMEM) loads.
#define HFX_CONST_AS __attribute__((address_space(4)))

// ---- Boys function tables ---------------------------------------------------
// For every order L (0..BOYS_NL-1) one block of 64-byte rows:
//   block_L[k * 8 + j] = F_{L+j}(T_k) / j!,  T_k = k * BOYS_DT,
// so that F_L(T) = sum_j block_L[k*8 + j] (T_k - T)^j about the nearest grid
// point (dF_m/dT = -F_{m+1}); one aligned row is one cache line.  Blocks are
// stored in the order 1, 0, 2, 3, ... (boys_block) so that the order-0 rows
// directly follow the order-1 rows: read from global memory, a class of
// total angular momentum L = 1 takes F_0 from the order-0 row.  The class
// kernels copy only their order's block into LDS, each row followed by
// e^{-T_k}: there a class with L = 1 gets F_0 = 2T F_1 + e^{-T} from one row.
#define BOYS_DT 0.1
#define BOYS_INV_DT 10.0
#define BOYS_TMAX 40.0
#define BOYS_NT 402
#define BOYS_NL 9
#define BOYS_ROW 8
#define BOYS_ORDER64 8   // Taylor terms, FP64 (|T - T_k| <= 0.05: remainder < 1e-15 F)
#define BOYS_ORDER32 5   // Taylor terms, FP32 (remainder < 3e-9 F)

#define BOYS_EXP_OFF (BOYS_NL * BOYS_NT * BOYS_ROW)   // e^{-T_k}, k < BOYS_NT, after the blocks
#define BOYS_TAB_ENTRIES (BOYS_EXP_OFF + BOYS_NT)
void hfx_boys_table(double* tab);   // host, BOYS_TAB_ENTRIES entries

__host__ __device__ constexpr int boys_block(int L) { return L == 0 ? 1 : (L == 1 ? 0 : L); }
// LDS copy of a class's block: BOYS_NT rows of BOYS_LROW64 doubles, the
// row's 8 coefficients, then e^{-T_k} (BOYS_EXP_SLOT), then one pad.  An
// 80-byte stride instead of 64 makes the 16-byte reads of lanes at
// different rows start in 8 distinct groups of 4 of the 32 LDS banks rather
// than in 2.
#define BOYS_LROW64 10
#define BOYS_EXP_SLOT 8
__host__ __device__ constexpr int boys_entries() { return BOYS_NT * BOYS_ROW; }
__host__ __device__ constexpr int boys_lds_bytes() { return BOYS_NT * BOYS_LROW64 * 8; }

__device__ __forceinline__ double hfx_sqrt(double x) { return sqrt(x); }
// 1/sqrt(x) for x > 0: hardware estimate refined by Newton steps
// y <- y (3/2 - x/2 y^2) (two steps for FP64, one for FP32).
__device__ __forceinline__ double hfx_rsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * (1.5 - h * y * y);
    y = y * (1.5 - h * y * y);
    return y;
}
__device__ __forceinline__ float hfx_rsqrt(float x) {
    float y = __builtin_amdgcn_rsqf(x);
    return y * (1.5f - 0.5f * x * y * y);
}
__device__ __forceinline__ float hfx_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double hfx_exp(double x) { return exp(x); }
__device__ __forceinline__ float hfx_exp(float x) { return __expf(x); }

// Taylor value of F_L at T from the order-L table (row k, offset d = T_k - T).
template <int NO>
__device__ __forceinline__ double boys_taylor(const double* __restrict__ row, double d) {
    const double2* r2 = reinterpret_cast<const double2*>(row);
    const double2 c01 = r2[0], c23 = r2[1], c45 = r2[2], c67 = r2[3];
    const double c[8] = {c01.x, c01.y, c23.x, c23.y, c45.x, c45.y, c67.x, c67.y};
    double f = c[NO - 1];
#pragma unroll
    for (int j = NO - 2; j >= 0; --j) f = c[j] + f * d;
    return f;
}
template <int NO>
__device__ __forceinline__ float boys_taylor(const float* __restrict__ row, float d) {
    const float4* r4 = reinterpret_cast<const float4*>(row);
    const float4 c03 = r4[0], c47 = r4[1];
    const float c[8] = {c03.x, c03.y, c03.z, c03.w, c47.x, c47.y, c47.z, c47.w};
    float f = c[NO - 1];
#pragma unroll
    for (int j = NO - 2; j >= 0; --j) f = c[j] + f * d;
    return f;
}

// FP32 value from the FP64 rows (the mixed kernels keep one table in LDS):
// the NO leading coefficients rounded to FP32, then the same Horner steps.
template <int NO>
__device__ __forceinline__ float boys_taylor(const double* __restrict__ row, float d) {
    static_assert(NO <= 6, "FP32 Taylor order");
    const double2* r2 = reinterpret_cast<const double2*>(row);
    const double2 c01 = r2[0], c23 = r2[1], c45 = r2[2];
    const float c[6] = {(float)c01.x, (float)c01.y, (float)c23.x, (float)c23.y, (float)c45.x, (float)c45.y};
    float f = c[NO - 1];
#pragma unroll
    for (int j = NO - 2; j >= 0; --j) f = c[j] + f * d;
    return f;
}

__host__ __device__ constexpr double boys_inv_fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return 1.0 / f;
}

template <typename R> struct BoysOrder;
template <> struct BoysOrder<double> { static constexpr int value = BOYS_ORDER64; };
template <> struct BoysOrder<float> { static constexpr int value = BOYS_ORDER32; };

// F[0..L] at T.  Below BOYS_TMAX: Taylor expansion of F_L about the nearest
// grid point, then the downward recursion F_m = (2T F_{m+1} + e^{-T})/(2m+1)
// (for L = 1: from the LDS rows, e^{-T} = e^{-T_k} e^{T_k - T} with a short
// series for the second factor; from the global table, F_0 from its own
// row, no exponential needed).
// For L <= 1 the two regimes are branches; for L >= 2 both are evaluated
// with one shared exponential and selected per lane.
// Above: F_0 = sqrt(pi/T)/2 (erf(sqrt T) = 1 to FP64 there) and the upward recursion
// F_{m+1} = ((2m+1) F_m - e^{-T})/(2T), stable for T >> m (for L = 1 the
// exponential term is below rounding and dropped).
// tab: the order-L block (followed by the order-0 block when L = 1), rows S
// elements apart, in the evaluation's precision or (FP32 evaluation) FP64.
template <typename R, int L, int S = BOYS_ROW, typename TT = R>
__device__ __forceinline__ void boys_eval(R T, R* F, const TT* __restrict__ tab) {
    constexpr int NO = BoysOrder<R>::value;
    if constexpr (L <= 1) {
        if (T < R(BOYS_TMAX)) {
            const int k = (int)(T * R(BOYS_INV_DT) + R(0.5));
            const R d = R(k) * R(BOYS_DT) - T;
            F[L] = boys_taylor<NO>(tab + k * S, d);
            if constexpr (L == 1) {
                if constexpr (S > BOYS_EXP_SLOT) {
                    // e^{d}, |d| <= 0.05: 9 terms (FP64), 5 (FP32), Horner
                    constexpr int NE = sizeof(R) == 8 ? 9 : 5;
                    R ed = R(boys_inv_fact(NE - 1));
#pragma unroll
                    for (int j = NE - 2; j >= 0; --j) ed = R(boys_inv_fact(j)) + ed * d;
                    F[0] = R(2) * T * F[1] + R(tab[k * S + BOYS_EXP_SLOT]) * ed;
                } else {
                    F[0] = boys_taylor<NO>(tab + (BOYS_NT + k) * S, d);
                }
            }
        } else {
            const R rt = hfx_rsqrt(T);
            F[0] = R(0.886226925452758013649083741671) * rt;   // sqrt(pi)/2 / sqrt(T)
            // e^{-T} / F_0(T) < 3.1e-17 for T >= 40, below half an FP64 ulp:
            // F_1 = F_0 / (2T) without the exponential
            if constexpr (L == 1) F[1] = F[0] * (R(0.5) * rt * rt);
        }
    } else {
        // both regimes evaluated with one exponential, each lane selects its
        // own (the lanes of a wave usually straddle BOYS_TMAX); rows clamped
        // into the table for lanes in the asymptotic regime
        const bool near = T < R(BOYS_TMAX);
        const int k = (int)(near ? T * R(BOYS_INV_DT) + R(0.5) : R(0));
        const R d = R(k) * R(BOYS_DT) - T;
        const R rt = hfx_rsqrt(T);
        const R h = R(0.5) * rt * rt;   // 1/(2T)
        const R e = hfx_exp(-T);
        R down[L + 1], up[L + 1];
        down[L] = boys_taylor<NO>(tab + k * S, d);
        const R t2 = R(2) * T;
#pragma unroll
        for (int m = L - 1; m >= 0; --m) down[m] = (t2 * down[m + 1] + e) * R(1.0 / (2 * m + 1));
        up[0] = R(0.886226925452758013649083741671) * rt;
#pragma unroll
        for (int m = 0; m < L; ++m) up[m + 1] = (R(2 * m + 1) * up[m] - e) * h;
#pragma unroll
        for (int m = 0; m <= L; ++m) F[m] = near ? down[m] : up[m];
    }
}

constexpr int hfx_ncart(int l) { return (l + 1) * (l + 2) / 2; }
