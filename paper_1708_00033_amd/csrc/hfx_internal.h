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

// One shell pair in canonical orientation: shells a (higher l) and b, their
// first basis functions, its primitive pairs, its Schwarz bound and A - B.
struct PairInfo {
    int a, b;
    int bfa, bfb;
    int prim_off, nprim;
    double Q;
    double AB[3];
    double pad;
};

// Arguments of one class kernel launch.
struct ClassArgs {
    const PairInfo* __restrict__ bra;   // bra pairs of the class, Q descending
    const PairInfo* __restrict__ ket;   // ket pairs of the class, Q descending
    const PrimPair* __restrict__ prim;  // all primitive pairs
    const int* __restrict__ nket;       // per bra: number of kets (screened prefix)
    const int* __restrict__ split;      // per bra: kets below this index use FP64 (nullptr: all)
    const int2* __restrict__ tasks;     // (bra index, first ket) per workgroup
    const double* __restrict__ boys64;
    const float* __restrict__ boys32;
    const double* __restrict__ D;       // component-scaled density D'
    double* __restrict__ W;             // accumulator, F_2e = s (W + W^T) s / 8
    unsigned long long* __restrict__ counters;  // [0] FP64 quartets, [1] FP32 quartets
    int nbf;
    int same_class;
    int task_quartets;
    double cj, ck;                      // W_ab += cj*2 g D_cd ; W_ac -= ck g D_bd
};

// ---- Boys function table -------------------------------------------------------
// F_m(T_k) on T_k = k * BOYS_DT, k = 0..BOYS_NT-1, m = 0..BOYS_NM-1.
// F_m(T) = sum_j F_{m+j}(T_k) (T_k - T)^j / j!  (dF_m/dT = -F_{m+1}).
#define BOYS_DT 0.1
#define BOYS_INV_DT 10.0
#define BOYS_TMAX 40.0
#define BOYS_NT 402
#define BOYS_NM 17
#define BOYS_ORDER64 8   // Taylor terms, FP64 (|T - T_k| <= 0.05: remainder < 1e-15 F)
#define BOYS_ORDER32 5   // Taylor terms, FP32 (remainder < 3e-9 F)

void hfx_boys_table(double* tab);   // host, BOYS_NT * BOYS_NM entries

__device__ __forceinline__ double hfx_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float hfx_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double hfx_exp(double x) { return exp(x); }
__device__ __forceinline__ float hfx_exp(float x) { return __expf(x); }

template <typename R> struct BoysOrder;
template <> struct BoysOrder<double> { static constexpr int value = BOYS_ORDER64; };
template <> struct BoysOrder<float> { static constexpr int value = BOYS_ORDER32; };

// F[0..L] at T.  Below BOYS_TMAX: Taylor expansion of F_L about the nearest
// grid point, then the downward recursion F_m = (2T F_{m+1} + e^{-T})/(2m+1)
// (for L <= 1 every order is taken from the table, no exponential needed).
// Above: F_0 = sqrt(pi/T)/2 and the upward recursion
// F_{m+1} = ((2m+1) F_m - e^{-T})/(2T), stable for T >> m.
template <typename R, int L>
__device__ __forceinline__ void boys_eval(R T, R* F, const R* __restrict__ tab) {
    constexpr int NO = BoysOrder<R>::value;
    if (T < R(BOYS_TMAX)) {
        const int k = (int)(T * R(BOYS_INV_DT) + R(0.5));
        const R d = R(k) * R(BOYS_DT) - T;
        const R* row = tab + k * BOYS_NM;
        if constexpr (L <= 1) {
#pragma unroll
            for (int m = 0; m <= L; ++m) {
                R f = row[m + NO - 1];
#pragma unroll
                for (int j = NO - 1; j >= 1; --j) f = row[m + j - 1] + f * d * R(1.0 / j);
                F[m] = f;
            }
        } else {
            R f = row[L + NO - 1];
#pragma unroll
            for (int j = NO - 1; j >= 1; --j) f = row[L + j - 1] + f * d * R(1.0 / j);
            F[L] = f;
            const R e = hfx_exp(-T);
            const R t2 = R(2) * T;
#pragma unroll
            for (int m = L - 1; m >= 0; --m) F[m] = (t2 * F[m + 1] + e) * R(1.0 / (2 * m + 1));
        }
    } else {
        const R it = R(1) / T;
        F[0] = R(0.886226925452758013649083741671) * hfx_sqrt(it);   // sqrt(pi)/2
        if constexpr (L > 0) {
            const R e = hfx_exp(-T);
            const R h = R(0.5) * it;
#pragma unroll
            for (int m = 0; m < L; ++m) F[m + 1] = (R(2 * m + 1) * F[m] - e) * h;
        }
    }
}

constexpr int hfx_ncart(int l) { return (l + 1) * (l + 2) / 2; }
