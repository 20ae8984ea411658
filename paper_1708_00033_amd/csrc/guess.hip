// Learned initial guess: pair descriptors and frames, the network's BF16
// MFMA forward and backward passes with FP32 accumulation, Adam, and the
// rotation of density blocks between pair frames and the molecule.
//
// The SCF of section 3 needs a starting density; the library's default is a
// superposition of atomic densities (SAD).  This extension predicts, for each
// atom pair within 6 A, the converged-minus-SAD density block in a local frame
// of the pair, from a 164-number descriptor of the pair's surroundings:
//   [one-hot element of A, of B, 32 radial Gaussians of R_AB with a cosine
//    cutoff, A's environment (log(1 + the radial functions summed over
//    neighbours), one 32-block per element), B's environment].
// Network: 164 -> 256 -> 256 -> 256 (SiLU) -> one linear head per pair type
// (O-O 225, O-H 30, H-H 4 outputs = the 15 x 15, 15 x 2, 2 x 2 blocks).
// Layers run as MFMA GEMMs (v_mfma_f32_16x16x32_bf16): BF16 operands, FP32
// accumulation; pre-activations and gradients are kept in FP32, Adam
// updates FP32 master weights.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "hfx_ctx.h"

namespace {

constexpr int NFEAT = 164, NRAD = 32, HID = 256, XLD = 192;   // XLD: padded feature row (bf16)
constexpr int NTYPE = 3;
constexpr int HEAD_OUT[NTYPE] = {225, 30, 4};
constexpr int MAXB = 16;                 // basis functions per atom handled by the block kernels
constexpr double BOHR_PER_A = 1.0 / 0.529177210903;
constexpr double RCUT_A = 6.0;
constexpr double TIE_BOHR = 1e-6;
constexpr double NONCOLLINEAR_SIN = 0.1;
constexpr float INPUT_CLIP = 4.0f;       // standardised inputs are clipped to +-INPUT_CLIP

typedef unsigned short bf16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---- parameter layout (FP32, packed): W1 b1 W2 b2 W3 b3, per head W c,
//      feature mean, feature scale, three target scales -----------------------------------

struct ParamLayout {
    long long off[15], size[15], total;
    ParamLayout() {
        const long long s[15] = {(long long)HID * NFEAT, HID, (long long)HID * HID, HID, (long long)HID * HID, HID,
                                 (long long)HEAD_OUT[0] * HID, HEAD_OUT[0], (long long)HEAD_OUT[1] * HID, HEAD_OUT[1],
                                 (long long)HEAD_OUT[2] * HID, HEAD_OUT[2], NFEAT, NFEAT, NTYPE};
        long long o = 0;
        for (int i = 0; i < 15; ++i) {
            off[i] = o;
            size[i] = s[i];
            o += s[i];
        }
        total = o;
    }
};
const ParamLayout PL;
enum { P_W1, P_B1, P_W2, P_B2, P_W3, P_B3, P_H0, P_C0, P_H1, P_C1, P_H2, P_C2, P_FMEAN, P_FSCALE, P_TSCALE };
constexpr int NTRAIN = 12;

// ---- small helpers -------------------------------------------------------------------

__device__ __forceinline__ bf16_t f2bf(float f) {   // round to nearest even
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

constexpr int WG = 256;
inline unsigned blocks_for(long long n) { return (unsigned)std::max<long long>(1, (n + WG - 1) / WG); }

// ---- descriptors and frames ------------------------------------------------------------

__device__ void radial(double r_a, double* g) {
    const double dmu = 5.5 / (NRAD - 1), eta = 1.0 / (2.0 * dmu * dmu);
    const double fc = r_a < RCUT_A ? 0.5 * (cos(M_PI * r_a / RCUT_A) + 1.0) : 0.0;
    for (int k = 0; k < NRAD; ++k) {
        const double mu = 0.5 + dmu * k, d = r_a - mu;
        g[k] = exp(-eta * d * d) * fc;
    }
}

__device__ __forceinline__ double dist(const double* xyz, int a, int b) {
    const double dx = xyz[3 * b] - xyz[3 * a], dy = xyz[3 * b + 1] - xyz[3 * a + 1], dz = xyz[3 * b + 2] - xyz[3 * a + 2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

// env[a][e*32 + k] = log(1 + sum over atoms c != a of element e of G_k(R_ac));
// one thread per (atom, e, k)
__global__ void k_env(int natom, const double* __restrict__ xyz, const int* __restrict__ elem, double* __restrict__ env) {
    const long long i = (long long)blockIdx.x * WG + threadIdx.x;
    if (i >= (long long)natom * 2 * NRAD) return;
    const int a = (int)(i / (2 * NRAD)), q = (int)(i % (2 * NRAD)), e = q / NRAD, k = q % NRAD;
    const double dmu = 5.5 / (NRAD - 1), eta = 1.0 / (2.0 * dmu * dmu), mu = 0.5 + dmu * k;
    double acc = 0.0;
    for (int c = 0; c < natom; ++c) {
        if (c == a || elem[c] != e) continue;
        const double r = dist(xyz, a, c) / BOHR_PER_A;
        if (r >= RCUT_A) continue;
        const double d = r - mu;
        acc += exp(-eta * d * d) * 0.5 * (cos(M_PI * r / RCUT_A) + 1.0);
    }
    env[i] = log1p(acc);
}

// ordering key of candidate atoms: distance in bins of TIE_BOHR, then index
__device__ __forceinline__ bool key_less(double da, int a, double db, int b) {
    const double fa = floor(da / TIE_BOHR), fb = floor(db / TIE_BOHR);
    return fa < fb || (fa == fb && a < b);
}

// One thread per pair: 164 features and the frame (rows x, y, z).
__global__ void k_pair_setup(int natom, const double* __restrict__ xyz, const int* __restrict__ elem,
                             const double* __restrict__ env, int npair, const int4* __restrict__ pairs,
                             float* __restrict__ feat, double* __restrict__ frames) {
    const int p = blockIdx.x * WG + threadIdx.x;
    if (p >= npair) return;
    const int a = pairs[p].x;
    int b = pairs[p].y;
    float* f = feat + (size_t)p * NFEAT;
    for (int k = 0; k < NFEAT; ++k) f[k] = 0.0f;
    f[elem[a]] = 1.0f;
    f[2 + elem[b]] = 1.0f;
    double g[NRAD];
    radial(dist(xyz, a, b) / BOHR_PER_A, g);
    for (int k = 0; k < NRAD; ++k) f[4 + k] = (float)g[k];
    for (int k = 0; k < 2 * NRAD; ++k) {
        f[4 + NRAD + k] = (float)env[(size_t)a * 2 * NRAD + k];
        f[4 + 3 * NRAD + k] = (float)env[(size_t)b * 2 * NRAD + k];
    }
    // frame
    double* R = frames + (size_t)p * 9;
    if (a == b) {   // self block: z toward the nearest atom
        int best = -1;
        double bd = 0.0;
        for (int c = 0; c < natom; ++c) {
            if (c == a) continue;
            const double d = dist(xyz, a, c);
            if (best < 0 || key_less(d, c, bd, best)) { best = c; bd = d; }
        }
        if (best < 0) {
            for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0 : 0.0;
            return;
        }
        b = best;
    }
    double z[3] = {xyz[3 * b] - xyz[3 * a], xyz[3 * b + 1] - xyz[3 * a + 1], xyz[3 * b + 2] - xyz[3 * a + 2]};
    double n = sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
    for (int i = 0; i < 3; ++i) z[i] /= n;
    int best = -1;
    double bd = 0.0;
    for (int c = 0; c < natom; ++c) {
        if (c == a || c == b) continue;
        const double v[3] = {xyz[3 * c] - xyz[3 * a], xyz[3 * c + 1] - xyz[3 * a + 1], xyz[3 * c + 2] - xyz[3 * a + 2]};
        const double d = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        const double cx = (v[1] * z[2] - v[2] * z[1]) / d, cy = (v[2] * z[0] - v[0] * z[2]) / d,
                     cz = (v[0] * z[1] - v[1] * z[0]) / d;
        if (sqrt(cx * cx + cy * cy + cz * cz) <= NONCOLLINEAR_SIN) continue;
        if (best < 0 || key_less(d, c, bd, best)) { best = c; bd = d; }
    }
    double x[3];
    if (best >= 0) {
        const double v[3] = {xyz[3 * best] - xyz[3 * a], xyz[3 * best + 1] - xyz[3 * a + 1],
                             xyz[3 * best + 2] - xyz[3 * a + 2]};
        const double vz = v[0] * z[0] + v[1] * z[1] + v[2] * z[2];
        for (int i = 0; i < 3; ++i) x[i] = v[i] - vz * z[i];
    } else {   // global axis least aligned with z
        int k = 0;
        for (int i = 1; i < 3; ++i)
            if (fabs(z[i]) < fabs(z[k])) k = i;
        for (int i = 0; i < 3; ++i) x[i] = (i == k ? 1.0 : 0.0) - z[k] * z[i];
    }
    n = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    for (int i = 0; i < 3; ++i) x[i] /= n;
    const double y[3] = {z[1] * x[2] - z[2] * x[1], z[2] * x[0] - z[0] * x[2], z[0] * x[1] - z[1] * x[0]};
    for (int i = 0; i < 3; ++i) {
        R[i] = x[i];
        R[3 + i] = y[i];
        R[6 + i] = z[i];
    }
}

// ---- block rotation --------------------------------------------------------------------

struct AtomBasis {
    const int* first;   // first basis function of the atom (molecule-local)
    const int* nb;      // functions on the atom
    const int* shoff;   // shell list offset
    const int* nsh;     // shells on the atom
    const int* shl;     // shell angular momenta
};

// T (n x n, row-major, LDS) with phi(R r) = T phi(r) for the atom's shells:
// s -> 1, p -> R, unit-normalised Cartesian d -> N M(R) N^-1.
__device__ void build_T(const AtomBasis& ab, int atom, const double* R, bool transpose_R, double* T, int n) {
    for (int i = threadIdx.x; i < n * n; i += blockDim.x) T[i] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
        double Q[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Q[3 * i + j] = transpose_R ? R[3 * j + i] : R[3 * i + j];
        const int dc[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
        const double s3 = 0.57735026918962576451;
        const double dn[6] = {s3, 1.0, 1.0, s3, 1.0, s3};
        int o = 0;
        for (int s = 0; s < ab.nsh[atom]; ++s) {
            const int l = ab.shl[ab.shoff[atom] + s];
            if (l == 0) {
                T[o * n + o] = 1.0;
                o += 1;
            } else if (l == 1) {
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) T[(o + i) * n + o + j] = Q[3 * i + j];
                o += 3;
            } else {
                for (int p = 0; p < 6; ++p)
                    for (int q = 0; q < 6; ++q) {
                        const int a = dc[p][0], b = dc[p][1], i = dc[q][0], j = dc[q][1];
                        double m = Q[3 * a + i] * Q[3 * b + j];
                        if (i != j) m += Q[3 * a + j] * Q[3 * b + i];
                        T[(o + p) * n + o + q] = dn[p] * m / dn[q];
                    }
                o += 6;
            }
        }
    }
    __syncthreads();
}

// P = TA^T X TB for one pair (n_a x n_b), all in LDS; tmp n_a x n_b.
__device__ void sandwich(const double* TA, int na, const double* X, const double* TB, int nb, double* tmp, double* P) {
    for (int i = threadIdx.x; i < na * nb; i += blockDim.x) {
        const int r = i / nb, c = i % nb;
        double s = 0.0;
        for (int k = 0; k < nb; ++k) s += X[r * nb + k] * TB[k * nb + c];
        tmp[i] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < na * nb; i += blockDim.x) {
        const int r = i / nb, c = i % nb;
        double s = 0.0;
        for (int k = 0; k < na; ++k) s += TA[k * na + r] * tmp[k * nb + c];
        P[i] = s;
    }
    __syncthreads();
}

// Local blocks of (D - Dbase): P = T_A(R^T)^T (D - Dbase)_AB T_B(R^T), packed FP32.
__global__ __launch_bounds__(64) void k_to_local(int npair, const int4* __restrict__ pairs,
                                                 const double* __restrict__ frames, AtomBasis ab,
                                                 const long long* __restrict__ out_off, const double* __restrict__ D,
                                                 const double* __restrict__ Db, int n, float* __restrict__ out) {
    __shared__ double TA[MAXB * MAXB], TB[MAXB * MAXB], X[MAXB * MAXB], tmp[MAXB * MAXB], P[MAXB * MAXB];
    const int p = blockIdx.x;
    const int a = pairs[p].x, b = pairs[p].y;
    const int na = ab.nb[a], nb = ab.nb[b];
    const double* R = frames + (size_t)p * 9;
    build_T(ab, a, R, true, TA, na);
    build_T(ab, b, R, true, TB, nb);
    const int fa = ab.first[a], fb = ab.first[b];
    for (int i = threadIdx.x; i < na * nb; i += blockDim.x) {
        const size_t g = (size_t)(fa + i / nb) * n + fb + i % nb;
        X[i] = D[g] - (Db ? Db[g] : 0.0);
    }
    __syncthreads();
    sandwich(TA, na, X, TB, nb, tmp, P);
    for (int i = threadIdx.x; i < na * nb; i += blockDim.x) out[out_off[p] + i] = (float)P[i];
}

// D = Dbase + sum over pairs of T_A(R)^T P T_B(R) at (A, B) and its transpose
// at (B, A) (a self block symmetrised).  Each block belongs to one pair.
__global__ __launch_bounds__(64) void k_assemble_blocks(int npair, const int4* __restrict__ pairs,
                                                        const double* __restrict__ frames, AtomBasis ab,
                                                        const long long* __restrict__ in_off,
                                                        const float* __restrict__ blocks, int n,
                                                        double* __restrict__ D) {
    __shared__ double TA[MAXB * MAXB], TB[MAXB * MAXB], X[MAXB * MAXB], tmp[MAXB * MAXB], P[MAXB * MAXB];
    const int p = blockIdx.x;
    const int a = pairs[p].x, b = pairs[p].y;
    const int na = ab.nb[a], nb = ab.nb[b];
    const double* R = frames + (size_t)p * 9;
    build_T(ab, a, R, false, TA, na);
    build_T(ab, b, R, false, TB, nb);
    const float* in = blocks + in_off[p];
    for (int i = threadIdx.x; i < na * nb; i += blockDim.x) {
        const int r = i / nb, c = i % nb;
        X[i] = a == b ? 0.5 * ((double)in[r * nb + c] + (double)in[c * nb + r]) : (double)in[i];
    }
    __syncthreads();
    sandwich(TA, na, X, TB, nb, tmp, P);
    const int fa = ab.first[a], fb = ab.first[b];
    for (int i = threadIdx.x; i < na * nb; i += blockDim.x) {
        const int r = i / nb, c = i % nb;
        D[(size_t)(fa + r) * n + fb + c] += P[i];
        if (a != b) D[(size_t)(fb + c) * n + fa + r] += P[i];
    }
}

__global__ void k_copy(const double* __restrict__ s, size_t n, double* __restrict__ d) {
    for (size_t i = (size_t)blockIdx.x * WG + threadIdx.x; i < n; i += (size_t)gridDim.x * WG) d[i] = s[i];
}

// out[0] += sum D_ij S_ij, out[1] += number of non-finite D_ij
__global__ void k_trace_check(const double* __restrict__ D, const double* __restrict__ S, size_t n, double* out) {
    double acc = 0.0, bad = 0.0;
    for (size_t i = (size_t)blockIdx.x * WG + threadIdx.x; i < n; i += (size_t)gridDim.x * WG) {
        const double d = D[i];
        if (isfinite(d)) acc += d * S[i]; else bad += 1.0;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        acc += __shfl_xor(acc, off, 64);
        bad += __shfl_xor(bad, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(out, acc);
        atomicAdd(out + 1, bad);
    }
}

// ---- the network -----------------------------------------------------------------------

enum { EPI_STORE = 0, EPI_SILU = 1, EPI_DSILU = 2 };

struct GemmArgs {
    int M, N, K;
    const bf16_t* A;
    long long asi, ask;    // A(i, k) = A[i asi + k ask]
    const bf16_t* B;
    long long bsk, bsj;    // B(k, j) = B[k bsk + j bsj]
    const float* bias;     // per column j (EPI_STORE optional, EPI_SILU required)
    float* C;              // FP32 result (pre-activation or gradient)
    long long ldc;
    bf16_t* Cb;            // BF16 copy for the next GEMM (SiLU output for EPI_SILU)
    long long ldcb;
    const float* Z;        // EPI_DSILU: pre-activation whose SiLU derivative scales the result
    long long ldz;
    int epi;
};

constexpr int GBM = 64, GBN = 64, GBK = 32, GPAD = 8;

// C = A B on 64 x 64 tiles; four waves, each a 32 x 32 quadrant of 2 x 2
// MFMA 16x16x32 blocks.  Operands staged through LDS as BF16 (zero outside
// M, N, K), FP32 accumulators, fused epilogue.
__global__ __launch_bounds__(256) void k_gemm(const GemmArgs g) {
    __shared__ __align__(16) bf16_t As[GBM][GBK + GPAD];
    __shared__ __align__(16) bf16_t Bs[GBN][GBK + GPAD];
    const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * GBN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int lr = t >> 2, lk = (t & 3) * 8;
    for (int k0 = 0; k0 < g.K; k0 += GBK) {
        const long long i = m0 + lr, j = n0 + lr;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const long long k = k0 + lk + e;
            As[lr][lk + e] = (i < g.M && k < g.K) ? g.A[i * g.asi + k * g.ask] : (bf16_t)0;
            Bs[lr][lk + e] = (j < g.N && k < g.K) ? g.B[k * g.bsk + j * g.bsj] : (bf16_t)0;
        }
        __syncthreads();
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                const uint4 ua = *reinterpret_cast<const uint4*>(&As[wr + bi * 16 + (lane & 15)][(lane >> 4) * 8]);
                const uint4 ub = *reinterpret_cast<const uint4*>(&Bs[wc + bj * 16 + (lane & 15)][(lane >> 4) * 8]);
                acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ua),
                                                                     __builtin_bit_cast(bf16x8, ub), acc[bi][bj], 0,
                                                                     0, 0);
            }
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long i = m0 + wr + bi * 16 + (lane >> 4) * 4 + r;
                const long long j = n0 + wc + bj * 16 + (lane & 15);
                if (i >= g.M || j >= g.N) continue;
                float v = acc[bi][bj][r];
                if (g.epi == EPI_DSILU) v *= dsilu_f(g.Z[i * g.ldz + j]);
                else if (g.bias) v += g.bias[j];
                if (g.C) g.C[i * g.ldc + j] = v;
                if (g.Cb) g.Cb[i * g.ldcb + j] = f2bf(g.epi == EPI_SILU ? silu_f(v) : v);
            }
}

// standardised, clipped features as BF16 rows of XLD (zero padding)
__global__ void k_feat_bf16(const float* __restrict__ X, long long M, const float* __restrict__ mean,
                            const float* __restrict__ scale, bf16_t* __restrict__ out) {
    const long long i = (long long)blockIdx.x * WG + threadIdx.x;
    if (i >= M * XLD) return;
    const long long r = i / XLD;
    const int c = (int)(i % XLD);
    out[i] = c < NFEAT ? f2bf(fminf(fmaxf((X[r * NFEAT + c] - mean[c]) / scale[c], -INPUT_CLIP), INPUT_CLIP))
                       : (bf16_t)0;
}

__global__ void k_to_bf16(const float* __restrict__ W, int rows, int cols, int ldo, bf16_t* __restrict__ out) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= rows * ldo) return;
    const int r = i / ldo, c = i % ldo;
    out[i] = c < cols ? f2bf(W[(size_t)r * cols + c]) : (bf16_t)0;
}

__global__ void k_fill_f(float* __restrict__ p, long long n, float v) {
    const long long i = (long long)blockIdx.x * WG + threadIdx.x;
    if (i < n) p[i] = v;
}

// squared error of one head: d = Y - T / tscale; dY = gs d (FP32 and BF16);
// loss += sum d^2 (double)
__global__ void k_mse(const float* __restrict__ Y, const float* __restrict__ T, long long n, float inv_scale,
                      float gs, float* __restrict__ dY, bf16_t* __restrict__ dYb, double* __restrict__ loss) {
    const long long i = (long long)blockIdx.x * WG + threadIdx.x;
    double e = 0.0;
    if (i < n) {
        const float d = Y[i] - T[i] * inv_scale;
        e = (double)d * d;
        dY[i] = gs * d;
        dYb[i] = f2bf(gs * d);
    }
    for (int off = 32; off >= 1; off >>= 1) e += __shfl_xor(e, off, 64);
    if ((threadIdx.x & 63) == 0 && e != 0.0) atomicAdd(loss, e);
}

__global__ void k_scale(const float* __restrict__ Y, long long n, float s, float* __restrict__ out) {
    const long long i = (long long)blockIdx.x * WG + threadIdx.x;
    if (i < n) out[i] = Y[i] * s;
}

// out[j] += sum over rows of G[r][j]: 64 columns x 4 row lanes per block,
// blockIdx.y = chunk of 1024 rows
__global__ void k_colsum(const float* __restrict__ G, long long M, int N, long long ld, float* __restrict__ out) {
    __shared__ float red[4][64];
    const int cx = threadIdx.x & 63, ry = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + cx;
    const long long r0 = (long long)blockIdx.y * 1024, r1 = std::min<long long>(M, r0 + 1024);
    float s = 0.0f;
    if (j < N)
        for (long long r = r0 + ry; r < r1; r += 4) s += G[r * ld + j];
    red[ry][cx] = s;
    __syncthreads();
    if (ry == 0 && j < N) atomicAdd(out + j, red[0][cx] + red[1][cx] + red[2][cx] + red[3][cx]);
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const long long i = (long long)blockIdx.x * WG + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

}  // namespace

// ---- context side: pairs, frames, features ----------------------------------------------

struct GuessPairsDev {
    int counts[NTYPE] = {0, 0, 0};
    int npair = 0;
    long long npacked = 0;
    int4* d_pairs = nullptr;
    double* d_frames = nullptr;
    float* d_feat = nullptr;
    long long* d_off = nullptr;
    double* d_xyz = nullptr;
    int* d_elem = nullptr;
    double* d_env = nullptr;
    int *d_first = nullptr, *d_nb = nullptr, *d_shoff = nullptr, *d_nsh = nullptr, *d_shl = nullptr;
    float* d_T = nullptr;
    double* d_red = nullptr;
    std::vector<int> hpairs;
    AtomBasis ab() const { return AtomBasis{d_first, d_nb, d_shoff, d_nsh, d_shl}; }
};

template <typename T>
static void gfree(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}
template <typename T>
static hipError_t galloc(T** p, size_t n) {
    *p = nullptr;
    return hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T));
}

void hfx_guess_release(hfx_ctx* c) {
    GuessPairsDev* G = c->guess;
    if (!G) return;
    gfree(G->d_pairs);
    gfree(G->d_frames);
    gfree(G->d_feat);
    gfree(G->d_off);
    gfree(G->d_xyz);
    gfree(G->d_elem);
    gfree(G->d_env);
    gfree(G->d_first);
    gfree(G->d_nb);
    gfree(G->d_shoff);
    gfree(G->d_nsh);
    gfree(G->d_shl);
    gfree(G->d_T);
    gfree(G->d_red);
    delete G;
    c->guess = nullptr;
}

#define GCK(call)                                                        \
    do {                                                                 \
        hfx_status _s = hfx_hip_check(c, (call), #call);                 \
        if (_s != HFX_OK) return _s;                                     \
    } while (0)

static int element_index(int z) { return z == 8 ? 0 : (z == 1 ? 1 : -1); }

extern "C" hfx_status hfx_guess_setup(hfx_ctx* c, int* counts) {
    if (!c) return HFX_ERR_INVALID_ARG;
    if (!c->loaded) return hfx_fail(c, HFX_ERR_STATE, "guess: nothing loaded");
    if (c->nmol != 1) return hfx_fail(c, HFX_ERR_STATE, "guess: single molecules only");
    GCK(hipSetDevice(c->opt.device));
    hfx_guess_release(c);
    const int na = c->natom;
    std::vector<int> elem(na), first(na, -1), nb(na, 0), nsh(na, 0), shoff(na, 0), shl;
    for (int a = 0; a < na; ++a) {
        elem[a] = element_index(c->Z[a]);
        if (elem[a] < 0) return hfx_fail(c, HFX_ERR_INVALID_ARG, "guess: elements O and H only");
    }
    std::vector<std::vector<int>> als(na);
    for (int s = 0; s < c->nshell; ++s) {
        const int a = c->shell_atom[s];
        if (first[a] < 0) first[a] = c->shells[s].bf;
        als[a].push_back(c->shells[s].l);
        nb[a] += (c->shells[s].l + 1) * (c->shells[s].l + 2) / 2;
    }
    for (int a = 0; a < na; ++a) {
        const int want = elem[a] == 0 ? 15 : 2;
        if (nb[a] != want)
            return hfx_fail(c, HFX_ERR_INVALID_ARG, "guess: the network needs 15 functions on O and 2 on H");
        shoff[a] = (int)shl.size();
        nsh[a] = (int)als[a].size();
        for (int l : als[a]) shl.push_back(l);
    }
    // pairs within the cutoff, A <= B in (element, index) order; sorted by type
    std::vector<int4> pairs;
    for (int a = 0; a < na; ++a)
        for (int b = 0; b < na; ++b) {
            if (std::make_pair(elem[a], a) > std::make_pair(elem[b], b)) continue;
            const double* pa = &c->axyz[3 * a];
            const double* pb = &c->axyz[3 * b];
            const double dx = pb[0] - pa[0], dy = pb[1] - pa[1], dz = pb[2] - pa[2];
            if (std::sqrt(dx * dx + dy * dy + dz * dz) / BOHR_PER_A >= RCUT_A) continue;
            pairs.push_back(int4{a, b, elem[a] + elem[b], 0});
        }
    std::stable_sort(pairs.begin(), pairs.end(), [](const int4& u, const int4& v) {
        return u.z != v.z ? u.z < v.z : (u.x != v.x ? u.x < v.x : u.y < v.y);
    });
    auto* G = new GuessPairsDev();
    c->guess = G;
    G->npair = (int)pairs.size();
    std::vector<long long> off(pairs.size());
    long long o = 0;
    for (size_t p = 0; p < pairs.size(); ++p) {
        G->counts[pairs[p].z]++;
        off[p] = o;
        o += (long long)nb[pairs[p].x] * nb[pairs[p].y];
    }
    G->npacked = o;
    for (auto& p : pairs) {
        G->hpairs.push_back(p.x);
        G->hpairs.push_back(p.y);
    }
    GCK(galloc(&G->d_pairs, pairs.size()));
    GCK(galloc(&G->d_frames, pairs.size() * 9));
    GCK(galloc(&G->d_feat, pairs.size() * NFEAT));
    GCK(galloc(&G->d_off, pairs.size()));
    GCK(galloc(&G->d_xyz, (size_t)na * 3));
    GCK(galloc(&G->d_elem, na));
    GCK(galloc(&G->d_env, (size_t)na * 2 * NRAD));
    GCK(galloc(&G->d_first, na));
    GCK(galloc(&G->d_nb, na));
    GCK(galloc(&G->d_shoff, na));
    GCK(galloc(&G->d_nsh, na));
    GCK(galloc(&G->d_shl, shl.size()));
    GCK(galloc(&G->d_T, (size_t)o));
    GCK(galloc(&G->d_red, 2));
    GCK(hipMemcpy(G->d_pairs, pairs.data(), pairs.size() * sizeof(int4), hipMemcpyHostToDevice));
    GCK(hipMemcpy(G->d_off, off.data(), off.size() * 8, hipMemcpyHostToDevice));
    GCK(hipMemcpy(G->d_xyz, c->axyz.data(), (size_t)na * 3 * 8, hipMemcpyHostToDevice));
    GCK(hipMemcpy(G->d_elem, elem.data(), na * 4, hipMemcpyHostToDevice));
    GCK(hipMemcpy(G->d_first, first.data(), na * 4, hipMemcpyHostToDevice));
    GCK(hipMemcpy(G->d_nb, nb.data(), na * 4, hipMemcpyHostToDevice));
    GCK(hipMemcpy(G->d_shoff, shoff.data(), na * 4, hipMemcpyHostToDevice));
    GCK(hipMemcpy(G->d_nsh, nsh.data(), na * 4, hipMemcpyHostToDevice));
    GCK(hipMemcpy(G->d_shl, shl.data(), shl.size() * 4, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_env, dim3(blocks_for((long long)na * 2 * NRAD)), dim3(WG), 0, nullptr, na, G->d_xyz,
                       G->d_elem, G->d_env);
    GCK(hipGetLastError());
    if (G->npair > 0) {
        hipLaunchKernelGGL(k_pair_setup, dim3(blocks_for(G->npair)), dim3(WG), 0, nullptr, na, G->d_xyz, G->d_elem,
                           G->d_env, G->npair, G->d_pairs, G->d_feat, G->d_frames);
        GCK(hipGetLastError());
    }
    GCK(hipDeviceSynchronize());
    if (counts)
        for (int t = 0; t < NTYPE; ++t) counts[t] = G->counts[t];
    return HFX_OK;
}

extern "C" hfx_status hfx_guess_features(hfx_ctx* c, float* X, int* pairs, double* frames) {
    if (!c) return HFX_ERR_INVALID_ARG;
    if (!c->guess) return hfx_fail(c, HFX_ERR_STATE, "guess: call hfx_guess_setup first");
    GuessPairsDev* G = c->guess;
    GCK(hipSetDevice(c->opt.device));
    if (X) GCK(hipMemcpy(X, G->d_feat, (size_t)G->npair * NFEAT * 4, hipMemcpyDeviceToHost));
    if (frames) GCK(hipMemcpy(frames, G->d_frames, (size_t)G->npair * 9 * 8, hipMemcpyDeviceToHost));
    if (pairs) std::memcpy(pairs, G->hpairs.data(), G->hpairs.size() * sizeof(int));
    return HFX_OK;
}

extern "C" hfx_status hfx_guess_features_dev(hfx_ctx* c, const float** dX) {
    if (!c || !dX) return HFX_ERR_INVALID_ARG;
    if (!c->guess) return hfx_fail(c, HFX_ERR_STATE, "guess: call hfx_guess_setup first");
    *dX = c->guess->d_feat;
    return HFX_OK;
}

extern "C" hfx_status hfx_guess_targets_dev(hfx_ctx* c, const double* dD, const double* dDbase, float* dT,
                                            void* stream) {
    if (!c || !dD || !dT) return c ? hfx_fail(c, HFX_ERR_INVALID_ARG, "null pointer") : HFX_ERR_INVALID_ARG;
    if (!c->guess) return hfx_fail(c, HFX_ERR_STATE, "guess: call hfx_guess_setup first");
    GuessPairsDev* G = c->guess;
    GCK(hipSetDevice(c->opt.device));
    if (G->npair == 0) return HFX_OK;
    hipLaunchKernelGGL(k_to_local, dim3(G->npair), dim3(64), 0, (hipStream_t)stream, G->npair, G->d_pairs,
                       G->d_frames, G->ab(), G->d_off, dD, dDbase, c->nbf, dT);
    GCK(hipGetLastError());
    return HFX_OK;
}

extern "C" hfx_status hfx_guess_assemble_dev(hfx_ctx* c, const float* dT, const double* dDbase, double* dD,
                                             void* stream) {
    if (!c || !dT || !dD) return c ? hfx_fail(c, HFX_ERR_INVALID_ARG, "null pointer") : HFX_ERR_INVALID_ARG;
    if (!c->guess) return hfx_fail(c, HFX_ERR_STATE, "guess: call hfx_guess_setup first");
    GuessPairsDev* G = c->guess;
    GCK(hipSetDevice(c->opt.device));
    const size_t nn = (size_t)c->nbf * c->nbf;
    if (dDbase && dDbase != dD)
        hipLaunchKernelGGL(k_copy, dim3(blocks_for((long long)std::min<size_t>(nn, 1u << 22))), dim3(WG), 0,
                           (hipStream_t)stream, dDbase, nn, dD);
    if (G->npair > 0)
        hipLaunchKernelGGL(k_assemble_blocks, dim3(G->npair), dim3(64), 0, (hipStream_t)stream, G->npair,
                           G->d_pairs, G->d_frames, G->ab(), G->d_off, dT, c->nbf, dD);
    GCK(hipGetLastError());
    return HFX_OK;
}

// ---- the network object ----------------------------------------------------------------

struct hfx_guess {
    int device = 0;
    std::string err;
    std::vector<float> hp;
    float *p = nullptr, *gr = nullptr, *m = nullptr, *v = nullptr;
    bf16_t *W1b = nullptr, *W2b = nullptr, *W3b = nullptr, *Hb[NTYPE] = {nullptr, nullptr, nullptr};
    long long cap = 0, ycap = 0;
    bf16_t *Xb = nullptr, *H1b = nullptr, *H2b = nullptr, *H3b = nullptr, *Gab = nullptr, *Gbb = nullptr,
           *dYb = nullptr;
    float *Z1 = nullptr, *Z2 = nullptr, *Z3 = nullptr, *Ga = nullptr, *Gb = nullptr, *Y = nullptr, *dY = nullptr;
    double* d_loss = nullptr;
    long long step = 0;
    bool wdirty = true;
};

static hfx_status gfail(hfx_guess* g, hfx_status s, const std::string& msg) {
    if (g) g->err = msg;
    return s;
}
#define NCK(call)                                                                                   \
    do {                                                                                            \
        hipError_t _e = (call);                                                                     \
        if (_e != hipSuccess)                                                                       \
            return gfail(g, _e == hipErrorOutOfMemory ? HFX_ERR_OOM : HFX_ERR_DEVICE,               \
                         std::string(#call) + ": " + hipGetErrorString(_e));                        \
    } while (0)

static void free_acts(hfx_guess* g) {
    gfree(g->Xb);
    gfree(g->H1b);
    gfree(g->H2b);
    gfree(g->H3b);
    gfree(g->Gab);
    gfree(g->Gbb);
    gfree(g->Z1);
    gfree(g->Z2);
    gfree(g->Z3);
    gfree(g->Ga);
    gfree(g->Gb);
    g->cap = 0;
}

extern "C" void hfx_guess_destroy(hfx_guess* g) {
    if (!g) return;
    (void)hipSetDevice(g->device);
    free_acts(g);
    gfree(g->Y);
    gfree(g->dY);
    gfree(g->dYb);
    gfree(g->p);
    gfree(g->gr);
    gfree(g->m);
    gfree(g->v);
    gfree(g->W1b);
    gfree(g->W2b);
    gfree(g->W3b);
    for (auto& h : g->Hb) gfree(h);
    gfree(g->d_loss);
    delete g;
}

extern "C" long long hfx_guess_param_count(void) { return PL.total; }

extern "C" hfx_status hfx_guess_create(int device, hfx_guess** out) {
    if (!out) return HFX_ERR_INVALID_ARG;
    *out = nullptr;
    auto* g = new hfx_guess();
    g->device = device;
    auto fail = [&](hfx_status s) {
        hfx_guess_destroy(g);
        return s;
    };
    if (hipSetDevice(device) != hipSuccess) return fail(HFX_ERR_DEVICE);
    const long long n = PL.total;
    if (galloc(&g->p, n) || galloc(&g->gr, n) || galloc(&g->m, n) || galloc(&g->v, n) ||
        galloc(&g->W1b, (size_t)HID * XLD) || galloc(&g->W2b, (size_t)HID * HID) || galloc(&g->W3b, (size_t)HID * HID) ||
        galloc(&g->Hb[0], (size_t)HEAD_OUT[0] * HID) || galloc(&g->Hb[1], (size_t)HEAD_OUT[1] * HID) ||
        galloc(&g->Hb[2], (size_t)HEAD_OUT[2] * HID) || galloc(&g->d_loss, 1))
        return fail(HFX_ERR_OOM);
    g->hp.assign(n, 0.0f);
    for (int k = 0; k < NFEAT; ++k) g->hp[PL.off[P_FSCALE] + k] = 1.0f;
    for (int t = 0; t < NTYPE; ++t) g->hp[PL.off[P_TSCALE] + t] = 1.0f;
    if (hipMemcpy(g->p, g->hp.data(), n * 4, hipMemcpyHostToDevice) != hipSuccess) return fail(HFX_ERR_DEVICE);
    hipLaunchKernelGGL(k_fill_f, dim3(blocks_for(n)), dim3(WG), 0, nullptr, g->m, n, 0.0f);
    hipLaunchKernelGGL(k_fill_f, dim3(blocks_for(n)), dim3(WG), 0, nullptr, g->v, n, 0.0f);
    hipLaunchKernelGGL(k_fill_f, dim3(blocks_for(n)), dim3(WG), 0, nullptr, g->gr, n, 0.0f);
    if (hipDeviceSynchronize() != hipSuccess) return fail(HFX_ERR_DEVICE);
    *out = g;
    return HFX_OK;
}

extern "C" const char* hfx_guess_last_error(const hfx_guess* g) { return g ? g->err.c_str() : "null network"; }

extern "C" hfx_status hfx_guess_set_params(hfx_guess* g, const float* params) {
    if (!g || !params) return HFX_ERR_INVALID_ARG;
    for (long long i = 0; i < PL.total; ++i)
        if (!std::isfinite(params[i])) return gfail(g, HFX_ERR_NUMERICAL, "guess: non-finite parameter");
    for (int k = 0; k < NFEAT; ++k)
        if (!(params[PL.off[P_FSCALE] + k] > 0.0f)) return gfail(g, HFX_ERR_INVALID_ARG, "guess: feature scale <= 0");
    for (int t = 0; t < NTYPE; ++t)
        if (!(params[PL.off[P_TSCALE] + t] > 0.0f)) return gfail(g, HFX_ERR_INVALID_ARG, "guess: target scale <= 0");
    NCK(hipSetDevice(g->device));
    g->hp.assign(params, params + PL.total);
    NCK(hipMemcpy(g->p, params, PL.total * 4, hipMemcpyHostToDevice));
    g->wdirty = true;
    return HFX_OK;
}

extern "C" hfx_status hfx_guess_get_params(hfx_guess* g, float* params) {
    if (!g || !params) return HFX_ERR_INVALID_ARG;
    NCK(hipSetDevice(g->device));
    NCK(hipMemcpy(params, g->p, PL.total * 4, hipMemcpyDeviceToHost));
    return HFX_OK;
}

extern "C" hfx_status hfx_guess_get_grads(hfx_guess* g, float* grads) {
    if (!g || !grads) return HFX_ERR_INVALID_ARG;
    NCK(hipSetDevice(g->device));
    NCK(hipMemcpy(grads, g->gr, PL.total * 4, hipMemcpyDeviceToHost));
    return HFX_OK;
}

static hfx_status ensure_cap(hfx_guess* g, long long M, long long ny) {
    if (M > g->cap) {
        free_acts(g);
        const long long cap = std::max<long long>(M, 1024);
        NCK(galloc(&g->Xb, cap * XLD));
        NCK(galloc(&g->H1b, cap * HID));
        NCK(galloc(&g->H2b, cap * HID));
        NCK(galloc(&g->H3b, cap * HID));
        NCK(galloc(&g->Gab, cap * HID));
        NCK(galloc(&g->Gbb, cap * HID));
        NCK(galloc(&g->Z1, cap * HID));
        NCK(galloc(&g->Z2, cap * HID));
        NCK(galloc(&g->Z3, cap * HID));
        NCK(galloc(&g->Ga, cap * HID));
        NCK(galloc(&g->Gb, cap * HID));
        g->cap = cap;
    }
    if (ny > g->ycap) {
        gfree(g->Y);
        gfree(g->dY);
        gfree(g->dYb);
        const long long cap = std::max<long long>(ny, 4096);
        NCK(galloc(&g->Y, cap));
        NCK(galloc(&g->dY, cap));
        NCK(galloc(&g->dYb, cap));
        g->ycap = cap;
    }
    return HFX_OK;
}

static hipError_t gemm(hipStream_t st, int M, int N, int K, const bf16_t* A, long long asi, long long ask,
                       const bf16_t* B, long long bsk, long long bsj, const float* bias, float* C, long long ldc,
                       bf16_t* Cb, long long ldcb, const float* Z, long long ldz, int epi) {
    if (M <= 0 || N <= 0) return hipSuccess;
    GemmArgs a{M, N, K, A, asi, ask, B, bsk, bsj, bias, C, ldc, Cb, ldcb, Z, ldz, epi};
    hipLaunchKernelGGL(k_gemm, dim3((M + GBM - 1) / GBM, (N + GBN - 1) / GBN), dim3(256), 0, st, a);
    return hipGetLastError();
}

static hipError_t pack_weights(hfx_guess* g, hipStream_t st) {
    if (!g->wdirty) return hipSuccess;
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for((long long)HID * XLD)), dim3(WG), 0, st, g->p + PL.off[P_W1], HID,
                       NFEAT, XLD, g->W1b);
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for((long long)HID * HID)), dim3(WG), 0, st, g->p + PL.off[P_W2], HID,
                       HID, HID, g->W2b);
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for((long long)HID * HID)), dim3(WG), 0, st, g->p + PL.off[P_W3], HID,
                       HID, HID, g->W3b);
    for (int t = 0; t < NTYPE; ++t)
        hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for((long long)HEAD_OUT[t] * HID)), dim3(WG), 0, st,
                           g->p + PL.off[P_H0 + 2 * t], HEAD_OUT[t], HID, HID, g->Hb[t]);
    g->wdirty = false;
    return hipGetLastError();
}

// rows of type t start at row0[t]; head outputs of type t start at yoff[t]
static void layout(const int* counts, long long* row0, long long* yoff, long long& M, long long& ny) {
    M = 0;
    ny = 0;
    for (int t = 0; t < NTYPE; ++t) {
        row0[t] = M;
        yoff[t] = ny;
        M += counts[t];
        ny += (long long)counts[t] * HEAD_OUT[t];
    }
}

static hfx_status forward(hfx_guess* g, const float* dX, const int* counts, hipStream_t st, long long* row0,
                          long long* yoff, long long& M, long long& ny) {
    for (int t = 0; t < NTYPE; ++t)
        if (counts[t] < 0) return gfail(g, HFX_ERR_INVALID_ARG, "guess: negative row count");
    layout(counts, row0, yoff, M, ny);
    hfx_status s = ensure_cap(g, M, ny);
    if (s != HFX_OK) return s;
    NCK(pack_weights(g, st));
    if (M == 0) return HFX_OK;
    hipLaunchKernelGGL(k_feat_bf16, dim3(blocks_for(M * XLD)), dim3(WG), 0, st, dX, M, g->p + PL.off[P_FMEAN],
                       g->p + PL.off[P_FSCALE], g->Xb);
    NCK(hipGetLastError());
    const float* p = g->p;
    NCK(gemm(st, (int)M, HID, NFEAT, g->Xb, XLD, 1, g->W1b, 1, XLD, p + PL.off[P_B1], g->Z1, HID, g->H1b, HID, nullptr,
             0, EPI_SILU));
    NCK(gemm(st, (int)M, HID, HID, g->H1b, HID, 1, g->W2b, 1, HID, p + PL.off[P_B2], g->Z2, HID, g->H2b, HID, nullptr,
             0, EPI_SILU));
    NCK(gemm(st, (int)M, HID, HID, g->H2b, HID, 1, g->W3b, 1, HID, p + PL.off[P_B3], g->Z3, HID, g->H3b, HID, nullptr,
             0, EPI_SILU));
    for (int t = 0; t < NTYPE; ++t)
        NCK(gemm(st, counts[t], HEAD_OUT[t], HID, g->H3b + row0[t] * HID, HID, 1, g->Hb[t], 1, HID,
                 p + PL.off[P_C0 + 2 * t], g->Y + yoff[t], HEAD_OUT[t], nullptr, 0, nullptr, 0, EPI_STORE));
    return HFX_OK;
}

extern "C" hfx_status hfx_guess_forward_dev(hfx_guess* g, const float* dX, const int* counts, float* dT,
                                            void* stream) {
    if (!g || !counts || !dT || !dX) return HFX_ERR_INVALID_ARG;
    NCK(hipSetDevice(g->device));
    hipStream_t st = (hipStream_t)stream;
    long long row0[NTYPE], yoff[NTYPE], M, ny;
    hfx_status s = forward(g, dX, counts, st, row0, yoff, M, ny);
    if (s != HFX_OK) return s;
    for (int t = 0; t < NTYPE; ++t) {
        const long long n = (long long)counts[t] * HEAD_OUT[t];
        if (n)
            hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(WG), 0, st, g->Y + yoff[t], n,
                               g->hp[PL.off[P_TSCALE] + t], dT + yoff[t]);
    }
    NCK(hipGetLastError());
    return HFX_OK;
}

extern "C" hfx_status hfx_guess_grad_dev(hfx_guess* g, const float* dX, const int* counts, const float* dT,
                                         void* stream, double* loss) {
    if (!g || !counts || !dT || !dX) return HFX_ERR_INVALID_ARG;
    NCK(hipSetDevice(g->device));
    hipStream_t st = (hipStream_t)stream;
    long long row0[NTYPE], yoff[NTYPE], M, ny;
    hfx_status s = forward(g, dX, counts, st, row0, yoff, M, ny);
    if (s != HFX_OK) return s;
    if (ny == 0) return gfail(g, HFX_ERR_INVALID_ARG, "guess: empty batch");
    hipLaunchKernelGGL(k_fill_f, dim3(blocks_for(PL.total)), dim3(WG), 0, st, g->gr, PL.total, 0.0f);
    NCK(hipMemsetAsync(g->d_loss, 0, 8, st));
    const float gs = 2.0f / (float)ny;
    float* gr = g->gr;
    for (int t = 0; t < NTYPE; ++t) {
        const long long n = (long long)counts[t] * HEAD_OUT[t];
        if (!n) continue;
        hipLaunchKernelGGL(k_mse, dim3(blocks_for(n)), dim3(WG), 0, st, g->Y + yoff[t], dT + yoff[t], n,
                           1.0f / g->hp[PL.off[P_TSCALE] + t], gs, g->dY + yoff[t], g->dYb + yoff[t], g->d_loss);
        const int nt = HEAD_OUT[t];
        // head weights: dH_t = dY_t^T H3_t; bias: column sums of dY_t
        NCK(gemm(st, nt, HID, counts[t], g->dYb + yoff[t], 1, nt, g->H3b + row0[t] * HID, HID, 1, nullptr,
                 gr + PL.off[P_H0 + 2 * t], HID, nullptr, 0, nullptr, 0, EPI_STORE));
        hipLaunchKernelGGL(k_colsum, dim3((nt + 63) / 64, (unsigned)((counts[t] + 1023) / 1024)), dim3(256), 0, st,
                           g->dY + yoff[t], (long long)counts[t], nt, (long long)nt, gr + PL.off[P_C0 + 2 * t]);
        // dZ3 (rows of type t) = (dY_t H_t) * silu'(Z3)
        NCK(gemm(st, counts[t], HID, nt, g->dYb + yoff[t], nt, 1, g->Hb[t], HID, 1, nullptr, g->Ga + row0[t] * HID,
                 HID, g->Gab + row0[t] * HID, HID, g->Z3 + row0[t] * HID, HID, EPI_DSILU));
    }
    // layer 3: dW3 = dZ3^T H2, db3, dZ2 = (dZ3 W3) * silu'(Z2)
    NCK(gemm(st, HID, HID, (int)M, g->Gab, 1, HID, g->H2b, HID, 1, nullptr, gr + PL.off[P_W3], HID, nullptr, 0,
             nullptr, 0, EPI_STORE));
    hipLaunchKernelGGL(k_colsum, dim3(HID / 64, (unsigned)((M + 1023) / 1024)), dim3(256), 0, st, g->Ga, M, HID,
                       (long long)HID, gr + PL.off[P_B3]);
    NCK(gemm(st, (int)M, HID, HID, g->Gab, HID, 1, g->W3b, HID, 1, nullptr, g->Gb, HID, g->Gbb, HID, g->Z2, HID,
             EPI_DSILU));
    // layer 2
    NCK(gemm(st, HID, HID, (int)M, g->Gbb, 1, HID, g->H1b, HID, 1, nullptr, gr + PL.off[P_W2], HID, nullptr, 0,
             nullptr, 0, EPI_STORE));
    hipLaunchKernelGGL(k_colsum, dim3(HID / 64, (unsigned)((M + 1023) / 1024)), dim3(256), 0, st, g->Gb, M, HID,
                       (long long)HID, gr + PL.off[P_B2]);
    NCK(gemm(st, (int)M, HID, HID, g->Gbb, HID, 1, g->W2b, HID, 1, nullptr, g->Ga, HID, g->Gab, HID, g->Z1, HID,
             EPI_DSILU));
    // layer 1: dW1 = dZ1^T Xstd (164 input columns), db1
    NCK(gemm(st, HID, NFEAT, (int)M, g->Gab, 1, HID, g->Xb, XLD, 1, nullptr, gr + PL.off[P_W1], NFEAT, nullptr, 0,
             nullptr, 0, EPI_STORE));
    hipLaunchKernelGGL(k_colsum, dim3(HID / 64, (unsigned)((M + 1023) / 1024)), dim3(256), 0, st, g->Ga, M, HID,
                       (long long)HID, gr + PL.off[P_B1]);
    NCK(hipGetLastError());
    if (loss) {
        double l = 0.0;
        NCK(hipMemcpyAsync(&l, g->d_loss, 8, hipMemcpyDeviceToHost, st));
        NCK(hipStreamSynchronize(st));
        *loss = l / (double)ny;
    }
    return HFX_OK;
}

extern "C" hfx_status hfx_guess_adam(hfx_guess* g, double lr, void* stream) {
    if (!g || !(lr > 0)) return g ? gfail(g, HFX_ERR_INVALID_ARG, "guess: lr must be positive") : HFX_ERR_INVALID_ARG;
    NCK(hipSetDevice(g->device));
    g->step += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)g->step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)g->step)));
    const long long n = PL.off[NTRAIN];   // weights and biases only
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(WG), 0, (hipStream_t)stream, g->p, g->gr, g->m, g->v, n,
                       (float)lr, (float)b1, (float)b2, 1e-8f, c1, c2);
    NCK(hipGetLastError());
    g->wdirty = true;
    return HFX_OK;
}

// D (device, in/out): the SAD density on entry; on success D + sum of the
// predicted blocks.  The prediction is rejected (D restored, *used = 0) when
// it is not finite or |tr(D S) - nocc| > 0.05 nocc.
extern "C" hfx_status hfx_guess_apply(hfx_ctx* c, hfx_guess* g, double* dD, void* stream, int* used) {
    if (!c || !g || !dD) return c ? hfx_fail(c, HFX_ERR_INVALID_ARG, "null pointer") : HFX_ERR_INVALID_ARG;
    if (used) *used = 0;
    hfx_status s = HFX_OK;
    if (!c->guess) {
        s = hfx_guess_setup(c, nullptr);
        if (s != HFX_OK) return s;
    }
    GuessPairsDev* G = c->guess;
    hipStream_t st = (hipStream_t)stream;
    GCK(hipSetDevice(c->opt.device));
    const size_t nn = (size_t)c->nbf * c->nbf;
    double* base = nullptr;
    GCK(galloc(&base, nn));
    hipLaunchKernelGGL(k_copy, dim3(blocks_for((long long)std::min<size_t>(nn, 1u << 22))), dim3(WG), 0, st, dD, nn,
                       base);
    s = hfx_guess_forward_dev(g, G->d_feat, G->counts, G->d_T, stream);
    if (s != HFX_OK) {
        gfree(base);
        return hfx_fail(c, s, std::string("guess network: ") + g->err);
    }
    s = hfx_guess_assemble_dev(c, G->d_T, nullptr, dD, stream);
    if (s != HFX_OK) {
        gfree(base);
        return s;
    }
    double red[2] = {0.0, 0.0};
    hipError_t e = hipMemsetAsync(G->d_red, 0, 16, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_trace_check, dim3(blocks_for((long long)std::min<size_t>(nn, 1u << 20))), dim3(WG), 0,
                           st, dD, c->d_S, nn, G->d_red);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(red, G->d_red, 16, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        gfree(base);
        return hfx_hip_check(c, e, "guess trace check");
    }
    const bool ok = red[1] == 0.0 && std::isfinite(red[0]) && std::fabs(red[0] - c->nocc) <= 0.05 * c->nocc;
    if (!ok)
        hipLaunchKernelGGL(k_copy, dim3(blocks_for((long long)std::min<size_t>(nn, 1u << 22))), dim3(WG), 0, st, base,
                           nn, dD);
    e = hipStreamSynchronize(st);
    gfree(base);
    GCK(e);
    if (used) *used = ok ? 1 : 0;
    return HFX_OK;
}
