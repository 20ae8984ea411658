// Support kernels around the class kernels: density preparation, the
// per-bra FP64/FP32 split, Fock assembly, one-electron integrals and the
// small SCF helpers.  All are HBM-bound elementwise passes or tiny.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "hfx_internal.h"

#define MISC_WG 256

// ---- per build --------------------------------------------------------------

// Matrices are stored per molecule (ragged): molecule m's nbf_m x nbf_m
// block starts at element moff[m]; its basis functions are global indices
// mboff[m] .. mboff[m] + nbf_m - 1 (component factors cs[]).  Elementwise
// kernels run on a (gx, nmol) grid, row y = molecule.

// D' = s_m s_n D (component normalisation moved onto the density),
// dmax = max |D| (bit pattern of a non-negative double is order preserving).
__global__ void k_prepare_density(const double* __restrict__ D, const double* __restrict__ cs,
                                  const long long* __restrict__ moff, const int* __restrict__ mdim,
                                  const int* __restrict__ mboff, double* __restrict__ Dp,
                                  unsigned long long* __restrict__ dmax_bits) {
    const int mol = blockIdx.y;
    const int n = mdim[mol];
    const size_t nn = (size_t)n * n, base = (size_t)moff[mol];
    const double* __restrict__ c = cs + mboff[mol];
    double mx = 0.0;
    for (size_t i = (size_t)blockIdx.x * MISC_WG + threadIdx.x; i < nn; i += (size_t)gridDim.x * MISC_WG) {
        const double d = D[base + i];
        Dp[base + i] = c[i / n] * c[i % n] * d;
        const double ad = fabs(d);
        mx = (ad > mx || ad != ad) ? ad : mx;   // NaN propagates
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_xor(mx, off, 64);
        mx = (o > mx || o != o) ? o : mx;
    }
    if ((threadIdx.x & 63) == 0 && dmax_bits) {
        unsigned long long b = mx != mx ? 0x7ff8000000000000ull : (unsigned long long)__double_as_longlong(mx);
        atomicMax(dmax_bits, b);
    }
}

__global__ void k_fill(double* __restrict__ p, size_t n, double v) {
    for (size_t i = (size_t)blockIdx.x * MISC_WG + threadIdx.x; i < n; i += (size_t)gridDim.x * MISC_WG) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* __restrict__ p, int n) {
    const int i = blockIdx.x * MISC_WG + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// FP64/FP32 split per task (bra r, kets [s0, s1) of one group): the kets s
// with Q_r Q_s max|D| >= fp32_tau come first (Q descending within a group);
// split[t] is the list position of the first FP32 ket (s1 if none).
__global__ void k_split(const PairInfo* __restrict__ bra, const double* __restrict__ ketq,
                        const int4* __restrict__ tasks, int ntask, double fp32_tau,
                        const unsigned long long* __restrict__ dmax_bits, int* __restrict__ split) {
    const int t = blockIdx.x * MISC_WG + threadIdx.x;
    if (t >= ntask) return;
    const int4 tk = tasks[t];
    if (tk.x < 0) {
        split[t] = 0;
        return;
    }
    const double qr = bra[tk.x].Q * __longlong_as_double((long long)*dmax_bits);
    int lo = tk.y, hi = tk.z;   // Q descending within a task's kets: the FP32 ones are a suffix
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ketq[mid] * qr >= fp32_tau) lo = mid + 1; else hi = mid;
    }
    split[t] = lo;
}

// F = H + s_m s_n (W + W^T) / 8 per molecule block (H may be null: two-electron
// part only); raises *bad if a non-finite value appears.
__global__ void k_assemble(const double* __restrict__ H, const double* __restrict__ W, const double* __restrict__ cs,
                           const long long* __restrict__ moff, const int* __restrict__ mdim,
                           const int* __restrict__ mboff, double* __restrict__ F, int* __restrict__ bad) {
    const int mol = blockIdx.y;
    const int n = mdim[mol];
    const size_t nn = (size_t)n * n, base = (size_t)moff[mol];
    const double* __restrict__ c = cs + mboff[mol];
    for (size_t i = (size_t)blockIdx.x * MISC_WG + threadIdx.x; i < nn; i += (size_t)gridDim.x * MISC_WG) {
        const size_t r = i / n, col = i % n;
        const double g = 0.125 * c[r] * c[col] * (W[base + i] + W[base + col * n + r]);
        const double f = (H ? H[base + i] : 0.0) + g;
        F[base + i] = f;
        if (!isfinite(f) && bad) *bad = 1;
    }
}

// W += sum of the nrep private copies of W (replica x at x * n): the
// reduction of algorithm 2's private Fock matrices, here one per XCD.
__global__ void k_reduce_replicas(const double* __restrict__ rep, int nrep, size_t n, double* __restrict__ W) {
    for (size_t i = (size_t)blockIdx.x * MISC_WG + threadIdx.x; i < n; i += (size_t)gridDim.x * MISC_WG) {
        double v = 0.0;
        for (int x = 0; x < nrep; ++x) v += rep[(size_t)x * n + i];
        W[i] += v;
    }
}

// dket[comp][s] = D'_cd of ket pair s of one list (component comp of its
// block), so that the class kernels read it coalesced by ket position.
__global__ void k_gather_ket(const PairInfo* __restrict__ kets, int n, int nc, int nd, const double* __restrict__ D,
                             const long long* __restrict__ moff, double* __restrict__ dket) {
    const int i = blockIdx.x * MISC_WG + threadIdx.x;
    if (i >= n * nc * nd) return;
    const int s = i % n, comp = i / n;
    const PairInfo p = kets[s];
    dket[i] = D[(size_t)moff[p.mol] + (size_t)(p.bfa + comp / nd) * p.ld + p.bfb + comp % nd];
}

// W_cd += wket[comp][s] for every ket pair s of one list: each pair owns its
// W block, so plain read-modify-write (no atomics) after the class kernels.
__global__ void k_scatter_ket(const PairInfo* __restrict__ kets, int n, int nc, int nd,
                              const double* __restrict__ wket, const long long* __restrict__ moff,
                              double* __restrict__ W) {
    const int i = blockIdx.x * MISC_WG + threadIdx.x;
    if (i >= n * nc * nd) return;
    const int s = i % n, comp = i / n;
    const double v = wket[i];
    if (v == 0.0) return;
    const PairInfo p = kets[s];
    const size_t idx = (size_t)moff[p.mol] + (size_t)(p.bfa + comp / nd) * p.ld + p.bfb + comp % nd;
    W[idx] += v;
}

// ---- one-electron integrals (Obara-Saika) ------------------------------------
// One thread per shell pair (a >= b).  Overlap from the 1-D recursion
//   S_{i+1,j} = X_PA S_ij + (i S_{i-1,j} + j S_{i,j-1})/(2p), same for j with X_PB;
// kinetic from -1/2 d^2/dx^2 acting on the ket Gaussian:
//   T_ij = -1/2 [ j(j-1) S_{i,j-2} - 2 beta (2j+1) S_ij + 4 beta^2 S_{i,j+2} ];
// nuclear attraction from the vertical recursion on centre A,
//   [a+1_i]^(m) = PA_i [a]^(m) - PC_i [a]^(m+1) + a_i/(2p) ([a-1_i]^(m) - [a-1_i]^(m+1)),
//   [0]^(m) = 2 pi / p exp(-alpha beta/p |AB|^2) F_m(p |PC|^2),
// then the transfer (a|b+1_i) = (a+1_i|b) + AB_i (a|b).
struct ShellDev {
    double x, y, z;
    int l, nprim, prim_off, bf;
};

__device__ __forceinline__ int cart_index(int x, int y, int z) {   // lexicographic index within |l|
    const int l = x + y + z;
    (void)l;
    const int yz = y + z;
    return yz * (yz + 1) / 2 + z;
}

__device__ __forceinline__ void cart_comp_dev(int l, int c, int* e) {
    int k = 0;
    for (int x = l; x >= 0; --x)
        for (int y = l - x; y >= 0; --y) {
            if (k == c) { e[0] = x; e[1] = y; e[2] = l - x - y; return; }
            ++k;
        }
}

__global__ void k_one_electron(const ShellDev* __restrict__ sh, int nshell, const double* __restrict__ exps,
                               const double* __restrict__ coefs, const double* __restrict__ atoms /*x,y,z,Z*/,
                               int natom, const double* __restrict__ cs, const double* __restrict__ boys, int n,
                               double* __restrict__ S, double* __restrict__ T, double* __restrict__ V) {
    const long long pid = (long long)blockIdx.x * MISC_WG + threadIdx.x;
    const long long npair = (long long)nshell * (nshell + 1) / 2;
    if (pid >= npair) return;
    int a = (int)((sqrt(8.0 * (double)pid + 1.0) - 1.0) * 0.5);
    while ((long long)a * (a + 1) / 2 > pid) --a;
    while ((long long)(a + 1) * (a + 2) / 2 <= pid) ++a;
    const int b = (int)(pid - (long long)a * (a + 1) / 2);
    const ShellDev A = sh[a], B = sh[b];
    const int la = A.l, lb = B.l, na = (la + 1) * (la + 2) / 2, nb = (lb + 1) * (lb + 2) / 2;
    const double Ap[3] = {A.x, A.y, A.z}, Bp[3] = {B.x, B.y, B.z};
    const double AB[3] = {A.x - B.x, A.y - B.y, A.z - B.z};
    const double ab2 = AB[0] * AB[0] + AB[1] * AB[1] + AB[2] * AB[2];
    double s_acc[36], t_acc[36], v_acc[36];
    for (int i = 0; i < 36; ++i) s_acc[i] = t_acc[i] = v_acc[i] = 0.0;
    for (int ia = 0; ia < A.nprim; ++ia)
        for (int ib = 0; ib < B.nprim; ++ib) {
            const double al = exps[A.prim_off + ia], be = exps[B.prim_off + ib];
            const double cc = coefs[A.prim_off + ia] * coefs[B.prim_off + ib];
            const double p = al + be, i2p = 0.5 / p, mu = al * be / p;
            const double P[3] = {(al * A.x + be * B.x) / p, (al * A.y + be * B.y) / p, (al * A.z + be * B.z) / p};
            const double kab = exp(-mu * ab2);
            // 1-D overlaps S[x][i][j], i <= 2, j <= 4
            double S1[3][3][5];
            for (int x = 0; x < 3; ++x) {
                const double PA = P[x] - Ap[x], PB = P[x] - Bp[x];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 5; ++j) S1[x][i][j] = 0.0;
                S1[x][0][0] = sqrt(M_PI / p);
                for (int i = 0; i <= la; ++i) {
                    if (i > 0)
                        S1[x][i][0] = PA * S1[x][i - 1][0] + (i - 1 > 0 ? (i - 1) * i2p * S1[x][i - 2][0] : 0.0);
                    for (int j = 1; j <= lb + 2; ++j)
                        S1[x][i][j] = PB * S1[x][i][j - 1] + i2p * ((i > 0 ? i * S1[x][i - 1][j - 1] : 0.0) +
                                                                     (j - 1 > 0 ? (j - 1) * S1[x][i][j - 2] : 0.0));
                }
            }
            // nuclear attraction: [e]^(m), |e| <= la+lb <= 4, m <= 4
            const int L = la + lb;
            const int off[6] = {0, 1, 4, 10, 20, 35};
            double Vacc[35];   // sum over nuclei of -Z [e]^(0), indexed by total order blocks
            for (int i = 0; i < 35; ++i) Vacc[i] = 0.0;
            for (int c = 0; c < natom; ++c) {
                const double Z = atoms[4 * c + 3];
                if (Z == 0.0) continue;
                const double PC[3] = {P[0] - atoms[4 * c], P[1] - atoms[4 * c + 1], P[2] - atoms[4 * c + 2]};
                const double Tc = p * (PC[0] * PC[0] + PC[1] * PC[1] + PC[2] * PC[2]);
                double F[5];
                boys_eval<double, 4>(Tc, F, boys + (size_t)boys_block(4) * BOYS_NT * BOYS_ROW);
                // e laid out as [lvl][comp] with offsets 0,1,4,10,20 ; m in [0..L-lvl]
                double th[35][5];
                const double pre = 2.0 * M_PI / p * kab;
                for (int m = 0; m <= L; ++m) th[0][m] = pre * F[m];
                for (int lvl = 1; lvl <= L; ++lvl) {
                    const int nc = (lvl + 1) * (lvl + 2) / 2;
                    for (int k = 0; k < nc; ++k) {
                        int e[3];
                        cart_comp_dev(lvl, k, e);
                        int dir = e[0] > 0 ? 0 : (e[1] > 0 ? 1 : 2);
                        int e1[3] = {e[0], e[1], e[2]};
                        e1[dir] -= 1;
                        const int i1 = off[lvl - 1] + cart_index(e1[0], e1[1], e1[2]);
                        int i2 = -1;
                        if (e1[dir] > 0) {
                            int e2[3] = {e1[0], e1[1], e1[2]};
                            e2[dir] -= 1;
                            i2 = off[lvl - 2] + cart_index(e2[0], e2[1], e2[2]);
                        }
                        const double PAd = P[dir] - Ap[dir];
                        for (int m = 0; m <= L - lvl; ++m) {
                            double v = PAd * th[i1][m] - PC[dir] * th[i1][m + 1];
                            if (i2 >= 0) v += e1[dir] * i2p * (th[i2][m] - th[i2][m + 1]);
                            th[off[lvl] + k][m] = v;
                        }
                    }
                }
                for (int i = 0; i < off[L + 1]; ++i) Vacc[i] -= Z * th[i][0];
            }
            // assemble the Cartesian blocks
            for (int mu = 0; mu < na; ++mu)
                for (int nu = 0; nu < nb; ++nu) {
                    int ea[3], eb[3];
                    cart_comp_dev(la, mu, ea);
                    cart_comp_dev(lb, nu, eb);
                    double s3 = 1.0, t3 = 0.0;
                    double sx[3], tx[3];
                    for (int x = 0; x < 3; ++x) {
                        const int i = ea[x], j = eb[x];
                        sx[x] = S1[x][i][j];
                        tx[x] = -0.5 * ((j >= 2 ? j * (j - 1) * S1[x][i][j - 2] : 0.0) -
                                        2.0 * be * (2 * j + 1) * S1[x][i][j] + 4.0 * be * be * S1[x][i][j + 2]);
                    }
                    s3 = sx[0] * sx[1] * sx[2];
                    t3 = tx[0] * sx[1] * sx[2] + sx[0] * tx[1] * sx[2] + sx[0] * sx[1] * tx[2];
                    // transfer: (ea | eb) from [e] with |e| >= la via (a|b+1_i) = (a+1_i|b) + AB_i (a|b)
                    // expand (x-B)^j = sum_k C(j,k) (x-A)^{j-k} (A-B)^k per axis
                    double vv = 0.0;
                    for (int kx = 0; kx <= eb[0]; ++kx)
                        for (int ky = 0; ky <= eb[1]; ++ky)
                            for (int kz = 0; kz <= eb[2]; ++kz) {
                                const int ex = ea[0] + eb[0] - kx, ey = ea[1] + eb[1] - ky, ez = ea[2] + eb[2] - kz;
                                const int lvl = ex + ey + ez;
                                const double binx = (kx == 0 || kx == eb[0]) ? 1.0 : (double)eb[0];
                                const double biny = (ky == 0 || ky == eb[1]) ? 1.0 : (double)eb[1];
                                const double binz = (kz == 0 || kz == eb[2]) ? 1.0 : (double)eb[2];
                                const double f = binx * biny * binz * pow(AB[0], kx) * pow(AB[1], ky) * pow(AB[2], kz);
                                vv += f * Vacc[off[lvl] + cart_index(ex, ey, ez)];
                            }
                    const double k3 = kab;   // overlap/kinetic carry exp(-mu AB^2) once (3-D product)
                    s_acc[mu * nb + nu] += cc * k3 * s3;
                    t_acc[mu * nb + nu] += cc * k3 * t3;
                    v_acc[mu * nb + nu] += cc * vv;
                }
        }
    for (int mu = 0; mu < na; ++mu)
        for (int nu = 0; nu < nb; ++nu) {
            const int r = A.bf + mu, c = B.bf + nu;
            const double sc = cs[r] * cs[c];
            const double sv = sc * s_acc[mu * nb + nu], tv = sc * t_acc[mu * nb + nu], vv = sc * v_acc[mu * nb + nu];
            S[(size_t)r * n + c] = sv; S[(size_t)c * n + r] = sv;
            T[(size_t)r * n + c] = tv; T[(size_t)c * n + r] = tv;
            V[(size_t)r * n + c] = vv; V[(size_t)c * n + r] = vv;
        }
}

// ---- SCF helpers ------------------------------------------------------------------

// out = A - A^T (column- or row-major alike)
__global__ void k_antisym(const double* __restrict__ A, int n, double* __restrict__ out) {
    const size_t nn = (size_t)n * n;
    for (size_t i = (size_t)blockIdx.x * MISC_WG + threadIdx.x; i < nn; i += (size_t)gridDim.x * MISC_WG) {
        const size_t r = i / n, c = i % n;
        out[i] = A[i] - A[c * n + r];
    }
}

// partial sums of sum_i a_i * b_i (b may be null: sum a_i^2) and of (a_i - b_i)^2 (mode 1)
__global__ void k_dot(const double* __restrict__ a, const double* __restrict__ b, size_t n, int mode,
                      double* __restrict__ out) {
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * MISC_WG + threadIdx.x; i < n; i += (size_t)gridDim.x * MISC_WG) {
        if (mode == 0) acc += a[i] * b[i];
        else { const double d = a[i] - b[i]; acc += d * d; }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __shared__ double red[MISC_WG / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < MISC_WG / 64; ++w) s += red[w];
        out[blockIdx.x] = s;
    }
}

// E-term: sum_ij D_ij (H_ij + F_ij)
__global__ void k_energy(const double* __restrict__ D, const double* __restrict__ H, const double* __restrict__ F,
                         size_t n, double* __restrict__ out) {
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * MISC_WG + threadIdx.x; i < n; i += (size_t)gridDim.x * MISC_WG)
        acc += D[i] * (H[i] + F[i]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __shared__ double red[MISC_WG / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < MISC_WG / 64; ++w) s += red[w];
        out[blockIdx.x] = s;
    }
}

// out = sum_k c_k M_k (k < m), matrices of size n
__global__ void k_lincomb(const double* const* __restrict__ M, const double* __restrict__ c, int m, size_t n,
                          double* __restrict__ out) {
    for (size_t i = (size_t)blockIdx.x * MISC_WG + threadIdx.x; i < n; i += (size_t)gridDim.x * MISC_WG) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += c[k] * M[k][i];
        out[i] = s;
    }
}

// X (column-major n x nk) from eigenpairs of S: symmetric S^{-1/2} when
// nothing is dropped, canonical U_k w_k^{-1/2} otherwise.
__global__ void k_scale_cols(const double* __restrict__ U, const double* __restrict__ w, const int* __restrict__ keep,
                             int n, int nk, double* __restrict__ out) {
    const size_t tot = (size_t)n * nk;
    for (size_t i = (size_t)blockIdx.x * MISC_WG + threadIdx.x; i < tot; i += (size_t)gridDim.x * MISC_WG) {
        const int col = (int)(i / n), row = (int)(i % n);
        const int src = keep[col];
        out[i] = U[(size_t)src * n + row] / sqrt(w[src]);
    }
}

// Batched eigensolves over molecules of different sizes: slot m (NP x NP) of
// dst holds molecule m's block (n_m x n_m) in its top-left corner, `pad` on
// the rest of the diagonal and zeros elsewhere, so that the slot's
// eigenpairs are the block's plus (pad, unit vectors), sorted after them.
__global__ void k_pad_blocks(const double* __restrict__ src, const long long* __restrict__ moff,
                             const int* __restrict__ dim, int NP, double pad, double* __restrict__ dst) {
    const int mol = blockIdx.y;
    const int n = dim[mol];
    const size_t tot = (size_t)NP * NP;
    double* __restrict__ d = dst + (size_t)mol * tot;
    for (size_t i = (size_t)blockIdx.x * MISC_WG + threadIdx.x; i < tot; i += (size_t)gridDim.x * MISC_WG) {
        const int r = (int)(i / NP), col = (int)(i % NP);
        d[i] = (r < n && col < n) ? src[moff[mol] + (size_t)r * n + col] : (r == col ? pad : 0.0);
    }
}

// Outside the top-left k_m x k_m block of every slot: pad on the diagonal, zeros elsewhere.
__global__ void k_pad_rest(const int* __restrict__ dim, int NP, double pad, double* __restrict__ dst) {
    const int mol = blockIdx.y;
    const int k = dim[mol];
    const size_t tot = (size_t)NP * NP;
    double* __restrict__ d = dst + (size_t)mol * tot;
    for (size_t i = (size_t)blockIdx.x * MISC_WG + threadIdx.x; i < tot; i += (size_t)gridDim.x * MISC_WG) {
        const int r = (int)(i / NP), col = (int)(i % NP);
        if (r >= k || col >= k) d[i] = (r == col) ? pad : 0.0;
    }
}

// C (column-major n x nmo) -> weighted density D = sum_k occ_k C_k C_k^T
__global__ void k_weight_cols(const double* __restrict__ C, const double* __restrict__ occ, int n, int nk,
                              double* __restrict__ out) {
    const size_t tot = (size_t)n * nk;
    for (size_t i = (size_t)blockIdx.x * MISC_WG + threadIdx.x; i < tot; i += (size_t)gridDim.x * MISC_WG)
        out[i] = C[i] * occ[i / n];
}

// ---- C wrappers ---------------------------------------------------------------------

static int grid_for(size_t n) {
    size_t g = (n + MISC_WG - 1) / MISC_WG;
    if (g > 4096) g = 4096;
    return (int)(g ? g : 1);
}

extern "C" {
static dim3 ragged_grid(int max_ld, int nmol) {
    size_t g = ((size_t)max_ld * max_ld + MISC_WG - 1) / MISC_WG;
    if (g > 4096) g = 4096;
    return dim3((unsigned)(g ? g : 1), (unsigned)nmol);
}
hipError_t hfx_prepare_density(const double* D, const double* cs, int nmol, const long long* moff, const int* mdim,
                               const int* mboff, int max_ld, double* Dp, unsigned long long* dmax_bits,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_prepare_density, ragged_grid(max_ld, nmol), dim3(MISC_WG), 0, st, D, cs, moff, mdim, mboff, Dp,
                       dmax_bits);
    return hipGetLastError();
}
hipError_t hfx_fill(double* p, size_t n, double v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(MISC_WG), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t hfx_reduce_replicas(const double* rep, int nrep, size_t n, double* W, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_replicas, dim3(grid_for(n)), dim3(MISC_WG), 0, st, rep, nrep, n, W);
    return hipGetLastError();
}
hipError_t hfx_fill_u64(unsigned long long* p, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3((n + MISC_WG - 1) / MISC_WG), dim3(MISC_WG), 0, st, p, n);
    return hipGetLastError();
}
hipError_t hfx_split(const PairInfo* bra, const double* ketq, const int4* tasks, int ntask, double fp32_tau,
                     const unsigned long long* dmax_bits, int* split, hipStream_t st) {
    if (ntask <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_split, dim3((ntask + MISC_WG - 1) / MISC_WG), dim3(MISC_WG), 0, st, bra, ketq, tasks,
                       ntask, fp32_tau, dmax_bits, split);
    return hipGetLastError();
}
hipError_t hfx_gather_ket(const PairInfo* kets, int n, int nc, int nd, const double* D, const long long* moff,
                          double* dket, hipStream_t st) {
    const int tot = n * nc * nd;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_ket, dim3((tot + MISC_WG - 1) / MISC_WG), dim3(MISC_WG), 0, st, kets, n, nc, nd, D, moff,
                       dket);
    return hipGetLastError();
}
hipError_t hfx_scatter_ket(const PairInfo* kets, int n, int nc, int nd, const double* wket, const long long* moff,
                           double* W, hipStream_t st) {
    const int tot = n * nc * nd;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_ket, dim3((tot + MISC_WG - 1) / MISC_WG), dim3(MISC_WG), 0, st, kets, n, nc, nd, wket,
                       moff, W);
    return hipGetLastError();
}
hipError_t hfx_assemble(const double* H, const double* W, const double* cs, int nmol, const long long* moff,
                        const int* mdim, const int* mboff, int max_ld, double* F, int* bad, hipStream_t st) {
    hipLaunchKernelGGL(k_assemble, ragged_grid(max_ld, nmol), dim3(MISC_WG), 0, st, H, W, cs, moff, mdim, mboff, F, bad);
    return hipGetLastError();
}
hipError_t hfx_one_electron(const void* sh, int nshell, const double* exps, const double* coefs, const double* atoms,
                            int natom, const double* cs, const double* boys, int n, double* S, double* T, double* V,
                            hipStream_t st) {
    const long long npair = (long long)nshell * (nshell + 1) / 2;
    if (npair == 0) return hipSuccess;
    hipLaunchKernelGGL(k_one_electron, dim3((unsigned)((npair + MISC_WG - 1) / MISC_WG)), dim3(MISC_WG), 0, st,
                       (const ShellDev*)sh, nshell, exps, coefs, atoms, natom, cs, boys, n, S, T, V);
    return hipGetLastError();
}
hipError_t hfx_antisym(const double* A, int n, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_antisym, dim3(grid_for((size_t)n * n)), dim3(MISC_WG), 0, st, A, n, out);
    return hipGetLastError();
}
// returns the number of partial sums written to out (<= 4096)
int hfx_dot_partial(const double* a, const double* b, size_t n, int mode, double* out, hipStream_t st) {
    const int g = grid_for(n);
    hipLaunchKernelGGL(k_dot, dim3(g), dim3(MISC_WG), 0, st, a, b, n, mode, out);
    return g;
}
int hfx_energy_partial(const double* D, const double* H, const double* F, size_t n, double* out, hipStream_t st) {
    const int g = grid_for(n);
    hipLaunchKernelGGL(k_energy, dim3(g), dim3(MISC_WG), 0, st, D, H, F, n, out);
    return g;
}
hipError_t hfx_lincomb(const double* const* M, const double* c, int m, size_t n, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_lincomb, dim3(grid_for(n)), dim3(MISC_WG), 0, st, M, c, m, n, out);
    return hipGetLastError();
}
hipError_t hfx_scale_cols(const double* U, const double* w, const int* keep, int n, int nk, double* out,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_scale_cols, dim3(grid_for((size_t)n * nk)), dim3(MISC_WG), 0, st, U, w, keep, n, nk, out);
    return hipGetLastError();
}
hipError_t hfx_pad_blocks(const double* src, const long long* moff, const int* dim, int nmol, int NP, double pad,
                          double* dst, hipStream_t st) {
    const unsigned gx = (unsigned)std::min<size_t>(((size_t)NP * NP + MISC_WG - 1) / MISC_WG, 1024);
    hipLaunchKernelGGL(k_pad_blocks, dim3(gx, nmol), dim3(MISC_WG), 0, st, src, moff, dim, NP, pad, dst);
    return hipGetLastError();
}
hipError_t hfx_pad_rest(const int* dim, int nmol, int NP, double pad, double* dst, hipStream_t st) {
    const unsigned gx = (unsigned)std::min<size_t>(((size_t)NP * NP + MISC_WG - 1) / MISC_WG, 1024);
    hipLaunchKernelGGL(k_pad_rest, dim3(gx, nmol), dim3(MISC_WG), 0, st, dim, NP, pad, dst);
    return hipGetLastError();
}
hipError_t hfx_weight_cols(const double* C, const double* occ, int n, int nk, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_weight_cols, dim3(grid_for((size_t)n * nk)), dim3(MISC_WG), 0, st, C, occ, n, nk, out);
    return hipGetLastError();
}
}
