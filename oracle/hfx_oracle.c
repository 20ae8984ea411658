/*
 * hfx_oracle.c -- plain, slow, FP64 reference for the closed-shell
 * Hartree-Fock Fock build.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code with the HIP library: it uses a different integral algorithm
 * (McMurchie-Davidson Hermite expansion; the GPU path uses Obara-Saika /
 * Head-Gordon-Pople recurrences) and its own normalisation, Boys function
 * and screening code.
 *
 * What it computes (paper: section 3 and section 4.1, eq. 2):
 *   - Cartesian Gaussian basis functions, each component normalised to one,
 *     contractions renormalised to unit self-overlap;
 *   - one-electron integrals S, T, V and the nuclear repulsion energy;
 *   - electron repulsion integrals (mu nu | lambda sigma) in chemists'
 *     notation, one contracted shell quartet at a time;
 *   - Schwarz bounds Q_ab = sqrt(max (mu nu|mu nu)) (Cauchy-Schwarz
 *     screening, section 4.1);
 *   - J_{mn} = sum_{ls} (mn|ls) D_ls and K_{mn} = sum_{ls} (ml|ns) D_ls in
 *     three ways: brute force over every ordered shell quartet; the
 *     8-fold-symmetric loop over unique shell quartets with the six updates
 *     of eq. 2 (algorithm 1's loop nest, with the l-limit read as
 *     "l <= (k == i ? j : k)"); and one shell block straight from the
 *     definition (for sampled checks on large systems).
 *
 * All routines are plain loops in FP64.  The one concession to speed is an
 * OpenMP loop over bra shell pairs with thread-private J/K (the private-Fock
 * pattern of algorithm 2), which changes only the order of the final sums.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_LMAX 4                 /* per shell */
#define ORC_LTOT (4 * ORC_LMAX)    /* per quartet */
#define ORC_NCMAX 15               /* Cartesian components of l = 4 */

typedef struct {
    int natom;
    int *Z;
    double *axyz;     /* natom*3 */
    int nshell;
    int *l, *np, *off, *atom, *bf;
    double *cxyz;     /* nshell*3 */
    double *exps;     /* primitive exponents */
    double *coefs;    /* coefficient * primitive norm (x^l component) * contraction renorm */
    int nbf;
} orc_basis;

/* ---- small helpers ------------------------------------------------------ */

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

/* Cartesian exponents of component c of shell l, lexicographic order. */
static void cart_comp(int l, int c, int *lx, int *ly, int *lz) {
    int k = 0;
    *lx = *ly = *lz = 0;
    for (int x = l; x >= 0; --x)
        for (int y = l - x; y >= 0; --y) {
            if (k == c) { *lx = x; *ly = y; *lz = l - x - y; return; }
            ++k;
        }
}

static double dfact_odd(int n) { /* (2n-1)!! for n >= 0 */
    double r = 1.0;
    for (int k = 2 * n - 1; k > 1; k -= 2) r *= k;
    return r;
}

/* Per-component factor 1/sqrt((2lx-1)!!(2ly-1)!!(2lz-1)!!). */
static double comp_scale(int l, int c) {
    int x, y, z;
    cart_comp(l, c, &x, &y, &z);
    return 1.0 / sqrt(dfact_odd(x) * dfact_odd(y) * dfact_odd(z));
}

/* ---- Boys function --------------------------------------------------------
 * F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt.
 * T < 30: the convergent series F_m(T) = e^{-T} sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1)),
 * evaluated separately for every m.
 * T >= 30: F_0 = sqrt(pi/T) erf(sqrt T) / 2 and the upward recursion
 * F_{m+1} = ((2m+1) F_m - e^{-T}) / (2T), which is stable for T >> m.       */
void orc_boys(int mmax, double T, double *F) {
    if (T < 30.0) {
        double eT = exp(-T);
        for (int m = 0; m <= mmax; ++m) {
            double term = 1.0 / (2 * m + 1), sum = term;
            for (int k = 1; k < 2000; ++k) {
                term *= 2.0 * T / (2 * m + 2 * k + 1);
                sum += term;
                if (term < 1e-18 * sum) break;
            }
            F[m] = eT * sum;
        }
    } else {
        double eT = exp(-T);
        F[0] = 0.5 * sqrt(M_PI / T) * erf(sqrt(T));
        for (int m = 0; m < mmax; ++m) F[m + 1] = ((2 * m + 1) * F[m] - eT) / (2.0 * T);
    }
}

/* ---- basis construction ---------------------------------------------------- */

static double prim_norm(double a, int l) {     /* (2a/pi)^{3/4} (4a)^{l/2} */
    return pow(2.0 * a / M_PI, 0.75) * pow(4.0 * a, 0.5 * l);
}

orc_basis *orc_basis_new(int natom, const int *Z, const double *axyz, int nshell,
                         const int *sh_atom, const int *sh_l, const int *sh_np,
                         const int *sh_off, const double *exps, const double *coefs) {
    orc_basis *b = (orc_basis *)calloc(1, sizeof(orc_basis));
    int nprim = 0;
    for (int s = 0; s < nshell; ++s) {
        if (sh_l[s] < 0 || sh_l[s] > ORC_LMAX || sh_np[s] < 1) { free(b); return NULL; }
        if (sh_off[s] + sh_np[s] > nprim) nprim = sh_off[s] + sh_np[s];
    }
    b->natom = natom;
    b->Z = (int *)malloc(sizeof(int) * (natom > 0 ? natom : 1));
    b->axyz = (double *)malloc(sizeof(double) * 3 * (natom > 0 ? natom : 1));
    memcpy(b->Z, Z, sizeof(int) * natom);
    memcpy(b->axyz, axyz, sizeof(double) * 3 * natom);
    b->nshell = nshell;
    b->l = (int *)malloc(sizeof(int) * nshell);
    b->np = (int *)malloc(sizeof(int) * nshell);
    b->off = (int *)malloc(sizeof(int) * nshell);
    b->atom = (int *)malloc(sizeof(int) * nshell);
    b->bf = (int *)malloc(sizeof(int) * nshell);
    b->cxyz = (double *)malloc(sizeof(double) * 3 * nshell);
    b->exps = (double *)malloc(sizeof(double) * (nprim > 0 ? nprim : 1));
    b->coefs = (double *)malloc(sizeof(double) * (nprim > 0 ? nprim : 1));
    int nbf = 0;
    for (int s = 0; s < nshell; ++s) {
        b->l[s] = sh_l[s];
        b->np[s] = sh_np[s];
        b->off[s] = sh_off[s];
        b->atom[s] = sh_atom[s];
        b->bf[s] = nbf;
        nbf += ncart(sh_l[s]);
        for (int x = 0; x < 3; ++x) b->cxyz[3 * s + x] = axyz[3 * sh_atom[s] + x];
        int l = sh_l[s];
        /* primitive norms, then renormalise the contraction: the x^l component
         * sum_k c_k N_k x^l exp(-a_k r^2) / sqrt((2l-1)!!) must have unit
         * self-overlap; <x^l e^{-a r^2} | x^l e^{-b r^2}> = (2l-1)!!/(2p)^l (pi/p)^{3/2}. */
        double ss = 0.0;
        for (int i = 0; i < sh_np[s]; ++i)
            for (int j = 0; j < sh_np[s]; ++j) {
                double ai = exps[sh_off[s] + i], aj = exps[sh_off[s] + j], p = ai + aj;
                double ov = 1.0 / pow(2.0 * p, l) * pow(M_PI / p, 1.5);
                ss += coefs[sh_off[s] + i] * coefs[sh_off[s] + j] * prim_norm(ai, l) * prim_norm(aj, l) * ov;
            }
        double renorm = 1.0 / sqrt(ss);
        for (int i = 0; i < sh_np[s]; ++i) {
            double a = exps[sh_off[s] + i];
            b->exps[sh_off[s] + i] = a;
            b->coefs[sh_off[s] + i] = coefs[sh_off[s] + i] * prim_norm(a, l) * renorm;
        }
    }
    b->nbf = nbf;
    return b;
}

void orc_basis_free(orc_basis *b) {
    if (!b) return;
    free(b->Z); free(b->axyz); free(b->l); free(b->np); free(b->off); free(b->atom);
    free(b->bf); free(b->cxyz); free(b->exps); free(b->coefs); free(b);
}

int orc_nbf(const orc_basis *b) { return b->nbf; }

void orc_shell_bf(const orc_basis *b, int *bf) { memcpy(bf, b->bf, sizeof(int) * b->nshell); }

/* ---- McMurchie-Davidson building blocks ------------------------------------
 * Hermite expansion coefficients E^{ij}_t of the 1-D Gaussian product
 * (x-A)^i e^{-a(x-A)^2} (x-B)^j e^{-b(x-B)^2} = sum_t E^{ij}_t Lambda_t(x),
 * Lambda_t = (d/dP_x)^t e^{-p(x-P)^2}, from E^{00}_0 = exp(-ab/p X_AB^2) and
 *   E^{i+1,j}_t = E^{ij}_{t-1}/(2p) + X_PA E^{ij}_t + (t+1) E^{ij}_{t+1}
 *   E^{i,j+1}_t = E^{ij}_{t-1}/(2p) + X_PB E^{ij}_t + (t+1) E^{ij}_{t+1}     */
#define EI 7
#define ET 15
typedef double Etab[EI][EI][ET];

static double eget(Etab E, int i, int j, int t) {
    if (t < 0 || t > i + j) return 0.0;
    return E[i][j][t];
}

static void hermite_E(int imax, int jmax, double a, double b, double XAB, Etab E) {
    double p = a + b, mu = a * b / p;
    double XPA = -b / p * XAB, XPB = a / p * XAB;
    memset(E, 0, sizeof(Etab));
    E[0][0][0] = exp(-mu * XAB * XAB);
    for (int i = 0; i < imax; ++i)
        for (int t = 0; t <= i + 1; ++t)
            E[i + 1][0][t] = eget(E, i, 0, t - 1) / (2.0 * p) + XPA * eget(E, i, 0, t) +
                             (t + 1) * eget(E, i, 0, t + 1);
    for (int i = 0; i <= imax; ++i)
        for (int j = 0; j < jmax; ++j)
            for (int t = 0; t <= i + j + 1; ++t)
                E[i][j + 1][t] = eget(E, i, j, t - 1) / (2.0 * p) + XPB * eget(E, i, j, t) +
                                 (t + 1) * eget(E, i, j, t + 1);
}

/* Hermite Coulomb integrals R_{tuv}(alpha, X, Y, Z) for t+u+v <= L:
 *   R^n_{000} = (-2 alpha)^n F_n(alpha (X^2+Y^2+Z^2))
 *   R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X R^{n+1}_{t,u,v}   (same for u/Y, v/Z)
 * R is returned as R[(t*(L+1) + u)*(L+1) + v] (n = 0 level). */
static void hermite_R(int L, double alpha, double X, double Y, double Z, double *R) {
    int d = L + 1;
    double *Rn = (double *)calloc((size_t)d * d * d * d, sizeof(double));
#define RN(n, t, u, v) Rn[(((size_t)(n) * d + (t)) * d + (u)) * d + (v)]
    double F[4 * ORC_LMAX + 8];
    orc_boys(L, alpha * (X * X + Y * Y + Z * Z), F);
    double f = 1.0;
    for (int n = 0; n <= L; ++n) { RN(n, 0, 0, 0) = f * F[n]; f *= -2.0 * alpha; }
    for (int s = 1; s <= L; ++s)
        for (int t = 0; t <= s; ++t)
            for (int u = 0; u <= s - t; ++u) {
                int v = s - t - u;
                for (int n = 0; n <= L - s; ++n) {
                    double val;
                    if (t > 0)
                        val = (t > 1 ? (t - 1) * RN(n + 1, t - 2, u, v) : 0.0) + X * RN(n + 1, t - 1, u, v);
                    else if (u > 0)
                        val = (u > 1 ? (u - 1) * RN(n + 1, t, u - 2, v) : 0.0) + Y * RN(n + 1, t, u - 1, v);
                    else
                        val = (v > 1 ? (v - 1) * RN(n + 1, t, u, v - 2) : 0.0) + Z * RN(n + 1, t, u, v - 1);
                    RN(n, t, u, v) = val;
                }
            }
    for (int t = 0; t <= L; ++t)
        for (int u = 0; u <= L; ++u)
            for (int v = 0; v <= L; ++v)
                R[(t * d + u) * d + v] = (t + u + v <= L) ? RN(0, t, u, v) : 0.0;
#undef RN
    free(Rn);
}

/* ---- one-electron integrals ------------------------------------------------ */

/* S, T, V (nbf x nbf, row-major) and the nuclear repulsion energy. */
void orc_one_electron(const orc_basis *b, double *S, double *T, double *V, double *enuc) {
    int n = b->nbf;
    memset(S, 0, sizeof(double) * n * n);
    memset(T, 0, sizeof(double) * n * n);
    memset(V, 0, sizeof(double) * n * n);
    for (int sa = 0; sa < b->nshell; ++sa)
        for (int sb = 0; sb < b->nshell; ++sb) {
            int la = b->l[sa], lb = b->l[sb];
            const double *A = b->cxyz + 3 * sa, *B = b->cxyz + 3 * sb;
            int L = la + lb, d = L + 1;
            double *R = (double *)malloc(sizeof(double) * d * d * d);
            for (int i = 0; i < b->np[sa]; ++i)
                for (int j = 0; j < b->np[sb]; ++j) {
                    double a = b->exps[b->off[sa] + i], bb = b->exps[b->off[sb] + j];
                    double ca = b->coefs[b->off[sa] + i], cb = b->coefs[b->off[sb] + j];
                    double p = a + bb;
                    double P[3];
                    Etab E[3];
                    for (int x = 0; x < 3; ++x) {
                        P[x] = (a * A[x] + bb * B[x]) / p;
                        hermite_E(la, lb + 2, a, bb, A[x] - B[x], E[x]);
                    }
                    double sq = sqrt(M_PI / p);
                    for (int mu = 0; mu < ncart(la); ++mu)
                        for (int nu = 0; nu < ncart(lb); ++nu) {
                            int ia[3] = {0, 0, 0}, ib[3] = {0, 0, 0};
                            cart_comp(la, mu, &ia[0], &ia[1], &ia[2]);
                            cart_comp(lb, nu, &ib[0], &ib[1], &ib[2]);
                            double s1[3], t1[3];
                            for (int x = 0; x < 3; ++x) {
                                int ii = ia[x], jj = ib[x];
                                s1[x] = E[x][ii][jj][0] * sq;
                                double sm2 = jj >= 2 ? E[x][ii][jj - 2][0] * sq : 0.0;
                                double sp2 = E[x][ii][jj + 2][0] * sq;
                                t1[x] = -0.5 * (jj * (jj - 1) * sm2 - 2.0 * bb * (2 * jj + 1) * s1[x] +
                                                4.0 * bb * bb * sp2);
                            }
                            double sv = s1[0] * s1[1] * s1[2];
                            double tv = t1[0] * s1[1] * s1[2] + s1[0] * t1[1] * s1[2] + s1[0] * s1[1] * t1[2];
                            double vv = 0.0;
                            for (int c = 0; c < b->natom; ++c) {
                                const double *C = b->axyz + 3 * c;
                                hermite_R(L, p, P[0] - C[0], P[1] - C[1], P[2] - C[2], R);
                                double acc = 0.0;
                                for (int t = 0; t <= ia[0] + ib[0]; ++t)
                                    for (int u = 0; u <= ia[1] + ib[1]; ++u)
                                        for (int v = 0; v <= ia[2] + ib[2]; ++v)
                                            acc += E[0][ia[0]][ib[0]][t] * E[1][ia[1]][ib[1]][u] *
                                                   E[2][ia[2]][ib[2]][v] * R[(t * d + u) * d + v];
                                vv += -b->Z[c] * 2.0 * M_PI / p * acc;
                            }
                            double sc = ca * cb * comp_scale(la, mu) * comp_scale(lb, nu);
                            int row = b->bf[sa] + mu, col = b->bf[sb] + nu;
                            S[row * n + col] += sc * sv;
                            T[row * n + col] += sc * tv;
                            V[row * n + col] += sc * vv;
                        }
                }
            free(R);
        }
    double e = 0.0;
    for (int A = 0; A < b->natom; ++A)
        for (int B = 0; B < A; ++B) {
            double dx = b->axyz[3 * A] - b->axyz[3 * B], dy = b->axyz[3 * A + 1] - b->axyz[3 * B + 1],
                   dz = b->axyz[3 * A + 2] - b->axyz[3 * B + 2];
            e += b->Z[A] * b->Z[B] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    *enuc = e;
}

/* ---- electron repulsion integrals --------------------------------------------
 * (ab|cd) = 2 pi^{5/2} / (p q sqrt(p+q))
 *           * sum_{tuv} E^{ab}_{tuv} sum_{tau nu phi} (-1)^{tau+nu+phi} E^{cd}_{tau nu phi}
 *             R_{t+tau, u+nu, v+phi}(pq/(p+q), P - Q)
 * out[((mu*nb + nu)*nc + la)*nd + si], contracted and normalised.          */
void orc_eri_shell(const orc_basis *b, int sa, int sb, int sc, int sd, double *out) {
    int la = b->l[sa], lb = b->l[sb], lc = b->l[sc], ld = b->l[sd];
    int na = ncart(la), nb = ncart(lb), nc = ncart(lc), nd = ncart(ld);
    const double *A = b->cxyz + 3 * sa, *B = b->cxyz + 3 * sb, *C = b->cxyz + 3 * sc, *D = b->cxyz + 3 * sd;
    int L = la + lb + lc + ld, d = L + 1;
    int nout = na * nb * nc * nd;
    memset(out, 0, sizeof(double) * nout);
    double *R = (double *)malloc(sizeof(double) * d * d * d);
    int cab[ORC_NCMAX * ORC_NCMAX][6], ccd[ORC_NCMAX * ORC_NCMAX][6];
    for (int mu = 0; mu < na; ++mu)
        for (int nu = 0; nu < nb; ++nu) {
            int *c = cab[mu * nb + nu];
            cart_comp(la, mu, &c[0], &c[1], &c[2]);
            cart_comp(lb, nu, &c[3], &c[4], &c[5]);
        }
    for (int l = 0; l < nc; ++l)
        for (int s = 0; s < nd; ++s) {
            int *c = ccd[l * nd + s];
            cart_comp(lc, l, &c[0], &c[1], &c[2]);
            cart_comp(ld, s, &c[3], &c[4], &c[5]);
        }
    int nh = (la + lb + 1) * (la + lb + 1) * (la + lb + 1);
    double *W = (double *)malloc(sizeof(double) * nh);
    for (int i = 0; i < b->np[sa]; ++i)
        for (int j = 0; j < b->np[sb]; ++j) {
            double a1 = b->exps[b->off[sa] + i], a2 = b->exps[b->off[sb] + j];
            double p = a1 + a2, P[3];
            Etab Eab[3];
            for (int x = 0; x < 3; ++x) {
                P[x] = (a1 * A[x] + a2 * B[x]) / p;
                hermite_E(la, lb, a1, a2, A[x] - B[x], Eab[x]);
            }
            double cij = b->coefs[b->off[sa] + i] * b->coefs[b->off[sb] + j];
            for (int k = 0; k < b->np[sc]; ++k)
                for (int m = 0; m < b->np[sd]; ++m) {
                    double a3 = b->exps[b->off[sc] + k], a4 = b->exps[b->off[sd] + m];
                    double q = a3 + a4, Q[3];
                    Etab Ecd[3];
                    for (int x = 0; x < 3; ++x) {
                        Q[x] = (a3 * C[x] + a4 * D[x]) / q;
                        hermite_E(lc, ld, a3, a4, C[x] - D[x], Ecd[x]);
                    }
                    double alpha = p * q / (p + q);
                    hermite_R(L, alpha, P[0] - Q[0], P[1] - Q[1], P[2] - Q[2], R);
                    double pref = 2.0 * pow(M_PI, 2.5) / (p * q * sqrt(p + q)) * cij *
                                  b->coefs[b->off[sc] + k] * b->coefs[b->off[sd] + m];
                    int hb = la + lb + 1;
                    for (int lsg = 0; lsg < nc * nd; ++lsg) {
                        const int *c2 = ccd[lsg];
                        /* W_{tuv} = sum (-1)^{tau+nu+phi} E^{cd}_{tau nu phi} R_{t+tau,u+nu,v+phi} */
                        for (int t = 0; t < hb; ++t)
                            for (int u = 0; u < hb; ++u)
                                for (int v = 0; v < hb; ++v) {
                                    double w = 0.0;
                                    if (t + u + v <= la + lb)
                                        for (int tt = 0; tt <= c2[0] + c2[3]; ++tt)
                                            for (int uu = 0; uu <= c2[1] + c2[4]; ++uu)
                                                for (int vv = 0; vv <= c2[2] + c2[5]; ++vv) {
                                                    double sg = ((tt + uu + vv) & 1) ? -1.0 : 1.0;
                                                    w += sg * Ecd[0][c2[0]][c2[3]][tt] * Ecd[1][c2[1]][c2[4]][uu] *
                                                         Ecd[2][c2[2]][c2[5]][vv] *
                                                         R[((t + tt) * d + (u + uu)) * d + (v + vv)];
                                                }
                                    W[(t * hb + u) * hb + v] = w;
                                }
                        for (int mn = 0; mn < na * nb; ++mn) {
                            const int *c1 = cab[mn];
                            double acc = 0.0;
                            for (int t = 0; t <= c1[0] + c1[3]; ++t)
                                for (int u = 0; u <= c1[1] + c1[4]; ++u)
                                    for (int v = 0; v <= c1[2] + c1[5]; ++v)
                                        acc += Eab[0][c1[0]][c1[3]][t] * Eab[1][c1[1]][c1[4]][u] *
                                               Eab[2][c1[2]][c1[5]][v] * W[(t * hb + u) * hb + v];
                            out[mn * nc * nd + lsg] += pref * acc;
                        }
                    }
                }
        }
    for (int mu = 0; mu < na; ++mu)
        for (int nu = 0; nu < nb; ++nu)
            for (int l = 0; l < nc; ++l)
                for (int s = 0; s < nd; ++s)
                    out[((mu * nb + nu) * nc + l) * nd + s] *=
                        comp_scale(la, mu) * comp_scale(lb, nu) * comp_scale(lc, l) * comp_scale(ld, s);
    free(W);
    free(R);
}

/* All nbf^4 integrals, out[((m*n + n2)*n + l)*n + s]; tiny systems only. */
void orc_eri_full(const orc_basis *b, double *out) {
    int n = b->nbf;
    double *blk = (double *)malloc(sizeof(double) * ORC_NCMAX * ORC_NCMAX * ORC_NCMAX * ORC_NCMAX);
    for (int a = 0; a < b->nshell; ++a)
        for (int bb = 0; bb < b->nshell; ++bb)
            for (int c = 0; c < b->nshell; ++c)
                for (int d = 0; d < b->nshell; ++d) {
                    orc_eri_shell(b, a, bb, c, d, blk);
                    int na = ncart(b->l[a]), nb = ncart(b->l[bb]), nc = ncart(b->l[c]), nd = ncart(b->l[d]);
                    for (int i = 0; i < na; ++i)
                        for (int j = 0; j < nb; ++j)
                            for (int k = 0; k < nc; ++k)
                                for (int l = 0; l < nd; ++l)
                                    out[(((size_t)(b->bf[a] + i) * n + b->bf[bb] + j) * n + b->bf[c] + k) * n +
                                        b->bf[d] + l] = blk[((i * nb + j) * nc + k) * nd + l];
                }
    free(blk);
}

/* Schwarz bounds Q[a*nshell+b] = sqrt(max_{mu in a, nu in b} (mu nu|mu nu)). */
void orc_schwarz(const orc_basis *b, double *Q) {
    int ns = b->nshell;
#pragma omp parallel
    {
        double *blk = (double *)malloc(sizeof(double) * ORC_NCMAX * ORC_NCMAX * ORC_NCMAX * ORC_NCMAX);
#pragma omp for schedule(dynamic, 1)
        for (int a = 0; a < ns; ++a)
            for (int bb = 0; bb <= a; ++bb) {
                orc_eri_shell(b, a, bb, a, bb, blk);
                int na = ncart(b->l[a]), nb = ncart(b->l[bb]);
                double mx = 0.0;
                for (int i = 0; i < na; ++i)
                    for (int j = 0; j < nb; ++j) {
                        double v = blk[((i * nb + j) * na + i) * nb + j];
                        if (v > mx) mx = v;
                    }
                Q[a * ns + bb] = Q[bb * ns + a] = sqrt(mx);
            }
        free(blk);
    }
}

static int nprim_shell(const orc_basis *b, int s) { return b->np[s]; }

/* ---- J and K ------------------------------------------------------------------ */

/* Brute force: every ordered shell quartet (a b|c d) kept iff Q_ab Q_cd >= tau
 * (tau <= 0 keeps all).  J_{mn} += (mn|ls) D_ls, K_{ml} += (mn|ls) D_ns. */
void orc_jk_brute(const orc_basis *b, const double *D, double tau, const double *Q, double *J, double *K) {
    int n = b->nbf, ns = b->nshell;
    memset(J, 0, sizeof(double) * n * n);
    memset(K, 0, sizeof(double) * n * n);
    double *blk = (double *)malloc(sizeof(double) * ORC_NCMAX * ORC_NCMAX * ORC_NCMAX * ORC_NCMAX);
    for (int a = 0; a < ns; ++a)
        for (int bb = 0; bb < ns; ++bb)
            for (int c = 0; c < ns; ++c)
                for (int d = 0; d < ns; ++d) {
                    if (tau > 0.0 && Q[a * ns + bb] * Q[c * ns + d] < tau) continue;
                    orc_eri_shell(b, a, bb, c, d, blk);
                    int na = ncart(b->l[a]), nb = ncart(b->l[bb]), nc = ncart(b->l[c]), nd = ncart(b->l[d]);
                    for (int i = 0; i < na; ++i)
                        for (int j = 0; j < nb; ++j)
                            for (int k = 0; k < nc; ++k)
                                for (int l = 0; l < nd; ++l) {
                                    double v = blk[((i * nb + j) * nc + k) * nd + l];
                                    int m = b->bf[a] + i, nn = b->bf[bb] + j, la = b->bf[c] + k, s = b->bf[d] + l;
                                    J[m * n + nn] += v * D[la * n + s];
                                    K[m * n + la] += v * D[nn * n + s];
                                }
                }
    free(blk);
}

/* The 8-fold-symmetric loop (section 4.1, algorithm 1's loop nest, eq. 2):
 * unique quartets i >= j, k <= i, l <= (k == i ? j : k), kept iff
 * Q_ij Q_kl >= tau.  With g = s * (ij|kl) and s = (i!=j ? 2:1)(k!=l ? 2:1)
 * ((ij)!=(kl) ? 2:1) the six updates of eq. 2 are accumulated into Jt and Kt,
 * and J = (Jt + Jt^T)/4, K = (Kt + Kt^T)/8.
 * Only bra pairs ij with (ij index % stride) == phase are processed (stride 1
 * = the whole build; larger strides give a bounded sample for timing).
 * stats[0..2] = surviving quartets, integrals, primitive quartets.          */
void orc_jk_8fold(const orc_basis *b, const double *D, double tau, const double *Q, long stride, long phase,
                  double *J, double *K, long long *stats) {
    int n = b->nbf, ns = b->nshell;
    long npair = (long)ns * (ns + 1) / 2;
    long long nq = 0, nint = 0, nprq = 0;
    double *Jt = (double *)calloc((size_t)n * n, sizeof(double));
    double *Kt = (double *)calloc((size_t)n * n, sizeof(double));
#pragma omp parallel reduction(+ : nq, nint, nprq)
    {
        double *Jp = (double *)calloc((size_t)n * n, sizeof(double));
        double *Kp = (double *)calloc((size_t)n * n, sizeof(double));
        double *blk = (double *)malloc(sizeof(double) * ORC_NCMAX * ORC_NCMAX * ORC_NCMAX * ORC_NCMAX);
#pragma omp for schedule(dynamic, 1)
        for (long ij = 0; ij < npair; ++ij) {
            if (stride > 1 && ij % stride != phase) continue;
            int i = (int)((sqrt(8.0 * ij + 1.0) - 1.0) / 2.0);
            while ((long)i * (i + 1) / 2 > ij) --i;
            while ((long)(i + 1) * (i + 2) / 2 <= ij) ++i;
            int j = (int)(ij - (long)i * (i + 1) / 2);
            for (int k = 0; k <= i; ++k) {
                int lmax = (k == i) ? j : k;
                for (int l = 0; l <= lmax; ++l) {
                    if (Q[i * ns + j] * Q[k * ns + l] < tau) continue;
                    orc_eri_shell(b, i, j, k, l, blk);
                    int na = ncart(b->l[i]), nb = ncart(b->l[j]), nc = ncart(b->l[k]), nd = ncart(b->l[l]);
                    double s = (i != j ? 2.0 : 1.0) * (k != l ? 2.0 : 1.0) * ((i != k || j != l) ? 2.0 : 1.0);
                    ++nq;
                    nint += (long long)na * nb * nc * nd;
                    nprq += (long long)nprim_shell(b, i) * nprim_shell(b, j) * nprim_shell(b, k) * nprim_shell(b, l);
                    for (int p = 0; p < na; ++p)
                        for (int q = 0; q < nb; ++q)
                            for (int r = 0; r < nc; ++r)
                                for (int t = 0; t < nd; ++t) {
                                    double g = s * blk[((p * nb + q) * nc + r) * nd + t];
                                    int mu = b->bf[i] + p, nu = b->bf[j] + q, la = b->bf[k] + r, si = b->bf[l] + t;
                                    Jp[mu * n + nu] += g * D[la * n + si];   /* eq. 2a */
                                    Jp[la * n + si] += g * D[mu * n + nu];   /* eq. 2b */
                                    Kp[mu * n + la] += g * D[nu * n + si];   /* eq. 2c */
                                    Kp[nu * n + si] += g * D[mu * n + la];   /* eq. 2d */
                                    Kp[mu * n + si] += g * D[nu * n + la];   /* eq. 2e */
                                    Kp[nu * n + la] += g * D[mu * n + si];   /* eq. 2f */
                                }
                }
            }
        }
#pragma omp critical
        {
            for (long x = 0; x < (long)n * n; ++x) { Jt[x] += Jp[x]; Kt[x] += Kp[x]; }
        }
        free(Jp); free(Kp); free(blk);
    }
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) {
            J[p * n + q] = (Jt[p * n + q] + Jt[q * n + p]) / 4.0;
            K[p * n + q] = (Kt[p * n + q] + Kt[q * n + p]) / 8.0;
        }
    free(Jt); free(Kt);
    if (stats) { stats[0] = nq; stats[1] = nint; stats[2] = nprq; }
}

/* One shell block (a, b) of J and K straight from the definition:
 *   J_{mn} = sum_{c,d} [Q_ab Q_cd >= tau] sum_{ls} (mn|ls) D_ls
 *   K_{mn} = sum_{c,d} [Q_ac Q_bd >= tau] sum_{ls} (ml|ns) D_ls
 * Jb, Kb: na x nb row-major. */
void orc_jk_block(const orc_basis *b, int sa, int sb, const double *D, double tau, const double *Q, double *Jb,
                  double *Kb) {
    int n = b->nbf, ns = b->nshell;
    int na = ncart(b->l[sa]), nb = ncart(b->l[sb]);
    memset(Jb, 0, sizeof(double) * na * nb);
    memset(Kb, 0, sizeof(double) * na * nb);
#pragma omp parallel
    {
        double *blk = (double *)malloc(sizeof(double) * ORC_NCMAX * ORC_NCMAX * ORC_NCMAX * ORC_NCMAX);
        double *jl = (double *)calloc(na * nb, sizeof(double));
        double *kl = (double *)calloc(na * nb, sizeof(double));
#pragma omp for schedule(dynamic, 4)
        for (int c = 0; c < ns; ++c)
            for (int d = 0; d < ns; ++d) {
                int nc = ncart(b->l[c]), nd = ncart(b->l[d]);
                if (Q[sa * ns + sb] * Q[c * ns + d] >= tau) {
                    orc_eri_shell(b, sa, sb, c, d, blk);
                    for (int i = 0; i < na; ++i)
                        for (int j = 0; j < nb; ++j)
                            for (int k = 0; k < nc; ++k)
                                for (int l = 0; l < nd; ++l)
                                    jl[i * nb + j] += blk[((i * nb + j) * nc + k) * nd + l] *
                                                      D[(b->bf[c] + k) * n + b->bf[d] + l];
                }
                if (Q[sa * ns + c] * Q[sb * ns + d] >= tau) {
                    orc_eri_shell(b, sa, c, sb, d, blk);
                    for (int i = 0; i < na; ++i)
                        for (int k = 0; k < nc; ++k)
                            for (int j = 0; j < nb; ++j)
                                for (int l = 0; l < nd; ++l)
                                    kl[i * nb + j] += blk[((i * nc + k) * nb + j) * nd + l] *
                                                      D[(b->bf[c] + k) * n + b->bf[d] + l];
                }
            }
#pragma omp critical
        {
            for (int x = 0; x < na * nb; ++x) { Jb[x] += jl[x]; Kb[x] += kl[x]; }
        }
        free(blk); free(jl); free(kl);
    }
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
