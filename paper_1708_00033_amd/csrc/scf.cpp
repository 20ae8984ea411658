// Closed-shell SCF driver (section 3, eq. 1: F C = eps S C).
//
// Per iteration, on the device: F = H + 2J - K from the direct build, the
// energy E = tr(D (H + F)) + E_nuc, the DIIS error e = X^T (F D S - S D F) X,
// the extrapolated F, F' = X^T F X, its eigensolution (rocSOLVER dsyevd),
// C = X C' and D = C_occ C_occ^T (rocBLAS dgemm).  The host keeps only the
// DIIS matrix B (at most 9 x 9) and solves it.  Converged when
// |E_k - E_{k-1}| < e_tol and rms(D_{k+1} - D_k) < d_rms_tol.
// Guesses: SAD (per element a spherically averaged fractional-occupation
// atomic SCF run by this same driver) or the core Hamiltonian.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <vector>

#include "hfx_ctx.h"

#define HIPCK(call)                                                      \
    do {                                                                 \
        hfx_status _s = hfx_hip_check(c, (call), #call);                 \
        if (_s != HFX_OK) return _s;                                     \
    } while (0)
#define BLASCK(call)                                                                         \
    do {                                                                                     \
        if ((call) != rocblas_status_success) return hfx_fail(c, HFX_ERR_DEVICE, #call);     \
    } while (0)

namespace {

struct DevBuf {
    double* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
    hipError_t alloc(size_t n) { return hipMalloc((void**)&p, (n ? n : 1) * sizeof(double)); }
};

// Symmetric eigenvalues of a small matrix (cyclic Jacobi), for cond(B).
std::vector<double> small_sym_eigs(std::vector<double> A, int m) {
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = i + 1; j < m; ++j) off += A[i * m + j] * A[i * m + j];
        if (off < 1e-300) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = A[p * m + q];
                if (apq == 0.0) continue;
                const double th = (A[q * m + q] - A[p * m + p]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < m; ++k) {
                    const double akp = A[k * m + p], akq = A[k * m + q];
                    A[k * m + p] = cs * akp - sn * akq;
                    A[k * m + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < m; ++k) {
                    const double apk = A[p * m + k], aqk = A[q * m + k];
                    A[p * m + k] = cs * apk - sn * aqk;
                    A[q * m + k] = sn * apk + cs * aqk;
                }
            }
    }
    std::vector<double> w(m);
    for (int i = 0; i < m; ++i) w[i] = A[i * m + i];
    return w;
}

// Gaussian elimination with partial pivoting; false if singular.
bool small_solve(std::vector<double> A, std::vector<double>& b, int m) {
    for (int k = 0; k < m; ++k) {
        int piv = k;
        for (int i = k + 1; i < m; ++i)
            if (std::fabs(A[i * m + k]) > std::fabs(A[piv * m + k])) piv = i;
        if (A[piv * m + k] == 0.0) return false;
        if (piv != k) {
            for (int j = 0; j < m; ++j) std::swap(A[k * m + j], A[piv * m + j]);
            std::swap(b[k], b[piv]);
        }
        for (int i = k + 1; i < m; ++i) {
            const double f = A[i * m + k] / A[k * m + k];
            for (int j = k; j < m; ++j) A[i * m + j] -= f * A[k * m + j];
            b[i] -= f * b[k];
        }
    }
    for (int k = m - 1; k >= 0; --k) {
        double s = b[k];
        for (int j = k + 1; j < m; ++j) s -= A[k * m + j] * b[j];
        b[k] = s / A[k * m + k];
    }
    return true;
}

// Electron pairs npairs spread over orbitals in ascending eps; a degenerate
// set (within window of its lowest member) at the Fermi level shares the rest.
std::vector<double> fractional_occupation(const std::vector<double>& eps, double npairs, double window = 1e-4) {
    const int m = (int)eps.size();
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return eps[a] < eps[b]; });
    std::vector<double> occ(m, 0.0);
    double rem = npairs;
    int i = 0;
    while (rem > 1e-14 && i < m) {
        int j = i;
        while (j + 1 < m && eps[order[j + 1]] - eps[order[i]] < window) ++j;
        const int g = j - i + 1;
        if (rem >= g - 1e-14) {
            for (int k = i; k <= j; ++k) occ[order[k]] = 1.0;
            rem -= g;
        } else {
            for (int k = i; k <= j; ++k) occ[order[k]] = rem / g;
            rem = 0.0;
        }
        i = j + 1;
    }
    return occ;
}

// DIIS Gram matrix B (row-major m x m, oldest vector first) of a ring buffer
// of dmax slots starting at head: make room for a new newest vector, dropping
// the oldest when full.  On return B is m x m with a zero last row and column
// for the new vector, stored in ring slot *slot.
void diis_make_room(std::vector<double>& B, int& m, int& head, int dmax, int* slot) {
    if (m < dmax) {
        *slot = (head + m) % dmax;
        std::vector<double> nb((size_t)(m + 1) * (m + 1), 0.0);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) nb[i * (m + 1) + j] = B[i * m + j];
        B.swap(nb);
        ++m;
    } else {
        *slot = head;
        head = (head + 1) % dmax;
        std::vector<double> nb((size_t)m * m, 0.0);
        for (int i = 1; i < m; ++i)
            for (int j = 1; j < m; ++j) nb[(i - 1) * m + (j - 1)] = B[i * m + j];
        B.swap(nb);
    }
}

double host_sum(const std::vector<double>& v, int n) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += v[i];
    return s;
}

}  // namespace

struct ScfRun {
    int iterations = 0;
    bool converged = false;
    double energy = 0.0;
    int nmo = 0;
    int ndropped = 0;
    double t_fock = 0.0;
};

// Core of the SCF: occ_pairs < 0 means aufbau with nocc doubly occupied
// orbitals, otherwise fractional occupation with occ_pairs electron pairs.
// dD (in/out): device density; on entry the guess unless guess_core.
static hfx_status scf_core(hfx_ctx* c, const hfx_scf_options& o, double occ_pairs, bool guess_core, double* dD,
                           ScfRun& out, std::vector<double>* C_host, std::vector<double>* eps_host) {
    const int n = c->nbf;
    const size_t nn = (size_t)n * n;
    rocblas_handle h = c->blas;
    hipStream_t st = 0;
    BLASCK(rocblas_set_stream(h, st));
    BLASCK(rocblas_set_pointer_mode(h, rocblas_pointer_mode_host));
    const double one = 1.0, zero = 0.0;

    // ---- orthogonaliser ----
    DevBuf U, w, E, X, keepd;
    HIPCK(U.alloc(nn));
    HIPCK(w.alloc(n));
    HIPCK(E.alloc(n));
    rocblas_int* info = nullptr;
    HIPCK(hipMalloc((void**)&info, sizeof(rocblas_int)));
    struct InfoFree { rocblas_int* p; ~InfoFree() { if (p) (void)hipFree(p); } } info_free{info};
    HIPCK(hipMemcpy(U.p, c->d_S, nn * 8, hipMemcpyDeviceToDevice));
    BLASCK(rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, n, U.p, n, w.p, E.p, info));
    std::vector<double> wh(n);
    HIPCK(hipMemcpy(wh.data(), w.p, n * 8, hipMemcpyDeviceToHost));
    std::vector<int> keep;
    for (int i = 0; i < n; ++i)
        if (wh[i] >= o.lindep) keep.push_back(i);
    const int nk = (int)keep.size();
    if (nk < std::max(1, (int)std::ceil(occ_pairs < 0 ? c->nocc : occ_pairs)))
        return hfx_fail(c, HFX_ERR_NUMERICAL, "overlap matrix too singular for the occupied space");
    out.ndropped = n - nk;
    out.nmo = nk;
    HIPCK(X.alloc((size_t)n * nk));
    {
        int* dk = nullptr;
        HIPCK(hipMalloc((void**)&dk, nk * sizeof(int)));
        HIPCK(hipMemcpy(dk, keep.data(), nk * sizeof(int), hipMemcpyHostToDevice));
        DevBuf Us;
        HIPCK(Us.alloc((size_t)n * nk));
        HIPCK(hfx_scale_cols(U.p, w.p, dk, n, nk, Us.p, st));
        (void)hipFree(dk);
        if (nk == n) {   // symmetric S^{-1/2} = (U w^{-1/2}) U^T
            BLASCK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, n, n, n, &one, Us.p, n, U.p, n,
                                 &zero, X.p, n));
        } else {         // canonical
            HIPCK(hipMemcpy(X.p, Us.p, (size_t)n * nk * 8, hipMemcpyDeviceToDevice));
        }
    }
    // ---- work buffers ----
    const int dmax = std::max(0, o.diis_max);
    DevBuf F, Fx, T1, T2, Dn, Fp, Cp, C, eps, Cw, part, Fh, Eh;
    HIPCK(F.alloc(nn));
    HIPCK(Fx.alloc(nn));
    HIPCK(T1.alloc(nn));
    HIPCK(T2.alloc(nn));
    HIPCK(Dn.alloc(nn));
    HIPCK(Fp.alloc((size_t)nk * nk));
    HIPCK(Cp.alloc((size_t)nk * nk));
    HIPCK(C.alloc((size_t)n * nk));
    HIPCK(Cw.alloc((size_t)n * nk));
    HIPCK(eps.alloc(nk));
    HIPCK(part.alloc(4096));
    HIPCK(Fh.alloc(nn * std::max(1, dmax)));
    HIPCK(Eh.alloc((size_t)nk * nk * std::max(1, dmax)));
    std::vector<double> parth(4096);
    std::vector<double> epsh(nk);
    // eigenvectors of X^T M X -> C, new density into dst
    auto diag_density = [&](const double* M, double* dst) -> hfx_status {
        BLASCK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, nk, n, &one, M, n, X.p, n, &zero,
                             T1.p, n));
        BLASCK(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, nk, nk, n, &one, X.p, n, T1.p, n,
                             &zero, Cp.p, nk));
        BLASCK(rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, nk, Cp.p, nk, eps.p, E.p, info));
        rocblas_int ih = 0;
        HIPCK(hipMemcpy(&ih, info, sizeof(ih), hipMemcpyDeviceToHost));
        if (ih != 0) return hfx_fail(c, HFX_ERR_NUMERICAL, "eigensolver did not converge");
        BLASCK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, nk, nk, &one, X.p, n, Cp.p, nk,
                             &zero, C.p, n));
        HIPCK(hipMemcpy(epsh.data(), eps.p, nk * 8, hipMemcpyDeviceToHost));
        for (double e : epsh)
            if (!std::isfinite(e)) return hfx_fail(c, HFX_ERR_NUMERICAL, "non-finite orbital energy");
        if (occ_pairs < 0) {
            BLASCK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, n, n, c->nocc, &one, C.p, n,
                                 C.p, n, &zero, dst, n));
        } else {
            std::vector<double> occ = fractional_occupation(epsh, occ_pairs);
            DevBuf docc;
            HIPCK(docc.alloc(nk));
            HIPCK(hipMemcpy(docc.p, occ.data(), nk * 8, hipMemcpyHostToDevice));
            HIPCK(hfx_weight_cols(C.p, docc.p, n, nk, Cw.p, st));
            BLASCK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, n, n, nk, &one, Cw.p, n, C.p,
                                 n, &zero, dst, n));
        }
        return HFX_OK;
    };
    if (guess_core) {
        hfx_status s = diag_density(c->d_H, dD);
        if (s != HFX_OK) return s;
    }
    // ---- iterations ----
    std::vector<double> B;   // DIIS Gram matrix, row-major m x m
    int m = 0, head = 0;     // ring buffer of m vectors starting at slot head
    std::vector<int> slot_of;   // age order -> slot
    double e_old = 0.0;
    bool have_old = false;
    out.converged = false;
    for (int it = 1; it <= o.max_iter; ++it) {
        auto tf = std::chrono::steady_clock::now();
        hfx_status s = hfx_build_internal(c, dD, 2.0, 1.0, c->d_H, F.p, st, nullptr, 0, 1);
        if (s != HFX_OK) return s;
        HIPCK(hipStreamSynchronize(st));
        out.t_fock += std::chrono::duration<double>(std::chrono::steady_clock::now() - tf).count();
        int np = hfx_energy_partial(dD, c->d_H, F.p, nn, part.p, st);
        HIPCK(hipMemcpy(parth.data(), part.p, np * 8, hipMemcpyDeviceToHost));
        const double Ek = host_sum(parth, np) + c->enuc;
        if (!std::isfinite(Ek)) return hfx_fail(c, HFX_ERR_NUMERICAL, "non-finite energy");
        out.energy = Ek;
        out.iterations = it;
        const double* Fuse = F.p;
        if (dmax > 0) {
            // error X^T (F D S - S D F) X
            BLASCK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, n, n, &one, F.p, n, dD, n, &zero,
                                 T1.p, n));
            BLASCK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, n, n, &one, T1.p, n, c->d_S, n,
                                 &zero, T2.p, n));
            HIPCK(hfx_antisym(T2.p, n, T1.p, st));
            BLASCK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, nk, n, &one, T1.p, n, X.p, n,
                                 &zero, T2.p, n));
            int slot;
            diis_make_room(B, m, head, dmax, &slot);
            double* eslot = Eh.p + (size_t)slot * nk * nk;
            BLASCK(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, nk, nk, n, &one, X.p, n, T2.p,
                                 n, &zero, eslot, nk));
            HIPCK(hipMemcpy(Fh.p + (size_t)slot * nn, F.p, nn * 8, hipMemcpyDeviceToDevice));
            for (int i = 0; i < m; ++i) {   // the new last row and column of B
                const int si = (head + i) % dmax;
                int np2 = hfx_dot_partial(Eh.p + (size_t)si * nk * nk, eslot, (size_t)nk * nk, 0, part.p, st);
                HIPCK(hipMemcpy(parth.data(), part.p, np2 * 8, hipMemcpyDeviceToHost));
                const double v = host_sum(parth, np2);
                B[i * m + (m - 1)] = v;
                B[(m - 1) * m + i] = v;
            }
            // extrapolate with the newest m' <= m vectors; drop the oldest while ill-conditioned
            int use = m;
            std::vector<double> coef;
            while (use >= 2) {
                const int off = m - use;
                const int q = use + 1;
                std::vector<double> A((size_t)q * q, 0.0);
                for (int i = 0; i < use; ++i)
                    for (int j = 0; j < use; ++j) A[i * q + j] = B[(off + i) * m + (off + j)];
                for (int i = 0; i < use; ++i) A[i * q + use] = A[use * q + i] = -1.0;
                std::vector<double> ev = small_sym_eigs(A, q);
                double amax = 0.0, amin = 1e300;
                for (double e : ev) {
                    amax = std::max(amax, std::fabs(e));
                    amin = std::min(amin, std::fabs(e));
                }
                std::vector<double> rhs(q, 0.0);
                rhs[use] = -1.0;
                if (amin > 0.0 && amax / amin <= 1e14 && small_solve(A, rhs, q)) {
                    coef.assign(rhs.begin(), rhs.begin() + use);
                    break;
                }
                // permanently drop the oldest vector
                head = (head + 1) % dmax;
                std::vector<double> nb((size_t)(m - 1) * (m - 1));
                for (int i = 1; i < m; ++i)
                    for (int j = 1; j < m; ++j) nb[(i - 1) * (m - 1) + (j - 1)] = B[i * m + j];
                B.swap(nb);
                --m;
                use = m;
            }
            if (!coef.empty()) {
                std::vector<const double*> ptrs(m);
                for (int i = 0; i < m; ++i) ptrs[i] = Fh.p + (size_t)((head + i) % dmax) * nn;
                const double** dptrs = nullptr;
                double* dcoef = nullptr;
                HIPCK(hipMalloc((void**)&dptrs, m * sizeof(double*)));
                HIPCK(hipMalloc((void**)&dcoef, m * sizeof(double)));
                HIPCK(hipMemcpy(dptrs, ptrs.data(), m * sizeof(double*), hipMemcpyHostToDevice));
                HIPCK(hipMemcpy(dcoef, coef.data(), m * sizeof(double), hipMemcpyHostToDevice));
                HIPCK(hfx_lincomb(dptrs, dcoef, m, nn, Fx.p, st));
                HIPCK(hipStreamSynchronize(st));
                (void)hipFree(dptrs);
                (void)hipFree(dcoef);
                Fuse = Fx.p;
            }
        }
        s = diag_density(Fuse, Dn.p);
        if (s != HFX_OK) return s;
        np = hfx_dot_partial(Dn.p, dD, nn, 1, part.p, st);
        HIPCK(hipMemcpy(parth.data(), part.p, np * 8, hipMemcpyDeviceToHost));
        const double drms = std::sqrt(host_sum(parth, np) / (double)nn);
        HIPCK(hipMemcpy(dD, Dn.p, nn * 8, hipMemcpyDeviceToDevice));
        if (c->opt.log_level > 0)
            std::fprintf(stderr, "[hfx scf] it %3d  E = %.12f  dE = %.3e  rmsD = %.3e  diis %d\n", it, Ek,
                         have_old ? Ek - e_old : 0.0, drms, m);
        if (have_old && std::fabs(Ek - e_old) < o.e_tol && drms < o.d_rms_tol) {
            out.converged = true;
            break;
        }
        e_old = Ek;
        have_old = true;
    }
    if (C_host) {
        C_host->resize((size_t)n * nk);
        HIPCK(hipMemcpy(C_host->data(), C.p, (size_t)n * nk * 8, hipMemcpyDeviceToHost));
    }
    if (eps_host) *eps_host = epsh;
    return HFX_OK;
}

// SAD: block-diagonal superposition of per-element atomic densities, in the
// ragged per-molecule layout (a single molecule: one nbf x nbf block).
static hfx_status sad_guess(hfx_ctx* c, std::vector<double>& Dsad) {
    Dsad.assign(c->nelem, 0.0);
    std::vector<std::vector<int>> atom_shells(c->natom);
    for (int s = 0; s < c->nshell; ++s) atom_shells[c->shell_atom[s]].push_back(s);
    std::vector<int> atom_mol(c->natom, 0);
    for (int m = 0; m < c->nmol; ++m)
        for (int a = 0; a < c->mol[m].natom; ++a) atom_mol[c->mol[m].aoff + a] = m;
    for (int a = 0; a < c->natom; ++a) {
        const int z = c->Z[a];
        const std::vector<int>& sh = atom_shells[a];
        const MolInfo& M = c->mol[atom_mol[a]];
        const int n = M.nbf;
        double* Dm = Dsad.data() + M.moff;
        if (sh.empty()) continue;
        // key: element and the raw shells (l, exponents, coefficients)
        std::string key(reinterpret_cast<const char*>(&z), sizeof(int));
        for (int s : sh) {
            key.append(reinterpret_cast<const char*>(&c->shell_exps_l[s]), sizeof(int));
            key.append(reinterpret_cast<const char*>(c->raw_exps[s].data()), c->raw_exps[s].size() * sizeof(double));
            key.append(reinterpret_cast<const char*>(c->raw_coefs[s].data()),
                       c->raw_coefs[s].size() * sizeof(double));
            key.push_back('|');
        }
        if (!c->sad_cache.count(key)) {
            hfx_options ao = c->opt;
            ao.precision = HFX_PREC_FP64;
            ao.log_level = 0;
            ao.task_quartets = 256;
            ao.schwarz_tau = 0.0;
            hfx_ctx* sub = nullptr;
            if (hfx_create(&ao, &sub) != HFX_OK) return hfx_fail(c, HFX_ERR_DEVICE, "SAD: context creation failed");
            std::vector<hfx_shell> shells;
            for (int s : sh) {
                hfx_shell x;
                x.atom = 0;
                x.l = c->shell_exps_l[s];
                x.nprim = (int)c->raw_exps[s].size();
                x.exps = c->raw_exps[s].data();
                x.coefs = c->raw_coefs[s].data();
                x.coefs_p = nullptr;
                shells.push_back(x);
            }
            const double origin[3] = {0.0, 0.0, 0.0};
            // the atom's own charge: Z electrons even or odd; fractional pairs Z/2
            int zz = z;
            hfx_status s = hfx_load(sub, 1, &zz, origin, (int)shells.size(), shells.data(), z % 2);
            if (s != HFX_OK) {
                std::string m = hfx_last_error(sub);
                hfx_destroy(sub);
                return hfx_fail(c, s, "SAD: atomic load failed: " + m);
            }
            const int na = sub->nbf;
            double* dDa = nullptr;
            if (hipMalloc((void**)&dDa, (size_t)na * na * 8) != hipSuccess) {
                hfx_destroy(sub);
                return hfx_fail(c, HFX_ERR_OOM, "SAD: allocation failed");
            }
            hfx_scf_options so;
            hfx_default_scf_options(&so);
            so.max_iter = 200;
            so.e_tol = 1e-11;
            so.d_rms_tol = 1e-9;
            ScfRun run;
            s = scf_core(sub, so, z / 2.0, true, dDa, run, nullptr, nullptr);
            std::vector<double> Da((size_t)na * na);
            if (s == HFX_OK && hipMemcpy(Da.data(), dDa, Da.size() * 8, hipMemcpyDeviceToHost) != hipSuccess)
                s = HFX_ERR_DEVICE;
            std::string m = hfx_last_error(sub);
            (void)hipFree(dDa);
            hfx_destroy(sub);
            if (s != HFX_OK) return hfx_fail(c, s, "SAD: atomic SCF failed: " + m);
            c->sad_cache[key] = Da;
        }
        const auto& Da = c->sad_cache[key];
        const int na = (int)std::lround(std::sqrt((double)Da.size()));
        const int o0 = c->shells[sh.front()].bf;
        int nloc = 0;
        for (int s : sh) nloc += (c->shells[s].l + 1) * (c->shells[s].l + 2) / 2;
        if (nloc != na) return hfx_fail(c, HFX_ERR_INVALID_ARG, "SAD: atoms of one element must share a basis");
        for (int i = 0; i < na; ++i)
            for (int j = 0; j < na; ++j) Dm[(size_t)(o0 + i) * n + o0 + j] = Da[(size_t)i * na + j];
    }
    return HFX_OK;
}

extern "C" hfx_status hfx_sad_density(hfx_ctx* c, double* D_out) {
    if (!c || !D_out) return c ? hfx_fail(c, HFX_ERR_INVALID_ARG, "null pointer") : HFX_ERR_INVALID_ARG;
    if (!c->loaded) return hfx_fail(c, HFX_ERR_STATE, "hfx_sad_density: nothing loaded");
    if (c->nmol != 1) return hfx_fail(c, HFX_ERR_STATE, "hfx_sad_density: single molecules only");
    HIPCK(hipSetDevice(c->opt.device));
    std::vector<double> Ds;
    hfx_status s = sad_guess(c, Ds);
    if (s != HFX_OK) return s;
    std::memcpy(D_out, Ds.data(), Ds.size() * sizeof(double));
    return HFX_OK;
}

extern "C" hfx_status hfx_scf(hfx_ctx* c, const hfx_scf_options* opt, hfx_scf_result* res, double* D_out,
                              double* C_out, double* eps_out) {
    if (!c || !res) return c ? hfx_fail(c, HFX_ERR_INVALID_ARG, "null pointer") : HFX_ERR_INVALID_ARG;
    if (!c->loaded) return hfx_fail(c, HFX_ERR_STATE, "hfx_scf: nothing loaded");
    if (c->nmol != 1) return hfx_fail(c, HFX_ERR_STATE, "hfx_scf: use hfx_batch_scf for a batch");
    hfx_scf_options o;
    if (opt) o = *opt; else hfx_default_scf_options(&o);
    if (o.max_iter < 1 || o.diis_max < 0 || o.diis_max > 32 || !(o.e_tol > 0) || !(o.d_rms_tol > 0) ||
        !(o.lindep > 0))
        return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_scf: invalid options");
    HIPCK(hipSetDevice(c->opt.device));
    auto t0 = std::chrono::steady_clock::now();
    const int n = c->nbf;
    const size_t nn = (size_t)n * n;
    DevBuf D;
    HIPCK(D.alloc(nn));
    int guess_used = o.guess;
    bool core = false;
    if (o.D0) {
        for (size_t i = 0; i < nn; ++i)
            if (!std::isfinite(o.D0[i])) return hfx_fail(c, HFX_ERR_NUMERICAL, "hfx_scf: non-finite D0");
        HIPCK(hipMemcpy(D.p, o.D0, nn * 8, hipMemcpyHostToDevice));
        guess_used = -1;
    } else if (o.guess == HFX_GUESS_CORE) {
        core = true;
    } else if (o.guess == HFX_GUESS_SAD || o.guess == HFX_GUESS_LEARNED) {
        if (o.guess == HFX_GUESS_LEARNED && !o.model)
            return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_scf: learned guess without a model");
        std::vector<double> Ds;
        hfx_status s = sad_guess(c, Ds);
        if (s != HFX_OK) return s;
        HIPCK(hipMemcpy(D.p, Ds.data(), nn * 8, hipMemcpyHostToDevice));
        if (o.guess == HFX_GUESS_LEARNED) {
            int used = 0;
            s = hfx_guess_apply(c, o.model, D.p, nullptr, &used);
            if (s != HFX_OK) return s;
            if (!used) guess_used = HFX_GUESS_SAD;   // prediction rejected: SAD fallback
        }
    } else {
        return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_scf: unknown guess");
    }
    ScfRun run;
    std::vector<double> Ch, epsh;
    hfx_status s = scf_core(c, o, -1.0, core, D.p, run, C_out ? &Ch : nullptr, &epsh);
    if (s != HFX_OK) return s;
    res->energy = run.energy;
    res->e_nuc = c->enuc;
    res->iterations = run.iterations;
    res->converged = run.converged ? 1 : 0;
    res->guess_used = guess_used;
    res->ndropped = run.ndropped;
    res->t_fock_s = run.t_fock;
    res->graph_segments = 0;
    res->t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (D_out) HIPCK(hipMemcpy(D_out, D.p, nn * 8, hipMemcpyDeviceToHost));
    if (C_out) {   // column-major n x nmo -> row-major
        const int nmo = run.nmo;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < nmo; ++j) C_out[(size_t)i * nmo + j] = Ch[(size_t)j * n + i];
    }
    if (eps_out) std::memcpy(eps_out, epsh.data(), epsh.size() * sizeof(double));
    return run.converged ? HFX_OK : hfx_fail(c, HFX_ERR_NOT_CONVERGED, "hfx_scf: not converged within max_iter");
}

// ---- batched SCF ------------------------------------------------------------------------
// Every molecule of a batch iterates in lockstep: one batched Fock build for
// all of them per iteration, then per molecule the energy, Pulay DIIS and
// X^T F X (the steps of the single-molecule driver above), and one batched
// eigensolve for all molecules: each X^T F X sits in the top-left corner of
// an NP x NP slot padded with a large diagonal, so its eigenpairs come first
// and the padding's (unit vectors) after them.
namespace {

constexpr double kPadDiag = 1.0e6;   // far above any orbital energy or overlap eigenvalue (hartree)

struct MolScf {
    int n = 0, nk = 0, nocc = 0;
    long long moff = 0;
    double enuc = 0.0;
    DevBuf X, T1, T2, Dn, Fx, C, Fh, Eh;
    std::vector<double> B;   // DIIS Gram matrix of the m stored vectors (oldest first)
    int m = 0, head = 0;
    double energy = 0.0, e_old = 0.0;
    bool have_old = false, converged = false;
    int iterations = 0, ndropped = 0;
};

double dev_sum(hfx_ctx* c, int np, DevBuf& part, std::vector<double>& parth, bool& ok) {
    ok = hipMemcpy(parth.data(), part.p, np * 8, hipMemcpyDeviceToHost) == hipSuccess;
    (void)c;
    return host_sum(parth, np);
}

}  // namespace

// ---- batched SCF with captured iterations ---------------------------------------
// The same steps as the eager batched driver below, on padded NP x NP slots
// (batch_scf.hip) so that each step is one launch for all molecules, and the
// device work of an iteration replayed from HIP graphs: (a) Fock build,
// energies, DIIS error X^T (F D S - S D F) X, ring store and Gram row;
// (b) extrapolation and projection X^T F X; (c) orbitals C = X C', aufbau
// density, rms change.  Between them: the batched eigensolve and the small
// DIIS solve on the host (one copy of the energies and Gram rows per
// iteration).  Iteration 1 runs eagerly (library workspaces, kernel
// attributes), then each segment is captured once; a segment whose capture
// fails runs eagerly from then on.
extern "C" {
hipError_t hfx_bscf_pack(const double* rag, const long long* moff, const int* dim, int nmol, int NP, double* pad,
                         hipStream_t st);
hipError_t hfx_bscf_energy(const double* D, const double* H, const double* F, const long long* moff, const int* dim,
                           int nmol, double* E, hipStream_t st);
hipError_t hfx_bscf_antisym(const double* A, int nmol, int NP, double* out, hipStream_t st);
hipError_t hfx_bscf_ring_store(const double* src, int nmol, int NP, const int* slot, int dmax, double* ring,
                               hipStream_t st);
hipError_t hfx_bscf_ring_dots(const double* e, const double* ring, int nmol, int NP, int dmax, double* dots,
                              hipStream_t st);
hipError_t hfx_bscf_ring_lincomb(const double* ring, const double* coef, int nmol, int NP, int dmax, double* out,
                                 hipStream_t st);
hipError_t hfx_bscf_occ_cols(const double* C, const int* nocc, int nmol, int NP, double* out, hipStream_t st);
hipError_t hfx_bscf_dsq(const double* Dn, const double* D, const int* dim, int nmol, int NP, double* sq,
                        hipStream_t st);
hipError_t hfx_bscf_take_density(const double* Dn, const int* active, const long long* moff, const int* dim, int nmol,
                                 int NP, double* Dpad, double* rag, hipStream_t st);
}

namespace {

struct GraphSeg {
    hipGraphExec_t exec = nullptr;
    bool eager = false;   // capture failed once: run eagerly
    ~GraphSeg() {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
};

struct StreamGuard {
    hipStream_t s = nullptr;
    ~StreamGuard() {
        if (s) (void)hipStreamDestroy(s);
    }
};

}  // namespace

static hfx_status batch_scf_graph(hfx_ctx* c, const hfx_scf_options& o, hfx_scf_result* res, double* D_out,
                                  int* segments_captured) {
    auto t0 = std::chrono::steady_clock::now();
    const int nmol = c->nmol;
    const size_t ne = c->nelem;
    const int NP = std::max(1, c->max_ld);
    const size_t slot = (size_t)NP * NP, all = slot * nmol;
    const int dmax = std::max(0, o.diis_max), dring = std::max(1, dmax);
    rocblas_handle h = c->blas;
    StreamGuard sg;
    HIPCK(hipStreamCreateWithFlags(&sg.s, hipStreamNonBlocking));
    hipStream_t st = sg.s;
    BLASCK(rocblas_set_stream(h, st));
    BLASCK(rocblas_set_pointer_mode(h, rocblas_pointer_mode_host));
    const double one = 1.0, zero = 0.0;
    const bool timing = c->timing;
    c->timing = false;   // no events inside captured work
    struct TimingRestore {
        hfx_ctx* c;
        bool t;
        ~TimingRestore() {
            c->timing = t;
            rocblas_set_stream(c->blas, 0);
        }
    } timing_restore{c, timing};

    // ---- guess (ragged) ----
    DevBuf D, F;
    HIPCK(D.alloc(ne));
    HIPCK(F.alloc(ne));
    bool core = false;
    int guess_used = o.guess;
    if (o.D0) {
        for (size_t i = 0; i < ne; ++i)
            if (!std::isfinite(o.D0[i])) return hfx_fail(c, HFX_ERR_NUMERICAL, "hfx_batch_scf: non-finite D0");
        HIPCK(hipMemcpy(D.p, o.D0, ne * 8, hipMemcpyHostToDevice));
        guess_used = -1;
    } else if (o.guess == HFX_GUESS_CORE) {
        core = true;
    } else if (o.guess == HFX_GUESS_SAD) {
        std::vector<double> Ds;
        hfx_status s = sad_guess(c, Ds);
        if (s != HFX_OK) return s;
        HIPCK(hipMemcpy(D.p, Ds.data(), ne * 8, hipMemcpyHostToDevice));
    } else {
        return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_batch_scf: unknown guess");
    }

    // ---- padded slots ----
    DevBuf Sp, Xp, Dp, Fp, T1, T2, Ep, Fx, P, C, Cw, Dn, Wv, Ew, ringF, ringE;
    for (DevBuf* b : {&Sp, &Xp, &Dp, &Fp, &T1, &T2, &Ep, &Fx, &P, &C, &Cw, &Dn}) HIPCK(b->alloc(all));
    HIPCK(Wv.alloc((size_t)NP * nmol));
    HIPCK(Ew.alloc((size_t)NP * nmol));
    HIPCK(ringF.alloc(all * dring));
    HIPCK(ringE.alloc(all * dring));
    HIPCK(hipMemsetAsync(ringF.p, 0, all * dring * 8, st));   // eager set-up, never captured
    HIPCK(hipMemsetAsync(ringE.p, 0, all * dring * 8, st));
    DevBuf dE, dots, coef, dsq;
    HIPCK(dE.alloc(nmol));
    HIPCK(dots.alloc((size_t)nmol * dring));
    HIPCK(coef.alloc((size_t)nmol * dring));
    HIPCK(dsq.alloc(nmol));
    int *d_slot = nullptr, *d_active = nullptr, *d_nk = nullptr, *d_nocc = nullptr;
    rocblas_int* info = nullptr;
    HIPCK(hipMalloc((void**)&d_slot, nmol * sizeof(int)));
    HIPCK(hipMalloc((void**)&d_active, nmol * sizeof(int)));
    HIPCK(hipMalloc((void**)&d_nk, nmol * sizeof(int)));
    HIPCK(hipMalloc((void**)&d_nocc, nmol * sizeof(int)));
    HIPCK(hipMalloc((void**)&info, nmol * sizeof(rocblas_int)));
    struct IntBufs {
        void* p[5];
        ~IntBufs() {
            for (void* q : p)
                if (q) (void)hipFree(q);
        }
    } int_bufs{{d_slot, d_active, d_nk, d_nocc, info}};

    // ---- orthogonalisers: one batched eigensolve of the padded S blocks ----
    HIPCK(hfx_pad_blocks(c->d_S, c->d_moff, c->d_mdim, nmol, NP, kPadDiag, P.p, st));
    BLASCK(rocsolver_dsyevd_strided_batched(h, rocblas_evect_original, rocblas_fill_upper, NP, P.p, NP,
                                            (rocblas_stride)slot, Wv.p, NP, Ew.p, NP, info, nmol));
    std::vector<double> wh((size_t)NP * nmol);
    std::vector<rocblas_int> infoh(nmol);
    HIPCK(hipMemcpyAsync(wh.data(), Wv.p, wh.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCK(hipMemcpyAsync(infoh.data(), info, nmol * sizeof(rocblas_int), hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    for (int m = 0; m < nmol; ++m)
        if (infoh[m] != 0) return hfx_fail(c, HFX_ERR_NUMERICAL, "hfx_batch_scf: overlap eigensolve failed");
    HIPCK(hipMemsetAsync(Xp.p, 0, all * 8, st));
    std::vector<int> nk(nmol), nocc(nmol), ndrop(nmol);
    for (int m = 0; m < nmol; ++m) {
        const int n = c->mol[m].nbf;
        std::vector<int> keep;
        for (int i = 0; i < n; ++i)
            if (wh[(size_t)m * NP + i] >= o.lindep) keep.push_back(i);
        nk[m] = (int)keep.size();
        nocc[m] = c->mol[m].nocc;
        ndrop[m] = n - nk[m];
        if (nk[m] < std::max(1, nocc[m]))
            return hfx_fail(c, HFX_ERR_NUMERICAL, "hfx_batch_scf: overlap matrix too singular for the occupied space");
        DevBuf U, Us, X;
        HIPCK(U.alloc((size_t)n * n));
        HIPCK(Us.alloc((size_t)n * nk[m]));
        HIPCK(X.alloc((size_t)n * nk[m]));
        HIPCK(hipMemcpy2DAsync(U.p, (size_t)n * 8, P.p + (size_t)m * slot, (size_t)NP * 8, (size_t)n * 8, n,
                               hipMemcpyDeviceToDevice, st));
        int* dk = nullptr;
        HIPCK(hipMalloc((void**)&dk, nk[m] * sizeof(int)));
        HIPCK(hipMemcpyAsync(dk, keep.data(), nk[m] * sizeof(int), hipMemcpyHostToDevice, st));
        hipError_t e = hfx_scale_cols(U.p, Wv.p + (size_t)m * NP, dk, n, nk[m], Us.p, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        (void)hipFree(dk);
        HIPCK(e);
        if (nk[m] == n)
            BLASCK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, n, n, n, &one, Us.p, n, U.p, n,
                                 &zero, X.p, n));
        else
            HIPCK(hipMemcpyAsync(X.p, Us.p, (size_t)n * nk[m] * 8, hipMemcpyDeviceToDevice, st));
        HIPCK(hipMemcpy2DAsync(Xp.p + (size_t)m * slot, (size_t)NP * 8, X.p, (size_t)n * 8, (size_t)n * 8, nk[m],
                               hipMemcpyDeviceToDevice, st));
        HIPCK(hipStreamSynchronize(st));
    }
    HIPCK(hipMemcpyAsync(d_nk, nk.data(), nmol * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(d_nocc, nocc.data(), nmol * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCK(hfx_bscf_pack(c->d_S, c->d_moff, c->d_mdim, nmol, NP, Sp.p, st));

    auto gemm = [&](rocblas_operation ta, rocblas_operation tb, const double* A, const double* B, double* Cm) {
        return rocblas_dgemm_strided_batched(h, ta, tb, NP, NP, NP, &one, A, NP, (rocblas_stride)slot, B, NP,
                                             (rocblas_stride)slot, &zero, Cm, NP, (rocblas_stride)slot, nmol);
    };
    const rocblas_operation N_ = rocblas_operation_none, T_ = rocblas_operation_transpose;
#define SEGCK(call)                                                                    \
    do {                                                                               \
        hipError_t _e = (call);                                                        \
        if (_e != hipSuccess) return hfx_hip_check(c, _e, #call);                      \
    } while (0)
#define SEGBLAS(call)                                                                  \
    do {                                                                               \
        if ((call) != rocblas_status_success) return hfx_fail(c, HFX_ERR_DEVICE, #call); \
    } while (0)
    // (a) build, energies, DIIS error, ring store, Gram row
    auto seg_a = [&]() -> hfx_status {
        hfx_status s = hfx_build_internal(c, D.p, 2.0, 1.0, c->d_H, F.p, st, nullptr, 0, 1);
        if (s != HFX_OK) return s;
        SEGCK(hfx_bscf_energy(D.p, c->d_H, F.p, c->d_moff, c->d_mdim, nmol, dE.p, st));
        SEGCK(hfx_bscf_pack(F.p, c->d_moff, c->d_mdim, nmol, NP, Fp.p, st));
        SEGBLAS(gemm(N_, N_, Fp.p, Dp.p, T1.p));   // F D
        SEGBLAS(gemm(N_, N_, T1.p, Sp.p, T2.p));   // F D S
        SEGCK(hfx_bscf_antisym(T2.p, nmol, NP, T1.p, st));   // F D S - S D F
        SEGBLAS(gemm(N_, N_, T1.p, Xp.p, T2.p));
        SEGBLAS(gemm(T_, N_, Xp.p, T2.p, Ep.p));   // X^T (F D S - S D F) X
        SEGCK(hfx_bscf_ring_store(Ep.p, nmol, NP, d_slot, dring, ringE.p, st));
        SEGCK(hfx_bscf_ring_store(Fp.p, nmol, NP, d_slot, dring, ringF.p, st));
        SEGCK(hfx_bscf_ring_dots(Ep.p, ringE.p, nmol, NP, dring, dots.p, st));
        return HFX_OK;
    };
    // (b) extrapolated F, projection, padding of the eigenproblem
    auto seg_b = [&]() -> hfx_status {
        SEGCK(hfx_bscf_ring_lincomb(ringF.p, coef.p, nmol, NP, dring, Fx.p, st));
        SEGBLAS(gemm(N_, N_, Fx.p, Xp.p, T1.p));
        SEGBLAS(gemm(T_, N_, Xp.p, T1.p, P.p));   // X^T F X
        SEGCK(hfx_pad_rest(d_nk, nmol, NP, kPadDiag, P.p, st));
        return HFX_OK;
    };
    // (c) orbitals, aufbau density, rms change, new density of the active molecules
    auto seg_c = [&]() -> hfx_status {
        SEGBLAS(gemm(N_, N_, Xp.p, P.p, C.p));   // C = X C'
        SEGCK(hfx_bscf_occ_cols(C.p, d_nocc, nmol, NP, Cw.p, st));
        SEGBLAS(gemm(N_, T_, Cw.p, C.p, Dn.p));   // C_occ C_occ^T
        SEGCK(hfx_bscf_dsq(Dn.p, Dp.p, c->d_mdim, nmol, NP, dsq.p, st));
        SEGCK(hfx_bscf_take_density(Dn.p, d_active, c->d_moff, c->d_mdim, nmol, NP, Dp.p, D.p, st));
        return HFX_OK;
    };
#undef SEGCK
#undef SEGBLAS
    auto eig = [&]() -> hfx_status {
        BLASCK(rocsolver_dsyevd_strided_batched(h, rocblas_evect_original, rocblas_fill_upper, NP, P.p, NP,
                                                (rocblas_stride)slot, Wv.p, NP, Ew.p, NP, info, nmol));
        return HFX_OK;
    };
    GraphSeg ga, gb, gc;
    int captured = 0;
    auto run = [&](GraphSeg& g, const std::function<hfx_status()>& seq, bool may_capture) -> hfx_status {
        if (g.exec) {
            HIPCK(hipGraphLaunch(g.exec, st));
            return HFX_OK;
        }
        if (!may_capture || g.eager) return seq();
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            g.eager = true;
            return seq();
        }
        hfx_status s = seq();
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(st, &graph);
        if (s == HFX_OK && e == hipSuccess && graph && hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) == hipSuccess) {
            (void)hipGraphDestroy(graph);
            ++captured;
            HIPCK(hipGraphLaunch(g.exec, st));
            return HFX_OK;
        }
        if (graph) (void)hipGraphDestroy(graph);
        g.exec = nullptr;
        g.eager = true;   // the captured work did not run: run it now
        (void)hipGetLastError();
        return seq();
    };

    // ---- host DIIS state per molecule (the eager driver's rules) ----
    struct Mol {
        std::vector<double> B;
        int m = 0, head = 0, iterations = 0;
        double energy = 0.0, e_old = 0.0;
        bool have_old = false, converged = false;
    };
    std::vector<Mol> mols(nmol);
    std::vector<int> slot_h(nmol, 0), active(nmol, 1);
    std::vector<double> Eh(nmol), dotsh((size_t)nmol * dring), coefh((size_t)nmol * dring), sqh(nmol);
    HIPCK(hipMemcpyAsync(d_active, active.data(), nmol * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCK(hipMemsetAsync(Dp.p, 0, all * 8, st));
    if (core) {   // diagonalise H: H stored in every molecule's ring slot 0, segments (b), (c) eagerly
        std::vector<int> s0(nmol, 0);
        HIPCK(hipMemcpyAsync(d_slot, s0.data(), nmol * sizeof(int), hipMemcpyHostToDevice, st));
        HIPCK(hfx_bscf_pack(c->d_H, c->d_moff, c->d_mdim, nmol, NP, Fx.p, st));
        HIPCK(hfx_bscf_ring_store(Fx.p, nmol, NP, d_slot, dring, ringF.p, st));
        std::fill(coefh.begin(), coefh.end(), 0.0);
        for (int m = 0; m < nmol; ++m) coefh[(size_t)m * dring] = 1.0;
        HIPCK(hipMemcpyAsync(coef.p, coefh.data(), coefh.size() * 8, hipMemcpyHostToDevice, st));
        hfx_status s = seg_b();
        if (s == HFX_OK) s = eig();
        if (s == HFX_OK) s = seg_c();
        if (s != HFX_OK) return s;
        HIPCK(hipMemsetAsync(ringF.p, 0, all * dring * 8, st));
    } else {
        HIPCK(hfx_bscf_pack(D.p, c->d_moff, c->d_mdim, nmol, NP, Dp.p, st));
    }
    double t_fock = 0.0;
    int nconv = 0;
    for (int it = 1; it <= o.max_iter && nconv < nmol; ++it) {
        // ring slot of this iteration's vector per active molecule
        for (int m = 0; m < nmol; ++m) {
            Mol& M = mols[m];
            if (M.converged) {
                slot_h[m] = -1;
                continue;
            }
            if (dmax > 0) {
                int sl;
                diis_make_room(M.B, M.m, M.head, dmax, &sl);
                slot_h[m] = sl;
            } else {
                slot_h[m] = 0;
            }
        }
        HIPCK(hipMemcpyAsync(d_slot, slot_h.data(), nmol * sizeof(int), hipMemcpyHostToDevice, st));
        auto tf = std::chrono::steady_clock::now();
        hfx_status s = run(ga, seg_a, it > 1);
        if (s != HFX_OK) return s;
        HIPCK(hipMemcpyAsync(Eh.data(), dE.p, nmol * 8, hipMemcpyDeviceToHost, st));
        HIPCK(hipMemcpyAsync(dotsh.data(), dots.p, dotsh.size() * 8, hipMemcpyDeviceToHost, st));
        HIPCK(hipStreamSynchronize(st));
        t_fock += std::chrono::duration<double>(std::chrono::steady_clock::now() - tf).count();
        std::fill(coefh.begin(), coefh.end(), 0.0);
        for (int m = 0; m < nmol; ++m) {
            Mol& M = mols[m];
            if (M.converged) continue;
            const double Ek = Eh[m] + c->mol[m].enuc;
            if (!std::isfinite(Ek)) return hfx_fail(c, HFX_ERR_NUMERICAL, "hfx_batch_scf: non-finite energy");
            M.energy = Ek;
            M.iterations = it;
            double* cm = coefh.data() + (size_t)m * dring;
            if (dmax == 0) {
                cm[0] = 1.0;
                continue;
            }
            for (int i = 0; i < M.m; ++i) {   // the new last row and column of B
                const double v = dotsh[(size_t)m * dring + (M.head + i) % dmax];
                M.B[i * M.m + (M.m - 1)] = v;
                M.B[(M.m - 1) * M.m + i] = v;
            }
            int use = M.m;
            std::vector<double> cf;
            while (use >= 2) {
                const int q = use + 1;
                std::vector<double> A((size_t)q * q, 0.0);
                for (int i = 0; i < use; ++i)
                    for (int j = 0; j < use; ++j) A[i * q + j] = M.B[i * M.m + j];
                for (int i = 0; i < use; ++i) A[i * q + use] = A[use * q + i] = -1.0;
                std::vector<double> ev = small_sym_eigs(A, q);
                double amax = 0.0, amin = 1e300;
                for (double e : ev) {
                    amax = std::max(amax, std::fabs(e));
                    amin = std::min(amin, std::fabs(e));
                }
                std::vector<double> rhs(q, 0.0);
                rhs[use] = -1.0;
                if (amin > 0.0 && amax / amin <= 1e14 && small_solve(A, rhs, q)) {
                    cf.assign(rhs.begin(), rhs.begin() + use);
                    break;
                }
                M.head = (M.head + 1) % dmax;   // drop the oldest vector
                std::vector<double> nb((size_t)(M.m - 1) * (M.m - 1));
                for (int i = 1; i < M.m; ++i)
                    for (int j = 1; j < M.m; ++j) nb[(i - 1) * (M.m - 1) + (j - 1)] = M.B[i * M.m + j];
                M.B.swap(nb);
                --M.m;
                use = M.m;
            }
            if (cf.empty())
                cm[slot_h[m]] = 1.0;   // no extrapolation: this iteration's F
            else
                for (int i = 0; i < M.m; ++i) cm[(M.head + i) % dmax] = cf[i];
        }
        HIPCK(hipMemcpyAsync(coef.p, coefh.data(), coefh.size() * 8, hipMemcpyHostToDevice, st));
        s = run(gb, seg_b, it > 1);
        if (s == HFX_OK) s = eig();
        if (s == HFX_OK) s = run(gc, seg_c, it > 1);
        if (s != HFX_OK) return s;
        HIPCK(hipMemcpyAsync(sqh.data(), dsq.p, nmol * 8, hipMemcpyDeviceToHost, st));
        HIPCK(hipMemcpyAsync(infoh.data(), info, nmol * sizeof(rocblas_int), hipMemcpyDeviceToHost, st));
        HIPCK(hipStreamSynchronize(st));
        bool changed = false;
        for (int m = 0; m < nmol; ++m) {
            Mol& M = mols[m];
            if (M.converged) continue;
            if (infoh[m] != 0) return hfx_fail(c, HFX_ERR_NUMERICAL, "hfx_batch_scf: eigensolver did not converge");
            const int n = c->mol[m].nbf;
            const double drms = std::sqrt(sqh[m] / ((double)n * n));
            if (M.have_old && std::fabs(M.energy - M.e_old) < o.e_tol && drms < o.d_rms_tol) {
                M.converged = true;
                active[m] = 0;
                changed = true;
                ++nconv;
            }
            M.e_old = M.energy;
            M.have_old = true;
        }
        if (changed) HIPCK(hipMemcpyAsync(d_active, active.data(), nmol * sizeof(int), hipMemcpyHostToDevice, st));
        if (c->opt.log_level > 0)
            std::fprintf(stderr, "[hfx batch scf, graphs] it %3d  converged %d / %d\n", it, nconv, nmol);
    }
    HIPCK(hipStreamSynchronize(st));
    const double t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int m = 0; m < nmol; ++m) {
        const Mol& M = mols[m];
        res[m].energy = M.energy;
        res[m].e_nuc = c->mol[m].enuc;
        res[m].iterations = M.iterations;
        res[m].converged = M.converged ? 1 : 0;
        res[m].guess_used = guess_used;
        res[m].ndropped = ndrop[m];
        res[m].t_fock_s = t_fock;
        res[m].t_total_s = t_total;
    }
    if (segments_captured) *segments_captured = captured;
    if (D_out) HIPCK(hipMemcpy(D_out, D.p, ne * 8, hipMemcpyDeviceToHost));
    return nconv == nmol ? HFX_OK : hfx_fail(c, HFX_ERR_NOT_CONVERGED, "hfx_batch_scf: not converged within max_iter");
}

extern "C" hfx_status hfx_batch_scf(hfx_ctx* c, const hfx_scf_options* opt, hfx_scf_result* res, double* D_out) {
    if (!c || !res) return c ? hfx_fail(c, HFX_ERR_INVALID_ARG, "null pointer") : HFX_ERR_INVALID_ARG;
    if (!c->loaded) return hfx_fail(c, HFX_ERR_STATE, "hfx_batch_scf: nothing loaded");
    hfx_scf_options o;
    if (opt) o = *opt; else hfx_default_scf_options(&o);
    if (o.max_iter < 1 || o.diis_max < 0 || o.diis_max > 32 || !(o.e_tol > 0) || !(o.d_rms_tol > 0) ||
        !(o.lindep > 0) || !(o.lindep < 1.0) || o.graph < 0 || o.graph > 1)
        return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_batch_scf: invalid options");
    if (o.guess == HFX_GUESS_LEARNED && !o.D0)
        return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_batch_scf: the learned guess runs per molecule (hfx_scf)");
    HIPCK(hipSetDevice(c->opt.device));
    if (o.graph) {
        int segs = 0;
        hfx_status s = batch_scf_graph(c, o, res, D_out, &segs);
        if (s == HFX_OK || s == HFX_ERR_NOT_CONVERGED)
            for (int m = 0; m < c->nmol; ++m) res[m].graph_segments = segs;
        return s;
    }
    for (int m = 0; m < c->nmol; ++m) res[m].graph_segments = 0;
    auto t0 = std::chrono::steady_clock::now();
    const int nmol = c->nmol;
    const size_t ne = c->nelem;
    rocblas_handle h = c->blas;
    hipStream_t st = 0;
    BLASCK(rocblas_set_stream(h, st));
    BLASCK(rocblas_set_pointer_mode(h, rocblas_pointer_mode_host));
    const double one = 1.0, zero = 0.0;

    // ---- guess ----
    DevBuf D;
    HIPCK(D.alloc(ne));
    bool core = false;
    int guess_used = o.guess;
    if (o.D0) {
        for (size_t i = 0; i < ne; ++i)
            if (!std::isfinite(o.D0[i])) return hfx_fail(c, HFX_ERR_NUMERICAL, "hfx_batch_scf: non-finite D0");
        HIPCK(hipMemcpy(D.p, o.D0, ne * 8, hipMemcpyHostToDevice));
        guess_used = -1;
    } else if (o.guess == HFX_GUESS_CORE) {
        core = true;
    } else if (o.guess == HFX_GUESS_SAD) {
        std::vector<double> Ds;
        hfx_status s = sad_guess(c, Ds);
        if (s != HFX_OK) return s;
        HIPCK(hipMemcpy(D.p, Ds.data(), ne * 8, hipMemcpyHostToDevice));
    } else {
        return hfx_fail(c, HFX_ERR_INVALID_ARG, "hfx_batch_scf: unknown guess");
    }

    // ---- orthogonalisers from one batched eigensolve of the S blocks ----
    const int NP = std::max(1, c->max_ld);
    const size_t slot = (size_t)NP * NP;
    DevBuf P, Wv, Ew;
    HIPCK(P.alloc(slot * nmol));
    HIPCK(Wv.alloc((size_t)NP * nmol));
    HIPCK(Ew.alloc((size_t)NP * nmol));
    rocblas_int* info = nullptr;
    HIPCK(hipMalloc((void**)&info, nmol * sizeof(rocblas_int)));
    struct InfoFree { rocblas_int* p; ~InfoFree() { if (p) (void)hipFree(p); } } info_free{info};
    std::vector<rocblas_int> infoh(nmol);
    auto batched_eig = [&]() -> hfx_status {
        BLASCK(rocsolver_dsyevd_strided_batched(h, rocblas_evect_original, rocblas_fill_upper, NP, P.p, NP,
                                                (rocblas_stride)slot, Wv.p, NP, Ew.p, NP, info, nmol));
        HIPCK(hipMemcpy(infoh.data(), info, nmol * sizeof(rocblas_int), hipMemcpyDeviceToHost));
        return HFX_OK;
    };
    HIPCK(hfx_pad_blocks(c->d_S, c->d_moff, c->d_mdim, nmol, NP, kPadDiag, P.p, st));
    hfx_status s = batched_eig();
    if (s != HFX_OK) return s;
    for (int m = 0; m < nmol; ++m)
        if (infoh[m] != 0) return hfx_fail(c, HFX_ERR_NUMERICAL, "hfx_batch_scf: overlap eigensolve failed");
    std::vector<double> wh((size_t)NP * nmol);
    HIPCK(hipMemcpy(wh.data(), Wv.p, wh.size() * 8, hipMemcpyDeviceToHost));
    const int dmax = std::max(0, o.diis_max);
    std::vector<std::unique_ptr<MolScf>> mols;
    std::vector<int> kdim(nmol);
    for (int m = 0; m < nmol; ++m) {
        auto M = std::make_unique<MolScf>();
        const MolInfo& I = c->mol[m];
        M->n = I.nbf;
        M->nocc = I.nocc;
        M->moff = I.moff;
        M->enuc = I.enuc;
        const int n = M->n;
        std::vector<int> keep;
        for (int i = 0; i < n; ++i)
            if (wh[(size_t)m * NP + i] >= o.lindep) keep.push_back(i);
        M->nk = (int)keep.size();
        M->ndropped = n - M->nk;
        if (M->nk < std::max(1, M->nocc))
            return hfx_fail(c, HFX_ERR_NUMERICAL, "hfx_batch_scf: overlap matrix too singular for the occupied space");
        kdim[m] = M->nk;
        const int nk = M->nk;
        DevBuf U, Us;
        HIPCK(U.alloc((size_t)n * n));
        HIPCK(Us.alloc((size_t)n * nk));
        HIPCK(hipMemcpy2D(U.p, (size_t)n * 8, P.p + (size_t)m * slot, (size_t)NP * 8, (size_t)n * 8, n,
                          hipMemcpyDeviceToDevice));
        int* dk = nullptr;
        HIPCK(hipMalloc((void**)&dk, nk * sizeof(int)));
        HIPCK(hipMemcpy(dk, keep.data(), nk * sizeof(int), hipMemcpyHostToDevice));
        hipError_t e = hfx_scale_cols(U.p, Wv.p + (size_t)m * NP, dk, n, nk, Us.p, st);
        (void)hipFree(dk);
        HIPCK(e);
        HIPCK(M->X.alloc((size_t)n * nk));
        if (nk == n) {
            BLASCK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, n, n, n, &one, Us.p, n, U.p, n,
                                 &zero, M->X.p, n));
        } else {
            HIPCK(hipMemcpy(M->X.p, Us.p, (size_t)n * nk * 8, hipMemcpyDeviceToDevice));
        }
        const size_t nn = (size_t)n * n;
        HIPCK(M->T1.alloc(nn));
        HIPCK(M->T2.alloc(nn));
        HIPCK(M->Dn.alloc(nn));
        HIPCK(M->Fx.alloc(nn));
        HIPCK(M->C.alloc((size_t)n * std::max(1, M->nocc)));
        HIPCK(M->Fh.alloc(nn * std::max(1, dmax)));
        HIPCK(M->Eh.alloc((size_t)nk * nk * std::max(1, dmax)));
        mols.push_back(std::move(M));
    }
    int* dkdim = nullptr;
    HIPCK(hipMalloc((void**)&dkdim, nmol * sizeof(int)));
    struct IntFree { int* p; ~IntFree() { if (p) (void)hipFree(p); } } kdim_free{dkdim};
    HIPCK(hipMemcpy(dkdim, kdim.data(), nmol * sizeof(int), hipMemcpyHostToDevice));
    HIPCK(hfx_pad_blocks(c->d_S, c->d_moff, c->d_mdim, nmol, NP, kPadDiag, P.p, st));   // finite start in every slot

    DevBuf F, part;
    HIPCK(F.alloc(ne));
    HIPCK(part.alloc(4096));
    std::vector<double> parth(4096);
    bool ok = true;

    // X^T M X into molecule m's slot
    auto project = [&](MolScf& M, const double* Mat, int m) -> hfx_status {
        BLASCK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, M.n, M.nk, M.n, &one, Mat, M.n, M.X.p,
                             M.n, &zero, M.T1.p, M.n));
        BLASCK(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, M.nk, M.nk, M.n, &one, M.X.p, M.n,
                             M.T1.p, M.n, &zero, P.p + (size_t)m * slot, NP));
        return HFX_OK;
    };
    // aufbau density of molecule m from its solved slot, into Dn
    auto density = [&](MolScf& M, int m) -> hfx_status {
        if (infoh[m] != 0) return hfx_fail(c, HFX_ERR_NUMERICAL, "hfx_batch_scf: eigensolver did not converge");
        BLASCK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, M.n, M.nocc, M.nk, &one, M.X.p, M.n,
                             P.p + (size_t)m * slot, NP, &zero, M.C.p, M.n));
        BLASCK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, M.n, M.n, M.nocc, &one, M.C.p,
                             M.n, M.C.p, M.n, &zero, M.Dn.p, M.n));
        return HFX_OK;
    };
    if (core) {
        for (int m = 0; m < nmol; ++m) {
            s = project(*mols[m], c->d_H + mols[m]->moff, m);
            if (s != HFX_OK) return s;
        }
        HIPCK(hfx_pad_rest(dkdim, nmol, NP, kPadDiag, P.p, st));
        s = batched_eig();
        if (s != HFX_OK) return s;
        for (int m = 0; m < nmol; ++m) {
            MolScf& M = *mols[m];
            s = density(M, m);
            if (s != HFX_OK) return s;
            HIPCK(hipMemcpy(D.p + M.moff, M.Dn.p, (size_t)M.n * M.n * 8, hipMemcpyDeviceToDevice));
        }
    }

    double t_fock = 0.0;
    int nconv = 0;
    for (int it = 1; it <= o.max_iter && nconv < nmol; ++it) {
        auto tf = std::chrono::steady_clock::now();
        s = hfx_build_internal(c, D.p, 2.0, 1.0, c->d_H, F.p, st, nullptr, 0, 1);
        if (s != HFX_OK) return s;
        HIPCK(hipStreamSynchronize(st));
        t_fock += std::chrono::duration<double>(std::chrono::steady_clock::now() - tf).count();
        for (int m = 0; m < nmol; ++m) {
            MolScf& M = *mols[m];
            if (M.converged) continue;
            const int n = M.n, nk = M.nk;
            const size_t nn = (size_t)n * n;
            const double* Dm = D.p + M.moff;
            const double* Fm = F.p + M.moff;
            const double* Sm = c->d_S + M.moff;
            int np = hfx_energy_partial(Dm, c->d_H + M.moff, Fm, nn, part.p, st);
            const double Ek = dev_sum(c, np, part, parth, ok) + M.enuc;
            if (!ok) return hfx_fail(c, HFX_ERR_DEVICE, "hfx_batch_scf: copy failed");
            if (!std::isfinite(Ek)) return hfx_fail(c, HFX_ERR_NUMERICAL, "hfx_batch_scf: non-finite energy");
            M.energy = Ek;
            M.iterations = it;
            const double* Fuse = Fm;
            if (dmax > 0) {   // Pulay DIIS on X^T (F D S - S D F) X, as in the single-molecule driver
                BLASCK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, n, n, &one, Fm, n, Dm, n,
                                     &zero, M.T1.p, n));
                BLASCK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, n, n, &one, M.T1.p, n, Sm, n,
                                     &zero, M.T2.p, n));
                HIPCK(hfx_antisym(M.T2.p, n, M.T1.p, st));
                BLASCK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, nk, n, &one, M.T1.p, n,
                                     M.X.p, n, &zero, M.T2.p, n));
                int sl;
                diis_make_room(M.B, M.m, M.head, dmax, &sl);
                double* eslot = M.Eh.p + (size_t)sl * nk * nk;
                BLASCK(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, nk, nk, n, &one, M.X.p, n,
                                     M.T2.p, n, &zero, eslot, nk));
                HIPCK(hipMemcpy(M.Fh.p + (size_t)sl * nn, Fm, nn * 8, hipMemcpyDeviceToDevice));
                for (int i = 0; i < M.m; ++i) {   // the new last row and column of B
                    const int si = (M.head + i) % dmax;
                    int np2 = hfx_dot_partial(M.Eh.p + (size_t)si * nk * nk, eslot, (size_t)nk * nk, 0, part.p, st);
                    const double v = dev_sum(c, np2, part, parth, ok);
                    if (!ok) return hfx_fail(c, HFX_ERR_DEVICE, "hfx_batch_scf: copy failed");
                    M.B[i * M.m + (M.m - 1)] = v;
                    M.B[(M.m - 1) * M.m + i] = v;
                }
                int use = M.m;
                std::vector<double> coef;
                while (use >= 2) {
                    const int q = use + 1;
                    std::vector<double> A((size_t)q * q, 0.0);
                    for (int i = 0; i < use; ++i)
                        for (int j = 0; j < use; ++j) A[i * q + j] = M.B[i * M.m + j];
                    for (int i = 0; i < use; ++i) A[i * q + use] = A[use * q + i] = -1.0;
                    std::vector<double> ev = small_sym_eigs(A, q);
                    double amax = 0.0, amin = 1e300;
                    for (double e : ev) {
                        amax = std::max(amax, std::fabs(e));
                        amin = std::min(amin, std::fabs(e));
                    }
                    std::vector<double> rhs(q, 0.0);
                    rhs[use] = -1.0;
                    if (amin > 0.0 && amax / amin <= 1e14 && small_solve(A, rhs, q)) {
                        coef.assign(rhs.begin(), rhs.begin() + use);
                        break;
                    }
                    M.head = (M.head + 1) % dmax;   // drop the oldest vector
                    std::vector<double> nb((size_t)(M.m - 1) * (M.m - 1));
                    for (int i = 1; i < M.m; ++i)
                        for (int j = 1; j < M.m; ++j) nb[(i - 1) * (M.m - 1) + (j - 1)] = M.B[i * M.m + j];
                    M.B.swap(nb);
                    --M.m;
                    use = M.m;
                }
                if (!coef.empty()) {
                    std::vector<const double*> ptrs(M.m);
                    for (int i = 0; i < M.m; ++i) ptrs[i] = M.Fh.p + (size_t)((M.head + i) % dmax) * nn;
                    const double** dptrs = nullptr;
                    double* dcoef = nullptr;
                    HIPCK(hipMalloc((void**)&dptrs, M.m * sizeof(double*)));
                    HIPCK(hipMalloc((void**)&dcoef, M.m * sizeof(double)));
                    HIPCK(hipMemcpy(dptrs, ptrs.data(), M.m * sizeof(double*), hipMemcpyHostToDevice));
                    HIPCK(hipMemcpy(dcoef, coef.data(), M.m * sizeof(double), hipMemcpyHostToDevice));
                    hipError_t e = hfx_lincomb(dptrs, dcoef, M.m, nn, M.Fx.p, st);
                    if (e == hipSuccess) e = hipStreamSynchronize(st);
                    (void)hipFree(dptrs);
                    (void)hipFree(dcoef);
                    HIPCK(e);
                    Fuse = M.Fx.p;
                }
            }
            s = project(M, Fuse, m);
            if (s != HFX_OK) return s;
        }
        HIPCK(hfx_pad_rest(dkdim, nmol, NP, kPadDiag, P.p, st));
        s = batched_eig();
        if (s != HFX_OK) return s;
        for (int m = 0; m < nmol; ++m) {
            MolScf& M = *mols[m];
            if (M.converged) continue;
            s = density(M, m);
            if (s != HFX_OK) return s;
            const size_t nn = (size_t)M.n * M.n;
            double* Dm = D.p + M.moff;
            int np = hfx_dot_partial(M.Dn.p, Dm, nn, 1, part.p, st);
            const double drms = std::sqrt(dev_sum(c, np, part, parth, ok) / (double)nn);
            if (!ok) return hfx_fail(c, HFX_ERR_DEVICE, "hfx_batch_scf: copy failed");
            HIPCK(hipMemcpy(Dm, M.Dn.p, nn * 8, hipMemcpyDeviceToDevice));
            if (M.have_old && std::fabs(M.energy - M.e_old) < o.e_tol && drms < o.d_rms_tol) {
                M.converged = true;
                ++nconv;
            }
            M.e_old = M.energy;
            M.have_old = true;
        }
        if (c->opt.log_level > 0)
            std::fprintf(stderr, "[hfx batch scf] it %3d  converged %d / %d\n", it, nconv, nmol);
    }
    const double t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int m = 0; m < nmol; ++m) {
        const MolScf& M = *mols[m];
        res[m].energy = M.energy;
        res[m].e_nuc = M.enuc;
        res[m].iterations = M.iterations;
        res[m].converged = M.converged ? 1 : 0;
        res[m].guess_used = guess_used;
        res[m].ndropped = M.ndropped;
        res[m].t_fock_s = t_fock;
        res[m].t_total_s = t_total;
    }
    if (D_out) HIPCK(hipMemcpy(D_out, D.p, ne * 8, hipMemcpyDeviceToHost));
    return nconv == nmol ? HFX_OK : hfx_fail(c, HFX_ERR_NOT_CONVERGED, "hfx_batch_scf: not converged within max_iter");
}
