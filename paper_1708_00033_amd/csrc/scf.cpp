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
#include <map>
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
            // push: slot for the new vector
            int slot;
            if (m < dmax) {
                slot = (head + m) % dmax;
                ++m;
            } else {   // drop the oldest
                slot = head;
                head = (head + 1) % dmax;
                std::vector<double> nb((size_t)m * m);
                for (int i = 1; i < m; ++i)
                    for (int j = 1; j < m; ++j) nb[(i - 1) * m + (j - 1)] = B[i * m + j];
                B.swap(nb);
            }
            double* eslot = Eh.p + (size_t)slot * nk * nk;
            BLASCK(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, nk, nk, n, &one, X.p, n, T2.p,
                                 n, &zero, eslot, nk));
            HIPCK(hipMemcpy(Fh.p + (size_t)slot * nn, F.p, nn * 8, hipMemcpyDeviceToDevice));
            B.resize((size_t)m * m, 0.0);
            {   // rebuild B with the new last row/column
                std::vector<double> nb((size_t)m * m, 0.0);
                const int mo = (int)std::sqrt((double)B.size());
                (void)mo;
                for (int i = 0; i < m - 1; ++i)
                    for (int j = 0; j < m - 1; ++j) nb[i * m + j] = B[i * (m) + j];
                for (int i = 0; i < m; ++i) {
                    const int si = (head + i) % dmax;
                    int np2 = hfx_dot_partial(Eh.p + (size_t)si * nk * nk, eslot, (size_t)nk * nk, 0, part.p, st);
                    HIPCK(hipMemcpy(parth.data(), part.p, np2 * 8, hipMemcpyDeviceToHost));
                    const double v = host_sum(parth, np2);
                    nb[i * m + (m - 1)] = v;
                    nb[(m - 1) * m + i] = v;
                }
                B.swap(nb);
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

// SAD: block-diagonal superposition of per-element atomic densities.
static hfx_status sad_guess(hfx_ctx* c, std::vector<double>& Dsad) {
    const int n = c->nbf;
    Dsad.assign((size_t)n * n, 0.0);
    for (int a = 0; a < c->natom; ++a) {
        const int z = c->Z[a];
        std::vector<int> sh;
        for (int s = 0; s < c->nshell; ++s)
            if (c->shell_atom[s] == a) sh.push_back(s);
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
            for (int j = 0; j < na; ++j) Dsad[(size_t)(o0 + i) * n + o0 + j] = Da[(size_t)i * na + j];
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
