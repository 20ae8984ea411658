/*
 * hfx.h -- C ABI of the MI355X direct closed-shell Hartree-Fock library.
 *
 * The library builds the closed-shell Fock matrix F = H + 2J - K directly
 * from Schwarz-screened electron repulsion integrals over contracted
 * Cartesian Gaussian shells (Mironov et al., SC17, "An efficient MPI/OpenMP
 * parallelization of the Hartree-Fock method for the second generation of
 * Intel Xeon Phi processor": section 3 for the SCF problem F C = eps S C
 * (eq. 1), section 4.1 for the symmetry-unique quartet loop with
 * Cauchy-Schwarz screening and the six Fock updates per integral (eq. 2)).
 * All arithmetic of a build runs on one AMD Instinct MI355X (gfx950) in
 * hand-written HIP kernels.
 *
 * Conventions
 *   units           bohr, hartree
 *   matrices        nbf x nbf, FP64, row-major, full symmetric storage
 *   basis order     atoms in input order, then shells in input order, then
 *                   Cartesian components lexicographically:
 *                   p: x y z;  d: xx xy xz yy yz zz
 *   normalisation   every Cartesian component has unit norm; contraction
 *                   coefficients refer to unit-normalised primitives and the
 *                   contraction is renormalised to unit self-overlap
 *   density         D = C_occ C_occ^T (no factor 2); F = H + 2J - K with
 *                   J_mn = sum_ls (mn|ls) D_ls, K_mn = sum_ls (ml|ns) D_ls
 *   screening       a unique shell quartet (ab|cd) is evaluated iff
 *                   Q_ab Q_cd >= schwarz_tau, Q_ab = sqrt(max (mn|mn))
 *
 * Ownership: host arrays passed in are copied (the caller keeps them); the
 * _dev entry points take caller-owned device pointers and a caller-owned
 * HIP stream, only enqueue work on that stream and never synchronise unless
 * a statistics pointer is passed.
 *
 * Errors: every call returns hfx_status (0 == HFX_OK).  On error the output
 * arguments are left untouched and hfx_last_error() describes the problem.
 * No call aborts or exits.  A context is not thread-safe; distinct contexts
 * are independent.
 */
#ifndef HFX_H
#define HFX_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HFX_OK = 0,
    HFX_ERR_INVALID_ARG = 1,   /* bad pointer, size, shell (l > 2, alpha <= 0), non-finite input */
    HFX_ERR_OOM = 2,           /* device or host allocation failed */
    HFX_ERR_DEVICE = 3,        /* a HIP / rocBLAS / rocSOLVER call failed */
    HFX_ERR_NOT_CONVERGED = 4, /* SCF reached max_iter */
    HFX_ERR_NUMERICAL = 5,     /* NaN/Inf in a density, Fock matrix or eigensolve */
    HFX_ERR_STATE = 6          /* call made in the wrong state (e.g. build before load) */
} hfx_status;

typedef struct hfx_ctx hfx_ctx;

/* One shell: atom index, angular momentum l (0, 1 or 2), nprim primitives
 * with exponents exps[nprim] (> 0) and coefficients coefs[nprim] of
 * unit-normalised primitives (section 4.1: a shell groups the functions of
 * one atom sharing exponents and coefficients). */
typedef struct {
    int atom, l, nprim;
    const double *exps, *coefs;
} hfx_shell;

enum { HFX_PREC_FP64 = 0, HFX_PREC_MIXED = 1 };
enum { HFX_DIGEST_LDS = 0, HFX_DIGEST_GLOBAL = 1 };
enum { HFX_GUESS_SAD = 0, HFX_GUESS_CORE = 1 };

typedef struct {
    int device;            /* HIP device ordinal */
    double schwarz_tau;    /* quartet kept iff Q_ab Q_cd >= tau (default 1e-10) */
    int precision;         /* HFX_PREC_FP64 or HFX_PREC_MIXED */
    double fp32_tau;       /* MIXED: FP32 iff Q_ab Q_cd max|D| < fp32_tau (default 1e-7) */
    int digest;            /* HFX_DIGEST_LDS (bra rows staged in LDS) or HFX_DIGEST_GLOBAL */
    int task_quartets;     /* quartets per workgroup task (default 8192; multiple of 256) */
    int log_level;         /* 0 silent, 1 SCF iterations to stderr */
} hfx_options;

typedef struct {
    int max_iter;          /* default 100 */
    double e_tol;          /* |E_k - E_{k-1}| < e_tol (default 1e-8) */
    double d_rms_tol;      /* and rms(D_{k+1} - D_k) < d_rms_tol (default 1e-7) */
    int diis_max;          /* Pulay DIIS subspace (default 8; 0 disables) */
    int guess;             /* HFX_GUESS_SAD or HFX_GUESS_CORE */
    const double *D0;      /* optional host nbf x nbf restart density (NULL: use guess) */
    double lindep;         /* S eigenvalues below this are dropped (default 1e-7) */
} hfx_scf_options;

typedef struct {
    double energy, e_nuc;
    int iterations, converged, guess_used, ndropped;
    double t_total_s, t_fock_s;
} hfx_scf_result;

typedef struct {
    long long quartets_fp64, quartets_fp32, integrals, prim_quartets;
    double t_s;            /* wall time of the build (host-synchronous variants only) */
} hfx_fock_stats;

/* Fill defaults (values listed in the struct comments). */
hfx_status hfx_default_options(hfx_options *opt);
hfx_status hfx_default_scf_options(hfx_scf_options *opt);

/* Create a context on opt->device.  *out owns all device memory it allocates. */
hfx_status hfx_create(const hfx_options *opt, hfx_ctx **out);

/* Load geometry and basis (section 4.1 shells).  Z[natom] nuclear charges,
 * xyz_bohr[natom*3], shells[nshell] (copied).  Computes normalisation,
 * shell-pair data, Schwarz bounds (on the GPU), the screened quartet plan,
 * and S, H = T + V, E_nuc.  charge: total molecular charge (even electron
 * count required).  Replaces any previously loaded system. */
hfx_status hfx_load(hfx_ctx *ctx, int natom, const int *Z, const double *xyz_bohr, int nshell,
                    const hfx_shell *shells, int charge);

/* Load a batch of nmol independent molecules (one context, one launch per
 * quartet class for all of them).  Molecule m has natom[m] atoms and
 * nshell[m] shells; Z, xyz_bohr and shells are the concatenations in molecule
 * order, each shell's atom index counting within its molecule; charge may be
 * NULL (all neutral).  Pairs and quartets never mix molecules.  All matrices
 * of a batch (D, F, S, H) are ragged: molecule m's nbf_m x nbf_m block at
 * element offset offset[m] (hfx_batch_layout).  hfx_load is the nmol = 1 case. */
hfx_status hfx_load_batch(hfx_ctx *ctx, int nmol, const int *natom, const int *Z, const double *xyz_bohr,
                          const int *nshell, const hfx_shell *shells, const int *charge);

/* Ragged layout of a loaded batch: nbf[nmol], nocc[nmol], offset[nmol] (any
 * may be NULL) and the total element count. */
hfx_status hfx_batch_layout(const hfx_ctx *ctx, int *nmol, int *nbf, int *nocc, long long *offset,
                            long long *total);

/* Basis size, doubly occupied orbitals, shells (totals over a batch). */
hfx_status hfx_dims(const hfx_ctx *ctx, int *nbf, int *nocc, int *nshell);

/* Host copies of S and H (ragged layout; nbf x nbf for one molecule) and the
 * total E_nuc; any pointer may be NULL. */
hfx_status hfx_core(hfx_ctx *ctx, double *S, double *H, double *e_nuc);

/* Schwarz bounds as an nshell x nshell host matrix. */
hfx_status hfx_schwarz(hfx_ctx *ctx, double *Q);

/* F = H + 2J(D) - K(D) (section 4.1, eq. 2) from a host density; host F. */
hfx_status hfx_build_fock(hfx_ctx *ctx, const double *D, double *F, hfx_fock_stats *stats);

/* Device variant: dD, dF device pointers (nbf x nbf FP64), stream a
 * hipStream_t (NULL = default stream).  Enqueues only; if stats != NULL the
 * call synchronises the stream to read the quartet counters. */
hfx_status hfx_build_fock_dev(hfx_ctx *ctx, const double *dD, double *dF, void *stream,
                              hfx_fock_stats *stats);

/* Two-electron part only: dG = cj J(D) - ck K(D) (device pointers).  cj=2,
 * ck=1 gives F - H; cj=1, ck=0 gives J; cj=0, ck=-1 gives K. */
hfx_status hfx_build_2e_dev(hfx_ctx *ctx, const double *dD, double cj, double ck, double *dG,
                            void *stream, hfx_fock_stats *stats);

/* Capture one Fock build dF = F(dD) on a non-null stream into a HIP graph
 * (an eager build runs first), and replay it.  The graph keeps dD, dF and
 * the context's buffers; re-capture after hfx_load, hfx_configure or
 * hfx_set_class_tuning. */
hfx_status hfx_graph_capture(hfx_ctx *ctx, const double *dD, double *dF, void *stream);
hfx_status hfx_graph_launch(hfx_ctx *ctx, void *stream);

/* One GPU's share of a multi-GPU build: dG = cj J - ck K restricted to the
 * bra shell pairs r with r % nshards == shard (r = position in each class's
 * Schwarz-ordered bra list).  Summing the nshards results gives the full
 * two-electron matrix (the partial Fock matrices that the paper's
 * ddi_gsumf reduces in algorithms 1-3). */
hfx_status hfx_build_2e_shard_dev(hfx_ctx *ctx, const double *dD, double cj, double ck, int shard,
                                  int nshards, double *dG, void *stream);

/* Closed-shell SCF to convergence (section 3, eq. 1): guess, Fock build,
 * Pulay DIIS, eigensolve of X^T F X, aufbau density.  D_out, C_out
 * (nbf x nmo, nmo = nbf - dropped), eps_out (nmo) are optional host arrays.
 * Returns HFX_ERR_NOT_CONVERGED (with *res filled) at max_iter. */
hfx_status hfx_scf(hfx_ctx *ctx, const hfx_scf_options *opt, hfx_scf_result *res, double *D_out,
                   double *C_out, double *eps_out);

/* Change precision / digestion / task size of a loaded context (schwarz_tau
 * and device must stay as created). */
hfx_status hfx_configure(hfx_ctx *ctx, const hfx_options *opt);

/* Per-class scheduling knobs (class index 0..20, or -1 for all): quartets
 * per workgroup task (0: the context's task_quartets) and XCD striping of
 * long ket prefixes (1 on, 0 off, -1 default on).  Re-plans a loaded
 * system; results are unchanged, only the work decomposition moves.  Set by
 * the autotuner (paper_1708_00033_amd/autotune.py). */
hfx_status hfx_set_class_tuning(hfx_ctx *ctx, int cls, int task_quartets, int xcd_stripe);

/* Per-class plan counts: counts[21*4] = {unique quartets, integrals,
 * primitive quartets, workgroup tasks} for each canonical quartet class in
 * the order (ss|ss), (ps|ss), (ps|ps), (pp|ss), ..., (dd|dd). */
hfx_status hfx_class_counts(const hfx_ctx *ctx, long long *counts);

/* Kernel timing: when enabled, every class kernel launch is bracketed by HIP
 * events on its stream; hfx_kernel_times returns per class the summed
 * milliseconds of its launches and the number of timed builds since the last
 * reset (synchronises on the recorded events). */
hfx_status hfx_kernel_timing(hfx_ctx *ctx, int enable);
hfx_status hfx_kernel_times(hfx_ctx *ctx, double *ms, long long *launches);

/* Launches of a build: one per (quartet class, ket primitive count).  info[9]
 * = {class index, ket primitives per pair, workgroups (one task each),
 * unique quartets, primitive quartets, integrals, timed launches, digestion
 * mode, work-items per workgroup}; *ms = summed event time of the timed
 * launches. */
hfx_status hfx_plan_count(const hfx_ctx *ctx, int *n);
hfx_status hfx_plan_info(hfx_ctx *ctx, int i, long long *info, double *ms);

const char *hfx_last_error(const hfx_ctx *ctx);
void hfx_destroy(hfx_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* HFX_H */
