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
    HFX_ERR_INVALID_ARG = 1,   /* bad pointer, size, shell (l not in -1..2, alpha <= 0), non-finite input */
    HFX_ERR_OOM = 2,           /* device or host allocation failed */
    HFX_ERR_DEVICE = 3,        /* a HIP / rocBLAS / rocSOLVER call failed */
    HFX_ERR_NOT_CONVERGED = 4, /* SCF reached max_iter */
    HFX_ERR_NUMERICAL = 5,     /* NaN/Inf in a density, Fock matrix or eigensolve */
    HFX_ERR_STATE = 6          /* call made in the wrong state (e.g. build before load) */
} hfx_status;

typedef struct hfx_ctx hfx_ctx;

/* One shell: atom index, angular momentum l (0, 1 or 2, or HFX_SHELL_SP),
 * nprim primitives with exponents exps[nprim] (> 0) and coefficients
 * coefs[nprim] of unit-normalised primitives (section 4.1: a shell groups
 * the functions of one atom sharing exponents and coefficients).
 * HFX_SHELL_SP: an SP (L) shell of split-valence bases such as the paper's
 * 6-31G(d) (section 5.2): an s and a p set sharing the exponents, with the s
 * coefficients in coefs and the p coefficients in coefs_p (ignored for other
 * l).  It is loaded as an s shell followed by a p shell, so its functions
 * come in the order s, x, y, z and it counts as two shells wherever shells
 * are counted (hfx_dims, hfx_schwarz). */
#define HFX_SHELL_SP (-1)
typedef struct {
    int atom, l, nprim;
    const double *exps, *coefs;
    const double *coefs_p;
} hfx_shell;

enum { HFX_PREC_FP64 = 0, HFX_PREC_MIXED = 1 };
/* Digestion of the integrals into the Fock matrix (eq. 2):
 *   LDS      the bra's rows of the Fock matrix staged in LDS for a task and
 *            flushed once (algorithm 3's private F_I / F_J buffers);
 *   LDS_D    as LDS, and the bra's rows of the density copied into LDS at
 *            the start of a task, so that the exchange updates read D from
 *            LDS instead of gathering it from global memory (both shells'
 *            rows when they fit in LDS, else shell a's; classes with more
 *            than 64 integrals per quartet, register-tiled launches and
 *            column-windowed rows, above 2048 basis functions, read D from
 *            global memory as LDS does; the default);
 *   GLOBAL   every update a device-wide atomic into one shared matrix;
 *   PRIVATE  every update an atomic into the copy of the matrix private to
 *            the XCD the wave runs on (algorithm 2's private Fock matrices,
 *            one per XCD: 8 copies of sum nbf_m^2 FP64 in HBM), summed by a
 *            reduction kernel after the class launches. */
enum { HFX_DIGEST_LDS = 0, HFX_DIGEST_GLOBAL = 1, HFX_DIGEST_PRIVATE = 2, HFX_DIGEST_LDS_D = 3 };
enum { HFX_GUESS_SAD = 0, HFX_GUESS_CORE = 1, HFX_GUESS_LEARNED = 2 };

/* Learned initial-guess network (see the section "Learned initial guess"). */
typedef struct hfx_guess hfx_guess;

typedef struct {
    int device;            /* HIP device ordinal */
    double schwarz_tau;    /* quartet kept iff Q_ab Q_cd >= tau (default 1e-10) */
    int precision;         /* HFX_PREC_FP64 or HFX_PREC_MIXED */
    double fp32_tau;       /* MIXED: FP32 iff Q_ab Q_cd max|D| < fp32_tau (default
                              1e-7); the classes with a d-d bra and a d-d or d-p
                              ket stay FP64.  One launch per class evaluates each
                              task's FP64 kets and its FP32 suffix (Q-sorted). */
    int digest;            /* HFX_DIGEST_LDS, _GLOBAL, _PRIVATE or _LDS_D */
    int task_quartets;     /* quartets per workgroup task (default 8192; multiple of 256) */
    int log_level;         /* 0 silent, 1 SCF iterations to stderr */
} hfx_options;

typedef struct {
    int max_iter;          /* default 100 */
    double e_tol;          /* |E_k - E_{k-1}| < e_tol (default 1e-8) */
    double d_rms_tol;      /* and rms(D_{k+1} - D_k) < d_rms_tol (default 1e-7) */
    int diis_max;          /* Pulay DIIS subspace (default 8; 0 disables) */
    int guess;             /* HFX_GUESS_SAD, HFX_GUESS_CORE or HFX_GUESS_LEARNED */
    const double *D0;      /* optional host nbf x nbf restart density (NULL: use guess) */
    double lindep;         /* S eigenvalues below this are dropped (default 1e-7) */
    hfx_guess *model;      /* HFX_GUESS_LEARNED: the network (SAD when its
                              prediction is rejected, see hfx_guess_apply) */
    int graph;             /* hfx_batch_scf: 1 = replay each iteration's device work
                              from HIP graphs (default 0: eager launches) */
} hfx_scf_options;

typedef struct {
    double energy, e_nuc;
    int iterations, converged, guess_used, ndropped;
    double t_total_s, t_fock_s;
    int graph_segments;    /* hfx_batch_scf with graph = 1: iteration segments
                              replayed from captured graphs (0..3) */
} hfx_scf_result;

typedef struct {
    long long quartets_fp64, quartets_fp32, integrals, prim_quartets;
    double t_s;            /* wall time of the build (host-synchronous variants only) */
} hfx_fock_stats;

/* Fill defaults (values listed in the struct comments). */
hfx_status hfx_default_options(hfx_options *opt);
hfx_status hfx_default_scf_options(hfx_scf_options *opt);

/* Resources of the quartet-class kernels, read from the code objects'
 * metadata (no launch): out[21*3] = per class {largest per-lane scratch
 * (private segment) in bytes over its kernel variants, largest register
 * count, the scratch budget per lane}.  hfx_create refuses (HFX_ERR_DEVICE)
 * when a class kernel needs more scratch than the budget: the runtime
 * reserves scratch for every wave slot, and a kernel far above the budget
 * can make its queue fail with out-of-resources at launch. */
hfx_status hfx_kernel_resources(int device, long long *out);

/* Create a context on opt->device.  *out owns all device memory it allocates.
 * HFX_ERR_DEVICE: no such device, or a class kernel exceeds the scratch
 * budget (hfx_kernel_resources). */
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

/* Several densities in one pass over the screened integrals (the loop
 * structure shared by UHF, GVB, DFT and CPHF, section 7): each integral is
 * evaluated once and digested for every density.  dD: ndens densities
 * (1 <= ndens <= 64), each nbf x nbf FP64 (ragged layout for a batch),
 * consecutive on the device; dJ, dK (either may be NULL): the J(D_d) and
 * K(D_d) of each density in the same layout, so that for example an
 * unrestricted build forms F_a = H + J_a + J_b - K_a and F_b = H + J_a + J_b
 * - K_b from the alpha and beta densities.  FP64 throughout (the context's
 * precision is ignored).  Digestion as the class's plan: LDS-staged classes
 * keep one set of bra rows per density in LDS and take the densities in
 * groups that fit (the integrals are evaluated once per group), the others
 * use device-wide atomics.  Work buffers of
 * 3 x ndens matrices (and the ket lists' D_cd per density) are allocated on
 * the first call with a larger ndens and kept by the context.  stats as in
 * hfx_build_2e_dev (quartets counted once per quartet). */
hfx_status hfx_build_jk_multi_dev(hfx_ctx *ctx, int ndens, const double *dD, double *dJ, double *dK, void *stream,
                                  hfx_fock_stats *stats);

/* Capture one Fock build dF = F(dD) on a non-null stream into a HIP graph
 * (an eager build runs first), and replay it.  The graph keeps dD, dF and
 * the context's buffers.  hfx_load, hfx_set_class_tuning, and any change of
 * precision, fp32_tau, digestion or task size (hfx_configure,
 * hfx_set_class_precision) discard the graph: hfx_graph_launch then returns
 * HFX_ERR_STATE until the next capture. */
hfx_status hfx_graph_capture(hfx_ctx *ctx, const double *dD, double *dF, void *stream);
hfx_status hfx_graph_launch(hfx_ctx *ctx, void *stream);

/* One GPU's share of a multi-GPU build: dG = cj J - ck K restricted to the
 * bra shell pairs r with r % nshards == shard (r = position in each class's
 * Schwarz-ordered bra list).  Summing the nshards results gives the full
 * two-electron matrix (the partial Fock matrices that the paper's
 * ddi_gsumf reduces in algorithms 1-3).  stats (optional, synchronises):
 * the shard's quartet counts; integral and primitive totals are the whole
 * build's. */
hfx_status hfx_build_2e_shard_dev(hfx_ctx *ctx, const double *dD, double cj, double ck, int shard,
                                  int nshards, double *dG, void *stream, hfx_fock_stats *stats);

/* Two-electron build that allocates nothing, for callers that cannot call
 * hipMalloc (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): dG = cj J - ck K exactly as hfx_build_2e_dev
 * (same kernels, same results), but the per-build scratch -- the accumulator
 * and the component-scaled density (sum of nbf_m^2 FP64 each), the max|D|
 * word, the quartet counters and the launch queue counters -- lives in a
 * fixed 32 MiB device array of the library, one per GPU, held until the
 * process ends, instead of context memory (the context's screened plans and
 * ket lists, made at hfx_load, are read as usual).
 * Limit: 16 x (sum of nbf_m^2) bytes plus 106.5 KiB within 32 MiB (one molecule:
 * nbf <= 1445) and at most 512 launch plans; a larger system gives
 * HFX_ERR_INVALID_ARG and launches nothing.  Every call on a GPU, whatever
 * its context, shares that GPU's array, which keeps the last call's contents;
 * each call clears what it accumulates.  Calls that overlap in time on one
 * GPU (concurrent streams or threads) race and give wrong results; calls
 * ordered on one stream, or synchronised, are safe.  stats as in
 * hfx_build_2e_dev (synchronises). */
hfx_status hfx_build_2e_noalloc_dev(hfx_ctx *ctx, const double *dD, double cj, double ck, double *dG,
                                    void *stream, hfx_fock_stats *stats);

/* Closed-shell SCF to convergence (section 3, eq. 1): guess, Fock build,
 * Pulay DIIS, eigensolve of X^T F X, aufbau density.  D_out, C_out
 * (nbf x nmo, nmo = nbf - dropped), eps_out (nmo) are optional host arrays.
 * Returns HFX_ERR_NOT_CONVERGED (with *res filled) at max_iter. */
hfx_status hfx_scf(hfx_ctx *ctx, const hfx_scf_options *opt, hfx_scf_result *res, double *D_out,
                   double *C_out, double *eps_out);

/* SCF of every molecule of a batch (hfx_load_batch) in lockstep: per
 * iteration one batched Fock build for all molecules, then per molecule the
 * energy and Pulay DIIS, and one batched eigensolve (rocSOLVER, each
 * X^T F X padded to the largest molecule).  opt->graph = 1: the matrices of
 * every molecule live in NP x NP slots (NP = the largest basis) so that each
 * step is one batched launch, and an iteration is three captured HIP graphs
 * -- (a) Fock build, energies, DIIS error X^T (F D S - S D F) X and its Gram
 * row, (b) extrapolation and X^T F X, (c) orbitals, density, rms change --
 * replayed from the second iteration on, with the batched eigensolve and the
 * small DIIS solve (host) between them; a segment whose capture fails runs
 * eagerly (res[].graph_segments tells how many were captured).  guess: SAD or CORE, or
 * opt->D0 as a ragged host density (hfx_batch_layout offsets); the learned
 * guess runs per molecule (hfx_scf).  res[nmol]: per molecule (times are
 * the whole batch's).  D_out (optional): ragged host densities.  A
 * converged molecule keeps its density while the others iterate.  Returns
 * HFX_ERR_NOT_CONVERGED (with res filled) if any molecule did not converge. */
hfx_status hfx_batch_scf(hfx_ctx *ctx, const hfx_scf_options *opt, hfx_scf_result *res, double *D_out);

/* Change precision / digestion / task size of a loaded context (schwarz_tau
 * and device must stay as created). */
hfx_status hfx_configure(hfx_ctx *ctx, const hfx_options *opt);

/* Per-class scheduling knobs (class index 0..20, or -1 for all): quartets
 * per workgroup task (0: the context's task_quartets), XCD striping of long
 * ket prefixes (1 on, 0 off, -1 default on), the launch form (0: one
 * workgroup per task; 1: persistent, a resident grid that takes tasks from
 * eight per-XCD queues through atomic counters, the dynamic load balancing
 * of algorithms 1-3's ddi_dlbnext; 2: persistent with one task per wave,
 * each wave with its own LDS bra rows, for short tasks; falls back to 1 when
 * the workgroup's rows do not fit in LDS; 3: persistent and register-tiled:
 * a ket's primitives (1, 3 or 9 per pair) are read into registers once and
 * serve a block of two Q-adjacent bras (one when their LDS rows do not
 * fit), FP64 only -- a mixed build evaluates such a class in FP64; classes
 * or ket lists without register-tiled kernels fall back to 1; 4: as 3 with
 * one bra per task) and the digestion (-1: the context's
 * option; HFX_DIGEST_LDS, _GLOBAL, _PRIVATE or _LDS_D; LDS staging needs
 * (n_a + n_b) x nbf x 8 bytes <= 160 KiB and falls back to global
 * otherwise).  Re-plans a loaded system; results are unchanged up to the
 * order of floating-point sums.  Set by the autotuner
 * (paper_1708_00033_amd/autotune.py). */
hfx_status hfx_set_class_tuning(hfx_ctx *ctx, int cls, int task_quartets, int xcd_stripe, int persistent,
                                int digest);

/* Mixed builds (class index 0..20, or -1 for all): 1 (default) evaluates
 * the class's FP32-eligible quartets in FP32 (its mixed kernel), 0 keeps the
 * class in FP64 (never less accurate).  Chosen per class by the autotuner. */
hfx_status hfx_set_class_precision(hfx_ctx *ctx, int cls, int fp32);

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

/* Streams of a build's class launches (1..4, default 2): with n > 1 the
 * launches are dealt round-robin over the caller's stream and n - 1 side
 * streams that the context owns, forked from and joined back into the
 * caller's stream (also under HIP graph capture), so a launch starts on the
 * CUs that the previous one frees while its last tasks finish.  While kernel
 * timing is enabled every launch runs on the caller's stream, in order, so
 * that its events bracket only its own kernel.  Results are unchanged up to
 * the order of floating-point sums. */
hfx_status hfx_set_streams(hfx_ctx *ctx, int n);

/* Launches of a build: one per (quartet class, ket primitive count).
 * info[13] = {class index, ket primitives per pair, workgroup tasks, unique
 * quartets, primitive quartets, integrals, timed launches, digestion used
 * (HFX_DIGEST_*),
 * work-items per workgroup, launch form (0..4 as in hfx_set_class_tuning),
 * workgroups of the FP64 kernel, bras per task, staged D' rows: 0 none, 1
 * shell a's, 3 both shells'}; *ms = summed event time of
 * the timed launches. */
hfx_status hfx_plan_count(const hfx_ctx *ctx, int *n);
hfx_status hfx_plan_info(hfx_ctx *ctx, int i, long long *info, double *ms);

/* Superposition-of-atomic-densities guess of the loaded molecule (the SCF
 * default start): host nbf x nbf out. */
hfx_status hfx_sad_density(hfx_ctx *ctx, double *D);

/* ---- Learned initial guess --------------------------------------------------
 * An extension of the SCF start (the paper's SCF of section 3 starts from a
 * core-Hamiltonian path): a network predicts, for every atom pair within
 * 6 A (A = B included), the converged-minus-SAD density block in a local
 * frame of the pair; the blocks are rotated back and added to SAD.
 * Molecules of O and H only, with 15 basis functions per O and 2 per H.
 *
 * Pairs: A <= B in (element O before H, atom index) order, sorted by type
 * (0 O-O, 1 O-H, 2 H-H), then A, then B.  Frame of a pair: z from A to B (for
 * A = B toward A's nearest atom), x toward the nearest atom C (distance in
 * 1e-6 bohr bins, then index) whose direction from A is not within
 * sin 0.1 of z, y = z x x; without such a C, x from the global axis least
 * aligned with z.  Local block P = T_A(R^T)^T D_AB T_B(R^T) where T(R)
 * rotates the atom's Cartesian s, p and unit-normalised d functions; packed
 * FP32 blocks: every pair's na x nb row-major block in pair order (type 0
 * rows are 225 floats, type 1 30, type 2 4).
 * Features: 164 FP32 per pair = one-hot element of A (O, H), of B, 32 radial
 * Gaussians exp(-eta (R_AB - mu_k)^2) fc(R_AB) (mu_k = 0.5 .. 6 A in 31
 * steps, eta = 1 / (2 dmu^2), fc = (cos(pi R / 6 A) + 1) / 2), then the
 * environments of A and of B (for O then H neighbours: log(1 + the radial
 * functions summed over the atoms of that element other than the atom
 * itself)). */

/* Pair list, frames and features of the loaded single molecule (device,
 * owned by ctx until the next load).  counts[3] (optional): pairs per type. */
hfx_status hfx_guess_setup(hfx_ctx *ctx, int *counts);
/* Host copies (each optional): X npair x 164, pairs npair x 2 atom indices,
 * frames npair x 9 (rows x, y, z). */
hfx_status hfx_guess_features(hfx_ctx *ctx, float *X, int *pairs, double *frames);
/* Device pointer to the features (owned by ctx). */
hfx_status hfx_guess_features_dev(hfx_ctx *ctx, const float **dX);
/* dT = packed local blocks of dD - dDbase (dDbase may be NULL): training targets. */
hfx_status hfx_guess_targets_dev(hfx_ctx *ctx, const double *dD, const double *dDbase, float *dT, void *stream);
/* dD = dDbase + the packed blocks dT rotated back into the molecule (each
 * pair's block at (A, B) and its transpose at (B, A); a self block is
 * symmetrised first).  dDbase NULL: add to dD in place. */
hfx_status hfx_guess_assemble_dev(hfx_ctx *ctx, const float *dT, const double *dDbase, double *dD, void *stream);

/* Network: 164 -> 256 -> 256 -> 256 (SiLU) -> per pair type a linear head of
 * 225 / 30 / 4 outputs, BF16 MFMA with FP32 accumulation.  Parameters (FP32,
 * packed): W1[256x164] b1[256] W2[256x256] b2 W3[256x256] b3, heads
 * H0[225x256] c0 H1[30x256] c1 H2[4x256] c2 (W: out x in, row-major), then
 * the feature mean[164], feature scale[164] and target scales[3]: input
 * (x - mean) / scale clipped to [-4, 4], block = output x target scale of
 * the pair's type. */
hfx_status hfx_guess_create(int device, hfx_guess **out);
void hfx_guess_destroy(hfx_guess *g);
long long hfx_guess_param_count(void);
hfx_status hfx_guess_set_params(hfx_guess *g, const float *params);   /* host */
hfx_status hfx_guess_get_params(hfx_guess *g, float *params);         /* host */
/* Gradient of the last hfx_guess_grad_dev, packed like the parameters
 * (zeros for the mean, scale and target-scale entries). */
hfx_status hfx_guess_get_grads(hfx_guess *g, float *grads);
/* dX: rows grouped by type (counts[t] rows of type t, 164 FP32 each);
 * dT: packed blocks (forward: written; grad: the targets). */
hfx_status hfx_guess_forward_dev(hfx_guess *g, const float *dX, const int *counts, float *dT, void *stream);
/* Loss = mean over all block elements of (output - target / target scale)^2;
 * computes the gradient (synchronises the stream when loss != NULL). */
hfx_status hfx_guess_grad_dev(hfx_guess *g, const float *dX, const int *counts, const float *dT, void *stream,
                              double *loss);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected) on the weights
 * and biases with the last gradient. */
hfx_status hfx_guess_adam(hfx_guess *g, double lr, void *stream);
/* dD (device, in/out): a base density (SAD) on entry, base + prediction on
 * return; *used = 0 and dD unchanged when the prediction is not finite or
 * |tr(D S) - nocc| > 0.05 nocc.  Synchronises the stream. */
hfx_status hfx_guess_apply(hfx_ctx *ctx, hfx_guess *g, double *dD, void *stream, int *used);
const char *hfx_guess_last_error(const hfx_guess *g);

const char *hfx_last_error(const hfx_ctx *ctx);
void hfx_destroy(hfx_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* HFX_H */
