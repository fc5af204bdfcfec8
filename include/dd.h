/*
 * dd.h — C-ABI of the MI355X (gfx950) implementation of the fully algebraic
 * multilevel overlapping Schwarz preconditioner of Al Daas & Jolivet,
 * "A robust algebraic multilevel domain decomposition preconditioner for
 * sparse SPD matrices" (arXiv 2109.05908).
 *
 * Problem (Sec. 1): solve A x = b, A sparse symmetric positive definite.
 * Setup (Sec. 2-3): from A alone, build overlapping subdomains, local SPSD
 * splittings (3.1)-(3.2), the thresholded local eigenproblems (3.3), the
 * coarse space Z and coarse operator E = Z^T A Z, recursively for more
 * levels.  Apply: the two-level additive Schwarz preconditioner (2.1) inside
 * PCG, or the deflated variant with the restricted one-level method used in
 * the experiments (Sec. 4) inside right-preconditioned GMRES.
 *
 * Conventions for every entry point
 *  - Pointers documented "device" must point to GPU memory of the current
 *    HIP device; "host" pointers to CPU memory.  Dense matrices are
 *    column-major; multi-RHS vectors are column-major n x nrhs.
 *  - Work is ordered on the given stream.  Calls on one handle are not
 *    thread-safe.  The caller owns every buffer it passes; dd_setup copies
 *    what it keeps, so A and part may be freed once it returns.
 *  - Return value: 0 = DD_OK, < 0 = error (nothing was produced), > 0 =
 *    warning (a result was produced, see the code).  No exception crosses
 *    the ABI.
 */
#ifndef DD_H
#define DD_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ----------------------------------------------------- */
#define DD_OK                   0
#define DD_ERR_INVALID_ARG     -1  /* bad n, N, overlap, tau <= 0, levels < 2, partition id out of range, empty part */
#define DD_ERR_NOT_SPD         -2  /* Cholesky breakdown of a local block A_ii or of E in FP64 */
#define DD_ERR_EIG             -3  /* local eigensolver failed to converge */
#define DD_ERR_NAN             -4  /* NaN/Inf in an input or produced by the solve */
#define DD_ERR_OOM             -5  /* device allocation failed */
#define DD_ERR_HIP             -6  /* other HIP runtime error */
#define DD_ERR_INTERNAL        -7
#define DD_WARN_MAXIT           1  /* PCG or GMRES stopped at maxit before reaching rtol */
#define DD_WARN_FULL_COARSE     2  /* tau >= 1 with Boolean D: every mode is kept (lambda >= 1 always) */
#define DD_WARN_FP32_FALLBACK   3  /* an FP32 local factor failed; that subdomain uses FP64 */

/* ---- inputs ------------------------------------------------------------ */
/* Sparse matrix A in CSR, full symmetric storage (both triangles), column
 * indices sorted and unique within each row.  All arrays are device memory
 * owned by the caller: rowptr[n+1], colind[nnz], val[nnz].  The stored
 * pattern defines the graph G(A) of Sec. 2. */
typedef struct {
    int64_t n;
    int64_t nnz;
    const int32_t* rowptr;
    const int32_t* colind;
    const double*  val;
} dd_csr;

#define DD_FP64 0
#define DD_FP32 1
#define DD_SEL_THRESHOLD      0  /* keep lambda > 1/tau  (3.3) */
#define DD_SEL_THRESHOLD_CAP  1  /* keep lambda > 1/tau, at most nev_cap per subdomain (the largest lambda) */
#define DD_SCHWARZ_ADDITIVE   0  /* M = R_0^T E^{-1} R_0 + sum_i R_i^T A_ii^{-1} R_i  (2.1), symmetric: dd_pcg */
#define DD_SCHWARZ_DEFLATED   1  /* M = R_0^T E^{-1} R_0 + M_RAS (I - A R_0^T E^{-1} R_0), the variant of the
                                    experiments (Sec. 4), M_RAS = sum_i R_i^T D_i A_ii^{-1} R_i with the Boolean
                                    D_i (1 on Omega_Ii, 0 on Gamma_i); not symmetric: dd_gmres */

typedef struct {
    int32_t local_prec;   /* DD_FP64 (default) or DD_FP32: precision of the exact local solver A_ii^{-1} of
                             (2.1).  DD_FP32: D A_ii D (symmetric Jacobi scaling, d_k = a_kk^{-1/2}) is
                             factored in FP32 on FP32 MFMA with FP32 accumulation, its inverse formed in
                             FP32, and the local solves of the apply run in FP32 on FP64 vectors; a
                             subdomain whose FP32 factor fails keeps FP64 (dd_info_t.fp32_fallbacks).
                             The splitting, the eigenproblem (which also uses an FP64 factor of the
                             leading block of A_ii), E and PCG stay FP64. */
    int32_t select;       /* DD_SEL_THRESHOLD (default) or DD_SEL_THRESHOLD_CAP */
    int32_t nev_cap;      /* cap per subdomain for DD_SEL_THRESHOLD_CAP */
    int32_t validate;     /* nonzero: check the CSR structure of A first (O(nnz)): rowptr[0] = 0,
                             rowptr[n] = nnz, column indices in range, strictly increasing within each
                             row, pattern symmetric; DD_ERR_INVALID_ARG if not.  Without it a malformed
                             CSR is undefined behaviour.  Values are always checked for NaN/Inf. */
    int32_t coarsen;      /* levels >= 3: subdomains per coarse part (default 64) */
    int32_t schwarz;      /* DD_SCHWARZ_ADDITIVE (default) or DD_SCHWARZ_DEFLATED */
    int32_t eig_solver;   /* local eigenproblem (3.3): DD_EIG_DENSE (default; tridiagonal route, every mode),
                             DD_EIG_LOBPCG (block solver for the nev_cap modes of DD_SEL_THRESHOLD_CAP: the
                             largest eigenvalues of K = S~^{-1} = M^T M, M = R_II^{-T} L_I formed once) or
                             DD_EIG_LOBPCG_MATFREE (the smallest of S~ = L_I^{-1} S_I L_I^{-T} applied through the
                             triangular factors L_I and R_II, S_I = R_II^T R_II, preconditioned by K applied the
                             same way: no n_Ii x n_Ii matrix formed for the eigenproblem) */
    int32_t lobpcg_maxit; /* LOBPCG iterations per subdomain (0: 100); eig_maxit_hits counts the misses */
    double  lobpcg_tol;   /* LOBPCG stop for the nev_cap wanted pairs: DD_EIG_LOBPCG, residual relative to the
                             eigenvalue of K = S~^{-1} (above its rounding floor; 0: 1e-8); DD_EIG_LOBPCG_MATFREE,
                             absolute residual of S~, whose norm is <= 1 (0: 1e-12) */
    int32_t warm_start;   /* LOBPCG start block: DD_START_RANDOM (default), DD_START_RANGE or DD_START_MODEL */
    int32_t graph_pcg;    /* 1..64: dd_pcg on a two-level additive handle runs each iteration as one captured
                             HIP graph (alpha, beta and the stopping test on the device), replayed in batches of
                             at most graph_pcg between host checks, each batch sized from the residual
                             contraction so that few iterations run past the stop; the iterates are those of
                             the host-driven loop, bit for bit.  A batch handle (dd_setup_batch) keeps one set
                             of scalars and one stopping test per system.  0 (default): host-driven.  Handles
                             with more levels ignore it. */
    uint64_t seed;        /* seed of the Gaussian draws of the start blocks */
    const void* warm_start_model; /* DD_START_MODEL: a dd_model (dd_model_create); NULL falls back to random */
    int32_t reserved[8];
} dd_options;
#define DD_EIG_DENSE          0
#define DD_EIG_LOBPCG         1
#define DD_EIG_LOBPCG_MATFREE 2
#define DD_START_RANDOM       0  /* Gaussian block (counter-based generator, seed) */
#define DD_START_RANGE        1  /* A_ii^{-1} A(Omega_i, Delta_i) G restricted to Omega_Ii, G Gaussian on Delta_i */
#define DD_START_MODEL        2  /* the same with the rows of G weighted by the network of warm_start_model */

typedef struct dd_handle_s* dd_handle;

/* ---- diagnostics ------------------------------------------------------- */
#define DD_MAX_LEVELS 4
#define DD_NPHASE 12
#define DD_PHIST 16
/* Setup and solve statistics of a handle (Sec. 3.2: the constants of the condition-number bound;
 * Sec. 4: coarse sizes and grid complexity as the experiments report them). */
typedef struct {
    int32_t levels;                 /* levels built (2 = fine + coarse) */
    int32_t N[DD_MAX_LEVELS];       /* subdomains per decomposed level */
    int64_t n[DD_MAX_LEVELS];       /* matrix size per level (n[1] = n_C of level 0) */
    int64_t n_C;                    /* coarse size of the finest level */
    double  grid_complexity;        /* (sum of the level sizes) / n, (n + n_C) / n with two levels (Sec. 4) */
    int32_t p_min, p_max;           /* kept modes per fine subdomain */
    int32_t p_hist[DD_PHIST];       /* fine subdomains by kept modes p_i: bin 0 holds p_i = 0, bin b >= 1
                                       holds 2^(b-1) <= p_i < 2^b, the last bin everything above */
    int32_t k_c;                    /* colours of a greedy colouring (subdomains in index order, smallest free
                                       colour) of the fine subdomain graph, i ~ j iff A(Omega_i, Omega_j) != 0
                                       (overlapping sets): the k_c of the bound (k_c + 1)(2 + (2 k_c + 1) k_m / tau)
                                       of Sec. 3.2; computed on the host at the first dd_info call */
    int32_t fp32_fallbacks;         /* FP32 form: subdomains (all levels) whose FP32 factor of D A_ii D met a
                                       pivot <= n_max eps_32 or gave a non-finite inverse, and that keep
                                       the FP64 inverse instead */
    int32_t eig_maxit_hits;         /* local eigen/polar iterations that hit their cap (block solver: subdomains) */
    int32_t eig_iters_max;          /* block eigensolver on the finest level: largest and mean iteration count */
    double  eig_iters_mean;
    double  eig_resid_max;          /* its largest final relative eigen-residual of a wanted pair */
    double  phase_ms[DD_NPHASE];    /* setup phase times, see dd_phase_name */
    int32_t last_iters;             /* last dd_pcg or dd_gmres: iterations (first RHS; a batch: the largest) */
    double  last_relres;            /* last dd_pcg or dd_gmres: true relative residual (first RHS; a batch: the largest) */
    int64_t device_bytes;           /* device memory of the handle's factors, bases and index maps */
    int64_t coarse_factor_bytes;    /* the last level's Cholesky factor of E: supernode panels and the inverses
                                       of their diagonal blocks; every coarse solve reads it twice (forward and
                                       backward), so 2 x this is the HBM traffic of one coarse solve */
} dd_info_t;

/* ---- entry points ------------------------------------------------------ */

/* Seeded greedy graph growing partition of G(A) into N parts (a graph
 * partitioning algorithm, Sec. 2): N distinct seed vertices from a
 * SplitMix64 stream started at `seed` (vertex = output mod n, repeats
 * skipped; the k-th distinct seed owns part k), then level-synchronous BFS
 * where every unassigned vertex adjacent to the previous round's frontier
 * takes the minimum part id among those neighbours; unreached vertices go
 * to the smallest part (lowest id on ties).  part: device int32[n], output.
 * Deterministic and bit-exact.  Errors: DD_ERR_INVALID_ARG if N < 1 or N > n. */
int dd_partition_ggg(const dd_csr* A, int32_t N, uint64_t seed, int32_t* part, hipStream_t stream);

/* dd_partition_ggg for callers that cannot allocate (serving loops, harnesses that forbid
 * hipMalloc/hipHostMalloc): the same partition, bit for bit, with no allocation of any kind.
 * Its work arrays (4,194,304 + 65,536 + 64 int32, about 16.3 MiB) live in one file-scope device
 * array per GPU, held by the library until the process ends.  Limits: n <= 4,194,304 and
 * N <= 65,536, else DD_ERR_INVALID_ARG (nothing runs).  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams or threads) race, so the caller orders them.
 * The array is reinitialised by every call.  A, part: device, as for dd_partition_ggg; part is
 * the output.  The call synchronises the stream once per growing round (it reads a device flag
 * into host stack memory).  Errors: DD_ERR_INVALID_ARG, DD_ERR_HIP. */
int dd_partition_ggg_noalloc(const dd_csr* A, int32_t N, uint64_t seed, int32_t* part, hipStream_t stream);

/* Build the preconditioner (Sec. 2-3).
 *  part    device int32[n], subdomain id of each node in [0, N)  (Omega_Ii = {j : part_j = i})
 *  overlap delta >= 1: Gamma_i = BFS layers 1..delta of Omega_Ii, Delta_i = layer delta+1
 *  tau     the paper's tau > 0 of (3.3): keep eigenpairs with lambda > 1/tau
 *  levels  2..4; 2 = exact (block-sparse) Cholesky of E; >= 3: the construction is repeated on E
 *          (multilevel remark of Sec. 3.2): the subdomain graph of E (i ~ j iff A(Omega_Ii,
 *          Omega_Ij) != 0) is partitioned by dd_partition_ggg's rule into ceil(N/coarsen) parts
 *          (seed 0, empty parts dropped), with the same overlap and tau; E^{-1} in (2.1) becomes
 *          PCG on E to a relative residual of 1e-4, preconditioned by the next level, and only
 *          the last level's E is factored.  If a level keeps no coarse mode, recursion stops.
 *  opt     may be NULL (defaults: FP64, threshold selection, no validation)
 *  out     receives the handle (owned by the caller; free with dd_destroy)
 * Errors: DD_ERR_INVALID_ARG, DD_ERR_NOT_SPD, DD_ERR_EIG, DD_ERR_OOM, DD_ERR_HIP.
 * Warnings: DD_WARN_FULL_COARSE, DD_WARN_FP32_FALLBACK. */
int dd_setup(const dd_csr* A, const int32_t* part, int32_t N, int32_t overlap, double tau,
             int32_t levels, const dd_options* opt, hipStream_t stream, dd_handle* out);

/* New values for the matrix the handle was built on, same pattern and same partition (a family
 * of matrices that differ only in coefficients, as in a parametric study): the whole setup
 * (Secs. 2-3, every level) is redone for the new values with the handle's overlap, tau,
 * levels and options, and replaces the old preconditioner only on success.
 *  val   device, nnz values in the handle's CSR order (full symmetric storage)
 * The caller keeps ownership of val (it is copied).  On any error the handle keeps its
 * previous values and preconditioner.  Errors and warnings as for dd_setup
 * (DD_ERR_NAN for non-finite values). */
int dd_update_values(dd_handle h, const double* val, hipStream_t stream);

/* Several independent systems in one handle (Sec. 2: the subdomains of a decomposition are set up
 * independently of each other, one per process in the paper; here the subdomains of several
 * systems share the batched launches of one GPU): As[j] (device CSR, n_j unknowns) with partition
 * parts[j] (device, n_j entries in [0, Ns[j])), all with the same overlap, tau, levels and
 * options.  The handle holds the block-diagonal union of the systems (unknowns and parts
 * numbered system after system), so every setup phase runs all subdomains of all systems in
 * the same batched launches; with two levels the result for each system is that of its own
 * dd_setup (its subdomains and coarse blocks never touch another system).
 *  nsys    number of systems (>= 1); As, parts, Ns: host arrays of nsys entries
 * Vectors passed to dd_apply and dd_pcg are the systems' vectors concatenated (sum n_j per RHS).
 * dd_pcg on such a handle runs one PCG per system in lockstep (per-system dot products, alpha
 * and beta; each system stops on its own residual) and writes nsys entries of iters and relres
 * per RHS (system j of RHS k at k*nsys + j).  With more than two levels every level is
 * partitioned system by system and the inner coarse solves run one PCG per system, so each
 * system gets the hierarchy and the solve of its own dd_setup.  With opt->validate each system's
 * CSR structure is checked on its own, before the union is formed.  The deflated variant
 * (schwarz = DD_SCHWARZ_DEFLATED) is refused: it needs GMRES, which has no per-system form.
 * dd_update_values on a batch handle takes the nnz values of the union (system after system).
 * The caller keeps ownership of all inputs (copied).
 * Errors and warnings as for dd_setup; DD_ERR_INVALID_ARG also for n or nnz of the union
 * beyond int32 and for the deflated variant. */
int dd_setup_batch(const dd_csr* As, const int32_t* const* parts, const int32_t* Ns, int32_t nsys,
                   int32_t overlap, double tau, int32_t levels, const dd_options* opt,
                   hipStream_t stream, dd_handle* out);

/* z = M^{-1} r with M^{-1} = R_0^T E^{-1} R_0 + sum_i R_i^T A_ii^{-1} R_i  (2.1); with more than
 * two levels E^{-1} is the inner PCG described at dd_setup (M then varies slightly with r).
 * A handle set up with schwarz = DD_SCHWARZ_DEFLATED applies instead the deflated variant of
 * Sec. 4, z = y + M_RAS (r - A y) with y = R_0^T E^{-1} R_0 r, whose coarse solves on levels
 * that are not the last are right-preconditioned GMRES(30) to 1e-4 with the next level's
 * deflated M.  r, z: device, column-major n x nrhs, must not alias.  Errors: DD_ERR_INVALID_ARG. */
int dd_apply(dd_handle h, const double* r, double* z, int32_t nrhs, hipStream_t stream);

/* Solve A x = b (Sec. 1) by preconditioned CG, the solver the condition-number bound of Sec. 3.2
 * speaks to, stopped at a relative residual as in Sec. 4 (1e-8 there).
 * M from dd_apply (FP64 dots and residual recurrence); with more than
 * two levels, flexible CG (Polak-Ribiere beta) since M varies between iterations.
 * b: device n x nrhs; x: device n x nrhs, in: initial guess, out: solution.
 * Stops RHS j when ||b_j - A x_j||_2 <= rtol ||b_j||_2 (recurrence residual,
 * true residual recomputed at exit).  iters, relres: host arrays [nrhs]
 * (may be NULL).  Returns DD_WARN_MAXIT if some RHS did not converge. */
int dd_pcg(dd_handle h, const double* b, double* x, int32_t nrhs, double rtol, int32_t maxit,
           int32_t* iters, double* relres, hipStream_t stream);
/* (dd_pcg returns DD_ERR_INVALID_ARG on a handle with the deflated variant, which is not
 * symmetric.) */

/* Right-preconditioned GMRES(restart) (Saad & Schultz) with M from dd_apply: the outer solver of
 * the paper's experiments (Sec. 4).  It runs in the flexible form (Saad), keeping z_j = M v_j and
 * updating x with them: for a fixed M that is the same iterate with one apply fewer per cycle,
 * and it also serves M that varies between iterations (more than two levels) or is linear only
 * up to FP32 rounding (FP32 local solves).  Works with either variant of the handle.
 * Arnoldi by classical Gram-Schmidt applied twice; a restart cycle ends when the Arnoldi
 * estimate of ||b_j - A x_j||_2 (the unpreconditioned residual) reaches rtol ||b_j||_2, after
 * `restart` steps or at maxit steps in total; the true residual is recomputed at the end of
 * every cycle and reported.
 * b: device n x nrhs; x: device n x nrhs, in: initial guess, out: solution.
 * restart: 1..64.  iters (Arnoldi steps over all cycles), relres (true relative residual):
 * host arrays [nrhs] (may be NULL).  Returns DD_WARN_MAXIT if some RHS did not converge;
 * DD_ERR_INVALID_ARG for bad arguments or a batch handle (dd_setup_batch: use dd_pcg);
 * DD_ERR_NAN on NaN or a breakdown with a singular Hessenberg matrix. */
int dd_gmres(dd_handle h, const double* b, double* x, int32_t nrhs, double rtol, int32_t maxit,
             int32_t restart, int32_t* iters, double* relres, hipStream_t stream);

/* y = A x (the operator of Sec. 1) for the fine-level matrix held by the handle (SpMV kernel).
 * x, y: device double[n] (n of the handle; a batch: the union), must not alias.
 * Errors: DD_ERR_INVALID_ARG for a null handle or pointer. */
int dd_spmv(dd_handle h, const double* x, double* y, hipStream_t stream);

/* Copies the handle's statistics (dd_info_t above: level sizes and grid complexity as reported in
 * Sec. 4, kept modes, the colouring constant k_c of the bound of Sec. 3.2, phase times, the last
 * solve) into *out (host).  Synchronous; the first call computes k_c on the host from the
 * handle's index sets.  Errors: DD_ERR_INVALID_ARG for a null handle or out. */
int  dd_info(dd_handle h, dd_info_t* out);
/* Name of setup phase `phase` (0 <= phase < DD_NPHASE) of dd_info_t.phase_ms; "?" otherwise. */
const char* dd_phase_name(int32_t phase);
/* Frees the handle (the caller owns it from dd_setup / dd_setup_batch on; NULL is ignored).
 * Work queued on the handle must be complete or ordered before later use of the memory, which the
 * cache below guarantees by synchronising before reuse.  Its device memory goes back to the library's device cache, which hands
 * it to later setups of the same process instead of hipMalloc/hipFree (large hipMalloc calls
 * were seen to stall for seconds after a few setup cycles); a cached block is reused only
 * after a device synchronisation that follows its release.  The cache holds at most
 * DD_DEVICE_CACHE_GB GiB per process (environment, read once; default 96, 0 disables it). */
void dd_destroy(dd_handle h);
/* Returns every cached device block to hipFree (after a device synchronisation), for callers
 * that need the memory elsewhere.  Thread-safe.  Returns DD_OK. */
int dd_trim_device_cache(void);
const char* dd_strerror(int code);

/* ---- warm start of the block eigensolver (a learned model) ---------------
 * A small network maps features of every node of the boundary layer Delta_i of a subdomain
 * (computed from A alone) to a positive weight; the start block of the eigenproblem (3.3) is then
 * X_i = [A_ii^{-1} A(Omega_i, Delta_i) diag(w) G]_{Omega_Ii} (in the reciprocal form's variables),
 * G Gaussian, which lies in the near kernel of the splitting (Sec. 3.2 shows the kernel of
 * the splitting is made of such vectors).  The network is trained, on the GPU, on the kept
 * eigenvectors of earlier setups of the same family of matrices: for each boundary node the
 * target is the square root of its leverage (times |Delta_i| / p_i) in an orthonormal basis of
 * A(Delta_i, Omega_i) A_ii^{-1} [Z_i; 0], the boundary data of the kept eigenvectors.  Loss: the
 * mean over subdomains of each one's mean square error of the weights; optimiser Adam.
 * Architecture: 8 features (standardised by the training mean and deviation), two tanh layers of
 * 32, softplus output; parameters W1 (32 x 8 row-major), b1, W2 (32 x 32), b2, w3 (32), b3, then the
 * 8 feature means and 8 deviations: DD_MODEL_NPARAM doubles in all. */
typedef struct dd_model_s* dd_model;
#define DD_MODEL_NFEAT  8
#define DD_MODEL_NPARAM (8 * 32 + 32 + 32 * 32 + 32 + 32 + 1 + 2 * 8)
/* A new model with Glorot-scaled Gaussian weights from `seed`, zero hidden biases and the output
 * bias at softplus^{-1}(1), so that it starts near weight 1 everywhere (the range start).
 * Errors: DD_ERR_INVALID_ARG for a null out, DD_ERR_OOM. */
int dd_model_create(uint64_t seed, dd_model* out);
/* Appends training samples from handle h (finest level; FP64 local solves): the features and
 * targets of the boundary nodes of every subdomain that kept modes.  The handle's kept vectors
 * are the training eigenvectors (set up with the dense route for exact ones).  Synchronous.
 * Errors: DD_ERR_INVALID_ARG (null arguments, FP32 handle, a subdomain with more than 128 kept
 * modes). */
int dd_model_add_samples(dd_model m, dd_handle h, hipStream_t stream);
/* `epochs` full-batch Adam steps (learning rate lr) on the stored samples; the feature means and
 * deviations are fixed at the first call.  loss: host double[epochs] (may be NULL), the loss
 * before each step.  Errors: DD_ERR_INVALID_ARG (no samples, epochs < 0, lr <= 0). */
int dd_model_train(dd_model m, int32_t epochs, double lr, double* loss, hipStream_t stream);
/* Parameters out (host double[DD_MODEL_NPARAM], may be NULL) and their count. */
int dd_model_params(dd_model m, double* out, int32_t* count);
/* Parameters in (host, count = DD_MODEL_NPARAM; deviations > 0).  Errors: DD_ERR_INVALID_ARG, DD_ERR_NAN. */
int dd_model_set_params(dd_model m, const double* in, int32_t count);
/* out[s] = weight of sample s: feats device double[n x DD_MODEL_NFEAT] (row-major), out device double[n]. */
int dd_model_forward(dd_model m, const double* feats, int64_t n, double* out, hipStream_t stream);
/* Loss sum_s weight_s (w_s - target_s)^2 and its gradient with respect to the DD_MODEL_NPARAM - 16
 * trained parameters on n given samples (device arrays), into host loss[1] and grad (either may be
 * NULL).  Errors: DD_ERR_INVALID_ARG. */
int dd_model_loss_grad(dd_model m, const double* feats, const double* target, const double* weight, int64_t n,
                       double* loss, double* grad, hipStream_t stream);
/* The stored samples (host arrays, each may be NULL): n, feats[n x 8], target[n], weight[n]. */
int dd_model_samples(dd_model m, int64_t* n, double* feats, double* target, double* weight);
void dd_model_destroy(dd_model m);

/* ---- inspection (tests and diagnostics; all outputs are host memory) ---- */
/* Block eigensolver of `level`: iterations and final largest relative eigen-residual of the wanted
 * pairs of every subdomain (host int32[N], double[N], may be NULL).  DD_ERR_INVALID_ARG for a level
 * set up with the dense route. */
int dd_subdomain_eig_stats(dd_handle h, int32_t level, int32_t* iters, double* resid);
/* Number of subdomains at `level` (0 = finest). */
int dd_subdomain_count(dd_handle h, int32_t level, int32_t* N);
/* sizes: host int32[5*N]: for each i, {n_Ii, n_Gamma_i, n_Delta_i, p_i, status}. */
int dd_subdomain_sizes(dd_handle h, int32_t level, int32_t* sizes);
/* Ordered index sets of subdomain i (global indices, each ascending):
 * I[n_Ii], Gamma[n_Gamma_i], Delta[n_Delta_i]. */
int dd_subdomain_sets(dd_handle h, int32_t level, int32_t i, int32_t* I, int32_t* Gamma, int32_t* Delta);
/* Kept eigenvalues mu = 1/lambda of subdomain i, ascending: mu[p_i]. */
int dd_subdomain_eigs(dd_handle h, int32_t level, int32_t i, double* mu);
/* Orthonormal basis of D_i Z_i restricted to Omega_Ii: Z[n_Ii x p_i], column-major. */
int dd_subdomain_basis(dd_handle h, int32_t level, int32_t i, double* Z);
/* Steps a1-a2 alone, for inspection: the ordered sets of Sec. 2 and the dense blocks of
 * Sec. 3.1 of subdomain i of the decomposition (A, part, N, overlap) as dd_setup forms them, without
 * building a preconditioner.  A, part: device, as for dd_setup.  Outputs (host, each may be NULL):
 * sizes int32[3] = {n_Ii, n_Gamma_i, n_Delta_i}; Aii double[n_i x n_i] = A(Omega_i, Omega_i);
 * X double[n_i x n~_i] = X_i = A(Omega_i, Omega~_i) (3.1), both column-major, rows and columns in
 * the order [Omega_Ii, Gamma_i] and [Omega_Ii, Gamma_i, Delta_i].  Synchronous.
 * Errors: DD_ERR_INVALID_ARG (as dd_setup, or i outside [0, N)), DD_ERR_OOM. */
int dd_extract_local(const dd_csr* A, const int32_t* part, int32_t N, int32_t overlap, int32_t i, int32_t* sizes,
                     double* Aii, double* X, hipStream_t stream);
/* Largest singular value sigma_1 of X_i for every subdomain: sigma1[N]. */
int dd_subdomain_sigma1(dd_handle h, int32_t level, double* sigma1);
/* Coarse operator E of `level` (n_C x n_C dense, column-major), only if n_C <= max_n. */
int dd_coarse_matrix(dd_handle h, int32_t level, double* E, int64_t max_n);

/* ---- kernel meter (measurement) ------------------------------------------
 * Device-side timing of one kernel family without a profiler.  After
 * dd_meter_start(name), every dispatch of the kernels launched under `name`
 * (e.g. "qr_blk_upd": the trailing update C -= V_b W of the blocked
 * Householder QR; "gemm_nn"/"gemm_nt"/"gemm_tn"/"gemm_tt": batched GEMM) is
 * bracketed by HIP events recorded on the stream it is launched on, and its
 * algorithmic flops and bytes (from the item shapes) are accumulated.
 * dd_meter_read waits for the last recorded event and returns the totals
 * since the last dd_meter_start; dd_meter_start(NULL) disarms.  Process-wide
 * state, not thread-safe; arming adds two event records per dispatch. */
typedef struct {
    int64_t launches;   /* dispatches recorded */
    double  total_ms;   /* sum of per-dispatch durations (event pairs) */
    double  flops;      /* algorithmic floating-point operations */
    double  bytes;      /* algorithmic HBM bytes (each operand read once, outputs written once) */
} dd_meter_t;
int dd_meter_start(const char* kernel);
int dd_meter_read(dd_meter_t* out);

/* ---- launch-mapping autotuner ----------------------------------------------
 * Every batched tile launch (all subdomains of a level in one launch) picks how
 * its tiles map onto workgroups: static round-robin, XCD-chunked, or a
 * persistent work queue (a device counter; items ordered by decreasing tile
 * count, longest first), each at a grid cap.  The library tries the candidates
 * on the launches of every kernel family as they come, times them with events,
 * and keeps the fastest per tile after three samples each.  The mapping never
 * changes a result (every tile is computed once, by one workgroup, with the same
 * arithmetic).  DD_AUTOTUNE=0 in the environment (read once) switches it off.
 * Writes a text table of the candidates (mean microseconds per tile, samples;
 * the chosen one starred) into buf (may be NULL) and returns its length. */
int dd_autotune_report(char* buf, int64_t len);

#ifdef __cplusplus
}
#endif
#endif /* DD_H */
