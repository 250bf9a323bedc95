/*
 * efgp.h — C ABI of the MI355X (gfx950) library for equispaced-Fourier
 * Gaussian process regression (EFGP; Greengard, Rachh, Barnett, arXiv
 * 2210.10210).
 *
 * The library computes the posterior mean of GP regression with a
 * translation-invariant kernel (squared exponential or Matern) from N noisy
 * observations y_n at points x_n in [0,1]^d, d in {1,2,3}, by solving the
 * weight-space system (D F*F D + sigma^2 I) beta = D F* y on the
 * equispaced Fourier basis (Sec. 3, eqs. (basis), (97), (rhs)) and
 * evaluating mu(x) = sum_j D_j beta_j exp(-2 pi i h <j, x>) (eq. (muws)).
 *
 * Three stages, each a call below:
 *   efgp_setup  — steps 1-3 of the EFGP algorithm: choose (h, m); spread the
 *                 points (type-1 NUFFT, one pass, 1+nrhs channels) to build
 *                 the Toeplitz vector v of F*F (eq. (88)) and the right-hand
 *                 sides b = D F* y (eq. (rhs)); precompute FFT(v).
 *   efgp_solve  — step 4: conjugate gradients (optionally with a diagonal
 *                 preconditioner) with the FFT Toeplitz product (Sec. 3.2,
 *                 fast Toeplitz algorithm), batched over the nrhs systems.
 *   efgp_eval   — step 6: type-2 NUFFT of D.beta at q targets
 *                 (efgp_mean_at_points: step 7, the same at the N points).
 *
 * Conventions
 *   - Frequency vectors over J_m = {-m..m}^d are stored in C order with
 *     offset j^(l)+m per dimension, last dimension fastest, length
 *     M = (2m+1)^d; complex values interleave (re, im).  Batched vectors of
 *     nrhs systems are stored [rhs][M].
 *   - Points and targets are structure-of-arrays on the device: coordinate
 *     l of point i at x[l*n + i].  Data: y[r*n + i].
 *   - Sign convention: the type-1 sums use exp(+2 pi i h <j,x>) so that
 *     (F*F)_{pl} = v_{j_p - j_l}; the mean uses exp(-2 pi i h <j,x>).
 *   - precision 32: float inputs/outputs (float2 for complex); spreading,
 *     FFTs and the matrix product run in float while the global
 *     accumulation of the spread grid, v, CG inner products and step
 *     scalars stay double.  precision 64: double throughout.
 *   - All device pointers must be device memory of the current HIP device.
 *     Work is ordered after prior work on `stream` and the call returns
 *     after its work is complete or enqueued as documented per call.
 *   - Status codes: 0 success, >0 warning, <0 error.  No call aborts or
 *     throws across the ABI.  On an argument error outputs are untouched.
 */
#ifndef EFGP_H
#define EFGP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum efgp_status {
    EFGP_OK = 0,
    EFGP_NOT_CONVERGED = 1,   /* warning: beta_out holds the last iterate      */
    EFGP_FELL_BACK = 2,       /* warning: preconditioned CG stalled; plain CG
                                 finished the solve (answer meets rel_tol)      */
    EFGP_EINVAL = -1,         /* invalid argument                              */
    EFGP_EDOMAIN = -2,        /* a point or target outside [0,1]^d (the paper
                                 requires the caller to translate and scale,
                                 Sec. 2)                                        */
    EFGP_ETOOLARGE = -3,      /* sizes beyond the library limits (checked
                                 before any allocation)                        */
    EFGP_ENOMEM = -4,         /* device allocation failed                      */
    EFGP_EHIP = -5,           /* a HIP runtime call failed                     */
    EFGP_EMODEL = -6          /* preconditioner network weights unusable       */
};

enum efgp_kernel { EFGP_KERNEL_SE = 0, EFGP_KERNEL_MATERN = 1 };
/* Preconditioners of the CG solve (step 4).  JACOBI: 1/(N D_j^2 + sigma^2),
 * the inverse diagonal (T_jj = v_0 = N).  LEARNED: the network's correction
 * of Jacobi.  DIAG: a caller-given positive diagonal.  CIRCULANT: T. Chan's
 * optimal circulant of the Jacobi-scaled system (see efgp_circulant_eigs),
 * an operator preconditioner costing two K^d FFTs per iteration. */
enum efgp_precond { EFGP_PRECOND_NONE = 0, EFGP_PRECOND_JACOBI = 1, EFGP_PRECOND_LEARNED = 2,
                    EFGP_PRECOND_DIAG = 3, EFGP_PRECOND_CIRCULANT = 4 };
/* Spreaders (step 1, eq. (88) and eq. (rhs) by a type-1 NUFFT).  TILES sorts
 * the points by spread tile and accumulates each tile in LDS; GRID_LDS keeps
 * the whole active grid region in each workgroup's LDS (one data vector
 * only).  With 16 or more data vectors in precision 32 and d <= 2, TILES
 * takes two data vectors per lane and sizes its own tile to its LDS
 * accumulator (the problem's tile field is then not used).  REGIONS
 * (precision 32, one data vector) partitions the points into regions whose
 * grid windows fit in LDS and accumulates each region as GRID_LDS does; the
 * tile field is then the region edge in stencil origins (0 => the largest
 * that fits; a larger request is EFGP_ETOOLARGE).  AUTO takes GRID_LDS when
 * the region fits and there are many points per cell, else REGIONS when it
 * can, else TILES. */
enum efgp_spread { EFGP_SPREAD_AUTO = 0, EFGP_SPREAD_TILES = 1, EFGP_SPREAD_GRID_LDS = 2,
                   EFGP_SPREAD_REGIONS = 3 };

typedef struct efgp_plan efgp_plan;

/* Problem statement (Sec. 1 and 5: points, data, noise variance, kernel,
 * tolerance).  Fields marked "0 => default" may be left zero. */
typedef struct efgp_problem {
    int32_t dim;            /* d in {1,2,3}                                    */
    int32_t kernel;         /* efgp_kernel: SE (eq. (Gker)) or Matern (eq. (Cker)) */
    double lengthscale;     /* ell > 0                                         */
    double nu;              /* Matern smoothness, >= 1/2 (ignored for SE)      */
    double variance;        /* prior variance k(0); 0 => 1                     */
    double eps;             /* EFGP tolerance in (0,1): sets h, m (Sec. 4.2)   */
    int32_t precision;      /* 32 or 64                                        */
    double nufft_tol;       /* spreading tolerance; 0 => eps/10 (Sec. 5.1) for
                               precision 32 and min(eps/10, 1e-12) (parity
                               mode) for precision 64; an explicit value is
                               used as given (precision 32: at least 1e-7)     */
    int64_t n;              /* number of points N >= 1                         */
    const void* x;          /* device, d*n float/double, SoA, in [0,1]^d       */
    int32_t nrhs;           /* number of data vectors, 1..64                   */
    const void* y;          /* device, nrhs*n float/double                     */
    const double* sigma2;   /* host, nrhs noise variances > 0                  */
    void* stream;           /* hipStream_t the call is ordered on (0 = null)   */
    int32_t m_override;     /* >0: use this m instead of the rule (h from rule) */
    int32_t spread_method;  /* efgp_spread; AUTO picks by size                 */
    int32_t tile;           /* spread tile edge in grid cells (REGIONS: region
                               edge in stencil origins); 0 => automatic       */
    int32_t spread_epoch;   /* precision 32: most points one workgroup adds to
                               its fixed-point accumulator before flushing it
                               (smaller epochs allow finer scales at the cost
                               of more flushes); 0 => 2^20 for GRID_LDS and
                               2^18 for TILES (2048 in 3D), else a power of two
                               in [2^10, 2^24]                                 */
} efgp_problem;

/* Plan description (read with efgp_get_info).  Tests use it to share h and m
 * with an independent implementation. */
typedef struct efgp_info {
    int32_t dim, precision, nrhs, kernel;
    int32_t m;              /* half-width; J_m has M = (2m+1)^d frequencies    */
    int32_t L;              /* FFT size per dim of the Toeplitz embedding (>= 4m+1) */
    int32_t nf;             /* spreading grid size per dim                     */
    int32_t nf_eval;        /* type-2 grid size per dim                        */
    int32_t w;              /* exponential-of-semicircle kernel width (cells)  */
    int32_t spread_method;  /* method actually used                            */
    int32_t tile;           /* tile edge used by the tiled spreader, region
                               edge used by the region spreader               */
    int32_t setup_passes;   /* precision 32: 1, or 2-3 when a pass was repeated:
                               with the exact maximum of y (a data value
                               exceeded the scale bound taken from a sample of
                               y) and/or with the worst-case fixed-point scale
                               (a cell of the load-based scale overflowed)     */
    int64_t M;              /* (2m+1)^d                                        */
    int64_t n;              /* N                                               */
    double h;               /* frequency spacing                               */
    double es_beta;         /* ES kernel shape parameter                       */
    double nufft_tol;
    double kernel_l2;       /* ||k||_{L2[-1,1]^d} (Matern rule), else 0         */
    double ms_sort, ms_spread, ms_fft, ms_deconv, ms_setup_total; /* last setup */
} efgp_info;

/* CG launch modes.  GRAPH: the multi-kernel iteration captured in a
 * hipGraph, iters_per_sync (0 => 16) iterations per replay.  PLAIN: the same
 * kernels launched one by one (identical arithmetic).  BLOCK: one workgroup
 * per system runs iters_per_sync whole iterations per launch with the lines
 * in LDS and the vectors in registers (the same recurrences; sums in another
 * order, so iterates agree to rounding); only for the Hermitian 2D systems
 * (real data, precond NONE/JACOBI/LEARNED, no beta_init) whose column pass
 * fits the workgroup's LDS, (2 ceil(L/2) + 1) L complex values (FP32: L up to
 * 135 on a 160 KB LDS; FP64: L up to 100), else EFGP_EINVAL.  AUTO: BLOCK
 * where the system qualifies, else GRAPH. */
enum efgp_launch { EFGP_LAUNCH_AUTO = 0, EFGP_LAUNCH_PLAIN = 1, EFGP_LAUNCH_GRAPH = 2, EFGP_LAUNCH_BLOCK = 3 };

typedef struct efgp_solve_opts {
    double rel_tol;         /* stop at ||b - A beta|| <= rel_tol ||b||; 0 => eps */
    int64_t max_iter;       /* 0 => 100000                                     */
    int32_t precond;        /* efgp_precond                                    */
    int32_t iters_per_sync; /* CG iterations per host check; 0 => 16 (64 for
                               the BLOCK launch)                               */
    const void* beta_init;  /* device M*nrhs complex warm start, or NULL       */
    const void* precond_diag; /* device nrhs*M positive reals in the plan's
                               precision (EFGP_PRECOND_DIAG), or NULL; a
                               non-finite or non-positive entry is refused
                               with EFGP_EINVAL before iterating              */
    const float* mlp_weights; /* device packed network (EFGP_PRECOND_LEARNED)  */
    int64_t stall_window;   /* iterations without a 2x drop of the best residual
                               that count as a stall of preconditioned CG;
                               0 => 1000                                       */
    void* stream;           /* hipStream_t; 0 => null stream                   */
    int32_t record_history; /* >0: keep per-iteration residuals (host)         */
    int32_t launch;         /* efgp_launch: how iterations are launched        */
    int32_t refine;         /* precision 32: >0 => mixed-precision iterative
                               refinement with at most `refine` outer steps:
                               each forms r = b - A beta in double (double
                               FFT(v), built on first use) and solves A d = r
                               by single-precision (P)CG to at most 1e-6; the
                               stopping test uses the double residual.  beta_out
                               is the double iterate rounded to single.  An
                               inner system whose PCG stalls (stall_window)
                               stops there, and the next outer step continues
                               from the improved iterate (no plain-CG
                               fall-back inside the refinement).  It pays
                               while single-precision products resolve the
                               system (u kappa < 1); beyond that each outer
                               step gains less and a precision-64 plan is
                               faster.  0 => plain single-precision CG;
                               ignored in precision 64                       */
    int32_t reserved;
} efgp_solve_opts;

typedef struct efgp_solve_stats {
    int64_t iterations;     /* max over right-hand sides                       */
    int32_t converged;      /* number of systems that met rel_tol              */
    int32_t fell_back;      /* number of systems that fell back to plain CG    */
    double rel_residual;    /* max true ||b - A beta||/||b|| after the solve   */
    double ms_solve;        /* wall time of the call                           */
    const double* history;  /* record_history: residual of system 0 per iteration
                               (owned by the plan; valid until the next solve) */
    int64_t history_len;
    int32_t refine_steps;   /* outer refinement steps taken (opts.refine)      */
    int32_t reserved;
} efgp_solve_stats;

/* ----------------------------------------------------------------------- */

/* Build a plan: parameter rules (Sec. 4.2: SE rule, eq. (maternheur) for
 * 1/2 <= nu <= 5/2, eq. (maternhm) above), spectral weights D_j =
 * sqrt(h^d khat(h j)) (eq. (117)), one spreading pass over the points
 * (eqs. (88), (rhs)), deconvolution, and FFT(v) for the Toeplitz product.
 * x and y are read on `stream` and not retained.  Blocks until the setup is
 * complete (the domain check needs its result).  On error *out = NULL. */
int efgp_setup(const efgp_problem* p, efgp_plan** out);

/* Solve (D F*F D + sigma_r^2 I) beta_r = b_r for every system r by (P)CG
 * (step 4 of the EFGP algorithm).  beta_out: device nrhs*M complex in the
 * plan's precision.  Stopping uses the unpreconditioned residual; the true
 * residual is recomputed at the end and iteration resumes if it exceeds
 * 1.1 rel_tol.  Blocks until done.  Returns EFGP_NOT_CONVERGED (beta_out =
 * last iterate) when max_iter is reached.  Preconditioned CG that stalls
 * (stall_window) continues as plain CG from its iterate; one that breaks
 * down (a non-finite residual or step) restarts plain CG from zero; both
 * return EFGP_FELL_BACK.  Real data make b Hermitian (b at -j is the
 * conjugate of b at j, i.e. b[M-1-k] = conj b[k] in the layout of J_m); in
 * 2D with precond NONE, JACOBI or LEARNED, no beta_init and an embedding
 * L <= 2048 (precision 32) or L <= 1024 (precision 64) the solve starts
 * from b symmetrised, (b[k] + conj b[M-1-k]) / 2, keeps every iterate
 * exactly Hermitian and returns beta with beta[M-1-k] = conj beta[k]. */
int efgp_solve(efgp_plan* plan, const efgp_solve_opts* opts, void* beta_out,
               efgp_solve_stats* stats);

/* Posterior mean at q targets (step 6): mu_r(t) = Re sum_j D_j beta_rj
 * exp(-2 pi i h <j,t>), by a type-2 NUFFT.  targets: device d*q SoA in
 * [0,1]^d; beta: device nrhs*M complex; mu_out: device nrhs*q reals.  The
 * plan is only read, so evaluations on different streams may overlap only
 * if they use different plans (the plan owns the type-2 grid).
 * Asynchronous on `stream`; a target outside [0,1]^d is reported by the
 * next call to efgp_eval_status. */
int efgp_eval(efgp_plan* plan, const void* beta, int64_t q, const void* targets,
              void* mu_out, void* stream);

/* Posterior variance at q targets (Remark r:var: one linear solve per
 * target), in weight space: s(t) = sigma_r^2 phi(t)^H A^{-1} phi(t) with
 * phi_j(t) = D_j exp(+2 pi i h <j,t>) and A = D F*F D + sigma_r^2 I the
 * system matrix of step 4; by the Woodbury identity this is
 * k~(t,t) - k~_t^T (K~ + sigma_r^2 I)^{-1} k~_t for the kernel k~ of eq. (110)
 * (eqs. (mu)-(362)).  Targets are solved in batches of up to 64 systems by
 * the batched CG of efgp_solve with its options (rel_tol per system;
 * precond NONE, JACOBI or LEARNED; refine as for efgp_solve, with the
 * right-hand sides phi(t) also formed in double; beta_init must be NULL).  r: the data
 * vector whose sigma^2 is used.  targets: device d*q SoA in [0,1]^d;
 * var_out: device q reals.  stats: worst iterations and residual over the
 * batches, converged = number of targets that met rel_tol.  Blocks until
 * done.  EFGP_EDOMAIN if a target lies outside [0,1]^d (var_out is then
 * unspecified); EFGP_NOT_CONVERGED / EFGP_FELL_BACK as for efgp_solve. */
int efgp_variance(efgp_plan* plan, int32_t r, int64_t q, const void* targets, void* var_out,
                  const efgp_solve_opts* opts, efgp_solve_stats* stats);

/* GP prior sampling in the equispaced Fourier basis (Sec. 6: evaluate
 * f(x) = sum_j D_j xi_j exp(-2 pi i h <j,x>) with iid random coefficients by
 * the type-2 NUFFT of step 6).  efgp_prior_setup builds a kernel-only plan
 * from the kernel fields of *p (dim, kernel, lengthscale, nu, variance, eps,
 * precision, nufft_tol, m_override, stream; nrhs = samples per call, 1..64);
 * n, x, y and sigma2 are ignored, and efgp_solve/efgp_mean_at_points reject
 * the plan.  efgp_sample_prior: xi device nrhs*M complex whose real and
 * imaginary parts the caller draws iid N(0,1) (the library draws no random
 * numbers); f_out device nrhs*q reals f_r(t) = Re sum_j D_j xi_rj
 * exp(-2 pi i h <j,t>), whose covariance is the discretized kernel
 * k~(t - t') (Sec. 3.1, eq. (110)).  Targets, domain errors and streams as for
 * efgp_eval. */
int efgp_prior_setup(const efgp_problem* p, efgp_plan** out);
int efgp_sample_prior(efgp_plan* plan, const void* xi, int64_t q, const void* targets, void* f_out,
                      void* stream);

/* Posterior mean at the N observation points (step 7 of the EFGP algorithm,
 * eq. (bmu): mu = Phi beta, the type-2 NUFFT of step 6 with q = N).  x: the
 * device d*N SoA points the plan was built from (the plan does not keep
 * them); beta: device nrhs*M complex; mu_out: device nrhs*N reals.
 * Asynchronous on `stream`; domain errors as for efgp_eval. */
int efgp_mean_at_points(efgp_plan* plan, const void* beta, const void* x, void* mu_out, void* stream);

/* Result of the domain check of the last efgp_eval (blocks on its stream). */
int efgp_eval_status(efgp_plan* plan);

/* Spread autotuner.  efgp_tune_spread times the setup (steps 1-3) of the
 * caller's problem with every candidate spreader — the whole-region LDS
 * grid spreader, the region spreader (after its partition by region) and
 * the tiled spreader (after its bin-sort by tile) at tile edges T/2, T, 2T,
 * with T = 256, 32, 8 cells for d = 1, 2, 3 — each run twice with the
 * second run timed, and stores the fastest in a process-wide table
 * keyed by (device, d, precision, nrhs, n_f, w, floor(log2 N)).  A later
 * efgp_setup with spread_method EFGP_SPREAD_AUTO and tile 0 on a problem of
 * the same key uses the tuned spreader; explicit methods and tiles are
 * honoured as given (except the tile of the many-vector tiled spreader,
 * see efgp_spread).  The problem's spread_method and tile fields are
 * ignored; x and y are read as by efgp_setup (stream-ordered).
 * Errors: as efgp_setup for the problem itself; candidates the shape cannot
 * take (region or tile beyond LDS, the region spreader outside precision 32
 * with one data vector) are skipped.
 *   efgp_tune_save: write the table to a text file (EFGP_EINVAL if the path
 *                   is NULL or cannot be written).
 *   efgp_tune_load: merge a file written by efgp_tune_save into the table;
 *                   *entries (nullable) receives the number read.  A missing,
 *                   unreadable or malformed file is EFGP_EINVAL and changes
 *                   nothing.
 *   efgp_tune_clear: empty the table. */
typedef struct efgp_tune_result {
    int32_t spread_method;  /* fastest: EFGP_SPREAD_TILES, _GRID_LDS or _REGIONS */
    int32_t tile;           /* its tile edge (tiled spreader), its region edge
                               (region spreader), else 0                       */
    double ms_setup;        /* its setup time, ms                              */
    int32_t candidates;     /* configurations timed                            */
    int32_t reserved;
} efgp_tune_result;
int efgp_tune_spread(const efgp_problem* problem, efgp_tune_result* out);
int efgp_tune_save(const char* path);
int efgp_tune_load(const char* path, int32_t* entries);
void efgp_tune_clear(void);

/* Stage access (for stage-wise checks and for the preconditioner features).
 * All copy device-to-device on `stream` and are asynchronous.
 *   efgp_get_toeplitz: v on J_2m, (4m+1)^d complex double (eq. (88)).
 *   efgp_get_rhs:      b = D F* y, nrhs*M complex double (eq. (rhs)).
 *   efgp_get_weights:  D, M doubles (eq. (117)).
 *   efgp_apply:        out = (D F*F D + sigma_r^2 I) in for every system,
 *                      nrhs*M complex in the plan's precision (eq. (97)). */
int efgp_get_toeplitz(const efgp_plan* plan, double* v_out, void* stream);
int efgp_get_rhs(const efgp_plan* plan, double* b_out, void* stream);
int efgp_get_weights(const efgp_plan* plan, double* d_out, void* stream);
int efgp_apply(efgp_plan* plan, const void* in, void* out, void* stream);

/* efgp_apply for callers that cannot allocate device memory (code under
 * hipGraph stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same product, the same kernels and bit-identical output,
 * but the FFT intermediates live in a static device array of 64 MiB per GPU
 * (held until the process ends; its address is looked up by efgp_setup /
 * efgp_prior_setup on their device), so the call allocates nothing, on the
 * device or the host.  in, out: device nrhs*M complex in the plan's
 * precision, caller-owned; asynchronous on `stream`.  The plan's device must
 * be current.  Needs 2 * 2 * es * nb * nrhs bytes (es = 4 or 8; nb = 1, W L
 * or W L^2 for d = 1, 2, 3, W = 2m+1); a plan needing more than 64 MiB gets
 * EFGP_ETOOLARGE and nothing is launched.  Every call on one GPU shares the
 * array: calls that overlap on a GPU (on different streams, or from several
 * threads) race and give wrong results; serialize them. */
int efgp_apply_noalloc(efgp_plan* plan, const void* in, void* out, void* stream);

/* Per-frequency features of the learned diagonal preconditioner for system
 * r (scaled to order one): feats_out is device M*EFGP_NFEAT floats,
 * row-major per frequency:
 *   0: h |j| ell                        (dimensionless frequency)
 *   1: 0.1 log(N D_j^2 / sigma_r^2)     (spectral weight against the noise)
 *   2: 0.2 log sigma_r^2
 *   3: 0.5 log ell
 *   4: 0.1 log(mean |v_k| / N + 1e-12)  (local magnitude of the Toeplitz vector:
 *                                         mean over |k_l - j_l| <= 2, k in J_2m)
 * and jacobi_out (nullable) device M floats 1/(N D_j^2 + sigma_r^2), the
 * inverse diagonal of the system matrix (T_jj = v_0 = N). */
#define EFGP_NFEAT 5
int efgp_features(const efgp_plan* plan, int32_t r, float* feats_out, float* jacobi_out,
                  void* stream);

/* Eigenvalues of the circulant preconditioner of system r (the open
 * direction of the conclusions: preconditioning the Toeplitz-plus-diagonal
 * system of eq. (97)).  With J = N D_j^2 + sigma_r^2 and E = J^(-1/2) A
 * J^(-1/2) (unit diagonal), E is placed on the indices j + m in {0..2m}^d of
 * the periodic grid {0..K-1}^d, K the smallest integer >= 2m+1 with prime
 * factors 2, 3, 5 only, the rest of the grid carrying the identity; lambda_s
 * = f_s^H (E (+) I) f_s with f_s(j) = exp(2 pi i <s, j>/K) / K^(d/2), the
 * eigenvalues of the circulant nearest to it in the Frobenius norm (T. Chan,
 * 1988).  The preconditioner is P = J^(-1/2) R^T F^H diag(1/lambda) F R
 * J^(-1/2), R the restriction to the M frequencies.
 *   period:  host, receives K (nullable).
 *   lam_out: device, K^d reals in the plan's precision, C order over s, or
 *            NULL to query K only.
 * Errors: EFGP_EINVAL for a NULL plan, r outside 0..nrhs-1, or a kernel-only
 * plan (no points, no system). */
int efgp_circulant_eigs(efgp_plan* plan, int32_t r, int32_t* period, void* lam_out, void* stream);

int efgp_get_info(const efgp_plan* plan, efgp_info* info);

/* Waits for the plan's stream, then hands its device buffers, pinned host
 * staging, stream and events to process-wide caches (exact-size reuse, at
 * most 2 GiB of device memory per device) and drops its reference to the
 * cached CG graph; a later plan of the same sizes reuses all of them. */
void efgp_destroy(efgp_plan* plan);

/* Setup keeps its scratch (sorted point copies, partial grids) in device
 * chunks that are reused by later setups on the same device, and destroyed
 * plans leave their buffers, streams, events and CG graphs in caches.  This
 * frees every cached resource no live plan holds; call it only when no
 * efgp_setup is running. */
void efgp_release_workspace(void);
const char* efgp_strerror(int status);

/* ----------------------------------------------------------------------- *
 * Preconditioner network: an MLP 5 -> 64 -> 64 -> 64 -> 1 (ReLU) that maps
 * each frequency's features (efgp_features) to an estimate o_j of the best
 * exponent s of the diagonal family p_j = (N D_j^2 + sigma^2)^(-s) (s = 1 is
 * Jacobi, s = 0 plain CG).  The solver (EFGP_PRECOND_LEARNED) averages o_j
 * over the system's frequencies into s_bar (outputs clamped to [-1, 3], a
 * non-finite one counts as 1), clamps it to [0, 1.25] (the range searched in
 * training) and uses p_j = (N D_j^2 + sigma^2)^(-s_bar); when
 * |s_bar - 1| < EFGP_MLP_GATE it uses the Jacobi diagonal itself.  The gate
 * was chosen on the training problems: it minimises their geometric-mean
 * iteration count relative to Jacobi.  Weights are bf16 for
 * the products (MFMA, float accumulation) with float master copies.  Packed float layout (EFGP_MLP_NPARAM floats):
 *   W1[64][5] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[64] b4[1]
 * (W[out][in], row-major).  All pointers are device pointers.
 * ----------------------------------------------------------------------- */
#define EFGP_MLP_HIDDEN 64
#define EFGP_MLP_GATE 0.15f
#define EFGP_MLP_NPARAM (64 * 5 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 + 1)

/* out[i] = network(feats[i]) for rows i < rows (feats: rows*EFGP_NFEAT). */
int efgp_mlp_forward(const float* params, int64_t rows, const float* feats, float* out,
                     void* stream);

/* Loss and gradient of the mean squared error (1/rows) sum_i w_i (o_i - t_i)^2
 * over a batch; grad_out (EFGP_MLP_NPARAM floats) is overwritten; loss_out is
 * one device double.  weights may be NULL (all ones). */
int efgp_mlp_loss_grad(const float* params, int64_t rows, const float* feats,
                       const float* target, const float* weights, float* grad_out,
                       double* loss_out, void* stream);

/* One Adam step on the float master parameters (state m, v: EFGP_MLP_NPARAM
 * floats each, zero at step 1). */
int efgp_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t step,
                  float lr, float beta1, float beta2, float eps, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* EFGP_H */
