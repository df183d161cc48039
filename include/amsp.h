/*
 * amsp.h -- C ABI of the MI355X two-grid algebraic multiscale preconditioner.
 *
 * Method: "An algebraic multiscale preconditioner for large sparse SPD
 * matrices" (Zhou, Fu, Chung).  Section 3.1 defines the non-overlapping
 * graph subdomains, the coarse space spanned by locally supported basis
 * vectors (columns of R0^T) and the Galerkin coarse matrix A0 = R0 A R0^T;
 * Section 3.2 defines the local matrices A_i = R_i A R_i^T, the Neumann
 * modification hat A_i (diagonal replaced by minus the sum of the row's
 * off-diagonals), the weighting S_i = diag(hat A_i) and the local generalized
 * eigenproblem hat A_i psi = lambda S_i psi whose lowest modes form R0^T;
 * Section 5 (parameter test) solves it in the standard form
 * S^{-1/2} hat A S^{-1/2} z = lambda z.
 *
 * The preconditioner applied here is the additive two-level operator
 *     M^{-1} r = sum_i R_i^T A_i^{-1} R_i r  +  R0^T A0^{-1} R0 r
 * on overlapping regions (delta graph layers around each core), with every
 * local eigenvector divided by the multiplicity of its dof (partition of
 * unity).  It is SPD, so the Krylov method is preconditioned CG.
 *
 * Conventions shared by every entry point:
 *   - Host inputs (CSR, partition) are borrowed for the call and copied.
 *   - Vectors named *_dev are caller-owned device buffers (HIP device
 *     pointers, e.g. torch tensors' data_ptr()), float64, column-major
 *     n x nrhs.
 *   - All device work is ordered on the stream given in amsp_options.stream
 *     (a hipStream_t; NULL = the legacy default stream).
 *   - Errors are status codes; nothing throws or aborts across the ABI.
 *     amsp_last_error() gives a message (e.g. the failing subdomain).
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef AMSP_H
#define AMSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AMSP_OK = 0,
  AMSP_ERR_ARG = -1,            /* bad argument (null pointer, nev < 0, ...)           */
  AMSP_ERR_CSR = -2,            /* malformed CSR (row_ptr, unsorted/out-of-range cols) */
  AMSP_ERR_NONSYM = -3,         /* values not symmetric to 1e-14 max|a|               */
  AMSP_ERR_PARTITION = -4,      /* part[j] out of range or an empty part              */
  AMSP_ERR_NEUMANN_DIAG = -5,   /* some S_jj <= 0 (weighting matrix not positive)      */
  AMSP_ERR_LOCAL_NOT_SPD = -6,  /* Cholesky of a local matrix failed                   */
  AMSP_ERR_EIG_NOCONV = -7,     /* local eigensolver hit eig_maxit (see setup info)    */
  AMSP_ERR_COARSE_NOT_SPD = -8, /* Cholesky of A0 failed                               */
  AMSP_ERR_PCG_NOCONV = -9,     /* PCG hit maxit; u holds the last iterate             */
  AMSP_ERR_BREAKDOWN = -10,     /* non-finite or zero curvature in PCG                 */
  AMSP_ERR_HIP = -11,           /* a HIP runtime call failed                           */
  AMSP_ERR_OOM = -12            /* device or host allocation failed                    */
} amsp_status;

/* Storage precision of the local factors, the coarse basis and the coarse
 * inverse factor used by the apply.  The outer CG, its dot products, A0 and
 * its Cholesky factorisation are float64 in every form. */
typedef enum {
  AMSP_FP64 = 0,        /* everything float64                                         */
  AMSP_MIXED_FP32 = 1,  /* local factors, basis, coarse inverse factor stored float32,  */
                        /* applied with float32 accumulation; eigensolve sweeps float32 */
  AMSP_MIXED_BF16 = 2   /* as MIXED_FP32 but the coarse basis stored bfloat16           */
} amsp_precision;

typedef enum {
  AMSP_ORDER_RCM = 0,     /* reverse Cuthill-McKee local order, tile profile (default) */
  AMSP_ORDER_NATURAL = 1  /* ascending global index, tile profile                       */
} amsp_local_order;

/* Host CSR matrix, symmetric positive definite, sorted columns, diagonal
 * present.  row_ptr has n+1 entries; nnz = row_ptr[n] < 2^31. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t *row_ptr;
  const int32_t *col_idx;
  const double *val;
} amsp_csr;

typedef struct {
  int32_t overlap;          /* delta: graph layers added around each core (default 1)  */
  amsp_precision precision; /* default AMSP_FP64                                        */
  int32_t pou;              /* 0: divide by dof multiplicity (default); 1: none         */
  int32_t local_order;      /* amsp_local_order                                         */
  int32_t dense_tiles;      /* 1: store the full lower triangle of tiles (no profile)   */
  double eig_tol;           /* residual bound ||B x - theta x|| for the kept pairs;      */
                            /* 0 (default): 1e-12, or 1e-4 for the mixed forms           */
  int32_t eig_maxit;        /* maximum subspace sweeps (default 80)                      */
  double eig_shift;         /* sigma in (B + sigma I)^{-1} (default 1e-4)                */
  int32_t chunk;            /* PCG iterations per host poll (default 8)                  */
  int32_t flexible;         /* 1: Polak-Ribiere beta; -1 (default): on for mixed forms   */
  int32_t keep_a0;          /* 1: keep a copy of A0 for amsp_get_coarse_matrix           */
  int32_t timing;           /* bit c set: time launches of PCG kernel class c (the        */
                            /* classes of amsp_info.kernel_ms) with HIP events; 0: off;  */
                            /* 0x1F: all.  Each timed launch adds two event records.     */
  int32_t timing_stride;    /* time every timing_stride-th launch of a class (>= 1)      */
  void *stream;             /* hipStream_t                                               */
  int32_t singular;         /* 1: A is singular with the constant vector as its null     */
                            /* space (homogeneous Neumann problem, Section 5).  The      */
                            /* coarse term is then the pseudo-inverse of A0 (Section     */
                            /* 3.1) on residuals orthogonal to the constants, applied as */
                            /* (A0 + alpha u u^T)^{-1} with u = R0 1, alpha = tr A0/u.u; */
                            /* it differs from A0^+ only by a constant vector, which A   */
                            /* annihilates.  f must then sum to zero; the solvers return */
                            /* a solution determined up to a constant.  Default 0.       */
  int32_t cycle;            /* 0: additive two-level operator (default);                 */
                            /* 1: symmetric multiplicative two-grid cycle (the paper's   */
                            /* two-grid algorithm analysed in Section 4): x1 = W r,      */
                            /* x2 = x1 + C (r - A x1), z = x2 + W (r - A x2), with the   */
                            /* smoother W = w sum_i R_i^T A_i^{-1} R_i and C the coarse  */
                            /* term; twice the local solves and two more SpMVs per apply */
  double smoother_weight;   /* w of cycle 1; 0 (default): 1 / (largest number of regions */
                            /* containing one dof), which keeps the cycle SPD            */
  int32_t coarse_basis;     /* mixed forms only: 0 (default): A0 = R0 A R0^T is formed   */
                            /* from the basis as stored (rounded to float32/bfloat16,    */
                            /* products in float64), the Galerkin matrix of the basis    */
                            /* the apply uses; 1: from the float64 basis before          */
                            /* rounding (the apply then uses an approximation of that    */
                            /* projection).  Measured with a bfloat16 basis on the 1M    */
                            /* high-contrast benchmark matrix: 0 reaches the rounding    */
                            /* floor's level in 805 steps, 1 stalls near 2e-3.           */
  int32_t coarse_solver;    /* factorisation of A0: 0 (default): automatic, the sparse   */
                            /* one when N_c > 8192; 1: dense tiled Cholesky and its      */
                            /* inverse factor W0 (two parallel triangular products per   */
                            /* solve); 2: sparse multifrontal Cholesky over a nested-    */
                            /* dissection order of the subdomains (the paper's sparse    */
                            /* direct coarse solver, Section 5), one launch per level    */
                            /* and direction per solve.  Problems with singular = 1 use  */
                            /* the dense factorisation.                                   */
} amsp_options;

typedef struct {
  int32_t iterations;       /* CG steps taken (SpMVs with the search direction)   */
  int32_t converged;        /* 1 if the true relative residual <= rtol            */
  double relres_recursive;  /* ||r_k|| / ||f|| from the recurrence                 */
  double relres_true;       /* ||f - A u|| / ||f|| recomputed at the end           */
  int32_t restarts;         /* residual replacements after a false convergence     */
  double solve_ms;          /* wall time of the call                               */
  int64_t bytes_per_iter;   /* algorithmic HBM bytes of one CG iteration           */
  /* with opt.timing: summed device time and count of the timed launches per
   * kernel class (average duration = kernel_ms / kernel_launches):
   * [0] SpMV (+ search-direction update), [1] local apply (gather,
   * forward/backward solves, prolongation of the coarse correction), [2]
   * coarse restriction and solve (both triangular products, or the sparse
   * factor's solve), [3] scatter-sum, [4] CG vector update and reductions */
  double kernel_ms[5];
  int32_t kernel_launches[5];
  int64_t local_apply_bytes; /* algorithmic bytes of one local-apply launch          */
  /* attainable-accuracy floor eps * || |A| |u| || / ||f||: no float64 vector u
   * can be certified below it; converged means relres_true <= max(rtol, floor) */
  double relres_floor;
  /* steps of the first CG segment: the step at which the recursive residual
   * first reached rtol, before any restart from the true residual (one
   * right-hand side; with several, their sum) */
  int32_t first_segment;
} amsp_info;

typedef struct {
  int32_t nsub;             /* N subdomains                                         */
  int32_t nc;               /* coarse dimension N_c = sum_i m_i                     */
  int64_t sum_ni;           /* sum of region sizes                                  */
  int32_t max_ni;
  int64_t factor_tiles;     /* 64x64 profile tiles of one local factor set (the     */
                            /* diagonal ones stored as packed lower triangles)     */
  int32_t eig_sweeps;       /* subspace sweeps used                                 */
  int32_t eig_unconverged;  /* subdomains not converged at eig_maxit                */
  int32_t n_gap_flags;      /* subdomains with lambda_{m+1} - lambda_m tiny         */
  double mu_c;              /* min_i lambda_{m_i+1}                                 */
  double phase_ms[8];       /* plan (host planning + upload of its index arrays),   */
                            /* input matrix host->device transfer, extract, local   */
                            /* chol, eig, basis+A0, coarse chol+inverse, total      */
  double coupling_ms;       /* host coupling-plan thread (overlaps device work)     */
  double coupling_wait_ms;  /* time the device path waited for it                   */
  double plan_host_ms;      /* part of phase_ms[0]: the host planning itself        */
  double plan_upload_ms;    /* part of phase_ms[0]: device copies of the plan       */
  int32_t coarse_solver;    /* 1: dense, 2: sparse multifrontal (as used)           */
  int32_t coarse_fronts;    /* sparse: fronts (supernodes) and levels of the tree   */
  int32_t coarse_levels;
  double coarse_gflop;      /* sparse: tile-product flops of factor + inverse parts */
  double coarse_factor_mb;  /* solve's factor bytes (dense W0 lower tiles, or the   */
                            /* sparse fronts' X), in MB, in the apply's precision   */
} amsp_setup_info;

typedef struct amsp_handle amsp_handle;

/* Fills *opt with the defaults listed above. */
void amsp_default_options(amsp_options *opt);

/* Setup (Sections 3.1-3.2): validates A and the partition on the host,
 * plans the overlapping regions, then on the device extracts the local
 * matrices, factors them, solves the batched local eigenproblems, builds the
 * PoU-scaled basis, forms A0 = R0 A R0^T and factors it.
 *   A         host CSR (copied).
 *   partition host int32[n], values in [0, nparts); every part non-empty.
 *   nev       eigenvectors kept per subdomain (m_i = min(nev, n_i)); 0 gives
 *             one-level additive Schwarz.
 *   opt       NULL for defaults.
 *   out       receives the handle; NULL on failure.
 * Blocks until the setup is complete. */
amsp_status amsp_setup(const amsp_csr *A, const int32_t *partition, int32_t nparts,
                       int32_t nev, const amsp_options *opt, amsp_handle **out);

/* z = M^{-1} r for nrhs columns (asynchronous on the handle's stream), with
 * M^{-1} = sum_i R_i^T A_i^{-1} R_i + R0^T A0^{-1} R0: the coarse term of
 * Section 3.1 (R0 from the eigenproblem of Section 3.2, A0 its Galerkin
 * matrix) plus the local solves on the overlapping regions (the additive
 * two-level reading of the method; with cycle = 1 the multiplicative cycle).
 * parts: 3 = both terms, 1 = local solves only, 2 = coarse correction only.
 * Columns are n apart (column-major).  Two or more columns are taken up to 16
 * at a time with one pass over the local factor: triangular solves with a
 * block of right-hand sides, whose diagonal products run on the matrix cores
 * (the mixed forms then use their f32-stored factor with float64 arithmetic,
 * so a column can differ from its single-column result at float32 rounding).
 * The first such call allocates the block workspace, 3 x 128 bytes per padded
 * local row, kept until amsp_destroy.  With cycle = 1, parts = 3 applies the
 * cycle column by column. */
amsp_status amsp_apply(amsp_handle *h, const double *r_dev, double *z_dev, int32_t nrhs);
amsp_status amsp_apply_parts(amsp_handle *h, const double *r_dev, double *z_dev,
                             int32_t nrhs, int32_t parts);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): z = M^{-1} r for
 * nrhs columns (n apart) through the block path of amsp_apply (up to 16
 * columns per pass, also for a single column), with its workspace -- the
 * gathered, solved and output blocks, the coarse vectors and the coarse
 * products' partial sums, 8 * (3 rows * 16 + 3 ncp * 16 + T0^2 * 1024) bytes
 * with rows the padded local rows and ncp = 64 T0 -- taken from a 64 MiB
 * array the library holds on each device until the process ends.  Calls no
 * allocating routine.  parts as for amsp_apply_parts (the additive operator
 * only).  Errors: AMSP_ERR_ARG when the workspace exceeds 64 MiB, when
 * cycle = 1 and parts = 3, or for a mixed form whose float32 block-solve
 * factor copy does not exist yet (the first amsp_apply with nrhs >= 2 builds
 * it).  Asynchronous on the handle's stream.  Every call on one device shares
 * that device's array: calls that overlap in time on one device (two
 * streams, two threads, two handles) race and must be serialised by the
 * caller.  Results equal amsp_apply's block path. */
amsp_status amsp_apply_noalloc(amsp_handle *h, const double *r_dev, double *z_dev, int32_t nrhs,
                               int32_t parts);

/* Preconditioned CG (Saad, Iterative Methods for Sparse Linear Systems,
 * Algorithm 9.1) with the operator of amsp_apply, which is SPD; the paper's
 * own Krylov method (Section 5) is GMRES, amsp_gmres below.  From u = 0
 * until the recursive residual satisfies
 * ||r_k|| <= rtol ||f||; the true residual f - A u is then recomputed and
 * accepted if it is below max(rtol, floor) with floor = eps || |A||u| || / ||f||
 * (the rounding level of any float64 residual); otherwise CG restarts from the
 * true residual (at most 3 times).  Blocks; info may be NULL.  On
 * AMSP_ERR_PCG_NOCONV u holds the last iterate and the handle stays valid.
 * The first call allocates two pinned host slots for the solver state (a few
 * hundred bytes), kept until amsp_destroy. */
amsp_status amsp_pcg(amsp_handle *h, const double *f_dev, double *u_dev, int32_t nrhs,
                     double rtol, int32_t maxit, amsp_info *info);
/* With nrhs >= 2 (columns n apart) and the additive operator, up to 16
 * columns run together: one CG recurrence per column, with the stopping rule
 * above applied per column, sharing every SpMV (matrix entries read once) and
 * every preconditioner application (the block path of amsp_apply).  The
 * workspace (4 n doubles per column) is allocated per call from the handle's
 * cache.  info sums the columns' iterations and reports the worst residuals;
 * a last single column takes the one-column path.  A column that meets
 * p.Ap <= 0 or a non-finite value stops there (keeping its last iterate);
 * the others run to their own end, restarts included, and the call then
 * returns AMSP_ERR_BREAKDOWN with u and info written for every column. */

/* Independent problems solved together (the batched form): the handle's
 * matrix is block-diagonal, block s being problem s on rows
 * [prob_ptr[s], prob_ptr[s+1]) (set up as one matrix with one partition,
 * the parts of each problem disjoint: every kernel of the setup and of each
 * step then covers all problems at once).  One CG recurrence per (problem,
 * column) pair, nrhs columns (1 .. 16, n apart, column-major): each shares
 * every matrix product and preconditioner application (the block path of
 * amsp_apply) but takes its scalars from its own problem's rows, so it
 * follows the iterates of that problem solved alone up to rounding.  The
 * stopping rule of amsp_pcg (true residual, attainable floor, at most 3
 * restarts) applies per recurrence, with ||f|| that problem's column norm.
 *   prob_ptr    host int64[nprob + 1]: 0 = prob_ptr[0] < ... < prob_ptr[nprob] = n
 *   iterations  host int32[nprob * nrhs] (problem-major) or NULL: steps taken
 *   relres      host double[nprob * nrhs] or NULL: true relative residuals
 * info sums the steps and reports the worst residuals.  Errors: AMSP_ERR_ARG
 * for a bad prob_ptr, nrhs outside 1..16, cycle = 1, or a stored entry of A
 * that couples two problems (checked on the device); AMSP_ERR_PCG_NOCONV if
 * some recurrence did not converge (u holds the last iterates);
 * AMSP_ERR_BREAKDOWN if p.Ap <= 0 or a non-finite value stopped some
 * recurrence: the others (every other problem's, and the same problem's
 * other columns) run to their own end, and u, info, iterations and relres
 * are written for all of them.  Workspace:
 * 4 n nrhs doubles and small tables from the handle's cache.  Blocks. */
amsp_status amsp_pcg_batched(amsp_handle *h, int32_t nprob, const int64_t *prob_ptr,
                             const double *f_dev, double *u_dev, int32_t nrhs, double rtol,
                             int32_t maxit, amsp_info *info, int32_t *iterations,
                             double *relres);

/* Restarted GMRES with the preconditioner, the Krylov method of the paper's
 * experiments (Section 5: GMRES preconditioned by the two-level method, run
 * until the relative residual has dropped by a factor 1e-6).  Right
 * preconditioning in flexible form: z_j = M^{-1} v_j are kept and
 * u = Z y, so the residual GMRES minimises is the true one, f - A u, as for
 * amsp_pcg.  From u = 0; every restart-th step (1 .. AMSP_GMRES_MAX_RESTART)
 * the iterate is formed, f - A u recomputed and the next cycle starts from it.
 * Stops when ||f - A u|| <= max(rtol, floor) ||f|| at the end of a cycle (the
 * cycle ends once its residual estimate reaches rtol), or after maxit steps
 * (AMSP_ERR_PCG_NOCONV; u holds the last iterate).  Arnoldi by classical
 * Gram-Schmidt applied twice, fixed-order reductions; the small least-squares
 * problem by Givens rotations on the host.  Workspace (allocated by the call,
 * kept in the handle's cache): (2 restart + 1) n doubles.  info: iterations =
 * GMRES steps (preconditioner applications), restarts = cycles after the
 * first, relres_recursive = last residual estimate; the history getter below
 * returns the estimates after every step.  Blocks; info may be NULL.  The
 * first call allocates two pinned host slots of 129 doubles for the step
 * coefficients, kept until amsp_destroy. */
#define AMSP_GMRES_MAX_RESTART 64
amsp_status amsp_gmres(amsp_handle *h, const double *f_dev, double *u_dev, int32_t nrhs,
                       int32_t restart, double rtol, int32_t maxit, amsp_info *info);

/* Relative residuals ||r_k|| / ||f|| of the last amsp_pcg (recursive
 * residuals) or amsp_gmres (residual estimates) call (last right-hand side;
 * k = 0 .. iterations).  *count receives the length; at most cap values are
 * written to relres_host (may be NULL). */
amsp_status amsp_get_pcg_history(const amsp_handle *h, double *relres_host, int32_t cap,
                                 int32_t *count);

/* y = A x with the handle's matrix (asynchronous). */
amsp_status amsp_spmv(amsp_handle *h, const double *x_dev, double *y_dev);

/* Adjoint of the solve u = A^{-1} f, for the gradient of a scalar loss J(u)
 * with respect to the stored values of A.  Not part of the paper's method:
 * it differentiates the solve the preconditioner serves.  The caller first
 * solves the adjoint system A lambda = dJ/du with amsp_pcg on the same handle
 * (A is symmetric); then dJ/df = lambda and, for every stored entry k of the
 * handle's CSR (row i, column j, in the order of the CSR given to
 * amsp_setup),
 *     grad_val[k] = -lambda[i] * u[j].
 * Each entry is treated as an independent value, so a symmetric perturbation
 * of the pair (i,j),(j,i) changes J by the sum of the two entries.
 *   lambda_dev, u_dev  device vectors of length n (read)
 *   grad_dev           device vector of length nnz (written)
 * Asynchronous on the handle's stream; AMSP_ERR_ARG on a null pointer. */
amsp_status amsp_grad_values(amsp_handle *h, const double *lambda_dev, const double *u_dev,
                             double *grad_dev);

/* Introspection (host copies; each blocks on the stream). */
amsp_status amsp_get_setup_info(const amsp_handle *h, amsp_setup_info *info);
/* Eigenvalues of the local eigenproblems hat A_i psi = lambda S_i psi
 * (Section 3.2, the algebraic eigenproblem), lowest first.  lambda_host:
 * N*(nev+1) values; row i holds lambda_1..lambda_{m_i+1} of subdomain i
 * (unused slots = NaN). */
amsp_status amsp_get_eigenvalues(const amsp_handle *h, double *lambda_host);
/* A0 as a dense row-major nc x nc float64 matrix (needs opt.keep_a0 = 1). */
amsp_status amsp_get_coarse_matrix(const amsp_handle *h, double *a0_host);
/* Region of subdomain i: fills dofs (n_i global indices in the handle's
 * local order) and, if phi is not NULL, the n_i x nev row-major block of
 * PoU-scaled basis vectors (columns >= m_i are zero).  Call with dofs = NULL
 * to get n_i in *ni first. */
amsp_status amsp_get_region(const amsp_handle *h, int32_t i, int32_t *ni, int32_t *dofs,
                            double *phi);

/* Host-only planning (no device work, usable without a GPU): validates the
 * inputs and plans the overlapping regions exactly as amsp_setup does.
 *   region_ptr   N+1 offsets (required)
 *   region_dofs  global dofs of every region in the local order used by the
 *                kernels; NULL to query sizes only; cap = its capacity
 *   ntiles       64x64 tiles of one local factor set (may be NULL)
 *   npairs       coupled subdomain pairs of A0 (may be NULL) */
amsp_status amsp_plan_regions(const amsp_csr *A, const int32_t *partition, int32_t nparts,
                              int32_t nev, const amsp_options *opt, int32_t *region_ptr,
                              int32_t *region_dofs, int64_t cap, int64_t *ntiles,
                              int64_t *npairs);

/* Device self-test of the matrix-core operand layout the kernels rely on:
 * D (16x16) = A (16x4) B (4x16) computed by one v_mfma_f64_16x16x4f64,
 * all three row-major host arrays.  Uses the default stream; blocks. */
amsp_status amsp_selftest_mfma(const double *a_host, const double *b_host, double *d_host);

void amsp_destroy(amsp_handle *h);
/* Returns the process-wide caches to the system: device blocks kept for
 * later setups (freed with hipFree on their own device), page-locked
 * planner blocks and the planner workers' index maps (at most 1 GiB, kept
 * between setups); stops and joins the planner's worker threads.  Blocks
 * still owned by live handles are untouched.  Later calls re-create the
 * caches on demand.  Must not run concurrently with any other call.  The
 * library also does this from an exit handler that runs before the HIP
 * runtime's own teardown. */
void amsp_release_caches(void);
const char *amsp_status_string(amsp_status s);
const char *amsp_last_error(const amsp_handle *h);
/* Message of the last failed amsp_setup in this thread (no handle exists). */
const char *amsp_setup_error(void);

#ifdef __cplusplus
}
#endif
#endif /* AMSP_H */
