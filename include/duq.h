/*
 * duq.h -- C ABI of libduq.so, an MI355X (gfx950) implementation of the
 * inexact (augmented) dual first-order method DFOM with inner Algorithm FOM
 * (Necoara & Patrascu, "DuQuad: an inexact (augmented) dual first order
 * algorithm for quadratic programming", arXiv 1504.05708).
 *
 * Problem (Sec. 2, eq. original_primal, with K = R^p_-):
 *     min  1/2 u^T Q u + q^T u   s.t.  G u + g <= 0,   lb <= u <= ub
 * Q is n x n symmetric positive definite (or semidefinite with rho > 0,
 * Sec. 2 Case 2), G is p x n, both dense and row-major.
 *
 * Conventions for every entry point:
 *   - Return value: DUQ_OK (0) on success, a negative DUQ_E* code on
 *     failure.  No C++ exception crosses this interface.
 *   - A handle belongs to one host thread at a time.
 *   - "HOST" pointers are read (copied) during the call and may be freed
 *     afterwards.  "DEVICE" pointers are borrowed: they must stay valid and
 *     unchanged until the handle that borrowed them is destroyed.
 *   - Outputs are written to caller-owned host buffers unless stated.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     All device work of a handle runs on that stream; calls that return
 *     results synchronise the stream before returning.
 *   - duq_last_error() returns a thread-local text for the last failure.
 */
#ifndef DUQ_H
#define DUQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define DUQ_OK           0
#define DUQ_EINVAL      -1   /* bad argument: null pointer, n <= 0, p < 0, lb > ub,
                                non-finite data, eps <= 0, rho < 0, rho = 0 with
                                lambda_min(Q) <= 0, unsupported combination      */
#define DUQ_ENOMEM      -2   /* device or host allocation failed                  */
#define DUQ_EDEVICE     -3   /* HIP runtime error or device-side fault flag       */
#define DUQ_EMAXITER    -4   /* max_outer reached; the last iterate is written    */
#define DUQ_ENUMERIC    -5   /* NaN/Inf produced during the iteration             */
#define DUQ_EAGAIN      -6   /* request not finished yet (duq_poll)               */
#define DUQ_ENOTFOUND   -7   /* unknown ticket or id                              */
#define DUQ_EINFEASIBLE -8   /* no point of the box satisfies G u + g <= 0: the
                                multipliers returned are a certificate mu >= 0 with
                                min over the box of mu^T (G u + g) > 0; x is the
                                last iterate (rho = 0)                             */

/* ---- enumerations ------------------------------------------------------ */
enum { DUQ_F64 = 0, DUQ_F32 = 1 };   /* storage of Q, G (FP64 arithmetic on either) */
enum { DUQ_HOST = 0, DUQ_DEVICE = 1 };                        /* memspace          */
enum { DUQ_DGM = 0, DUQ_DFGM = 1 };                           /* outer method, Sec. 3 */
enum { DUQ_LAST = 0, DUQ_AVG = 1 };                           /* primal output, Sec. 4 */
enum { DUQ_CERT = 0, DUQ_FIXED = 1 };                         /* inner stopping rule */
enum { DUQ_INNER_AUTO = 0, DUQ_INNER_GM = 1, DUQ_INNER_FGM = 2,
       DUQ_INNER_FGM_SIGMA = 3 };                             /* inner FOM variant, Sec. 2.1 */
enum { DUQ_ACC_F64 = 0, DUQ_ACC_F32 = 1 };                    /* product accumulation */
enum { DUQ_ENGINE_AUTO = 0, DUQ_ENGINE_BLOCK = 1, DUQ_ENGINE_GRID = 2,
       DUQ_ENGINE_TILE = 3 };   /* TILE: shared batches only, see duq_solve_batch */
enum { DUQ_SPX_AUTO = 0, DUQ_SPX_LDS = 1, DUQ_SPX_IN_PLACE = 2 };  /* options.sparse_x */
enum { DUQ_LB_AUTO = 0, DUQ_LB_SIGMA = 1, DUQ_LB_SIGMA_FREE = 2 };  /* options.lb_cert */

/* ---- problem data (Sec. 2, eq. original_primal) ------------------------- *
 * Constraints: G u + g <= 0 (K = R^p_-) when rlo and rhi are NULL.  With
 * both given, the user form of Sec. 2, rlo <= G u + g <= rhi row by row:
 * rlo_i = rhi_i makes row i an equality (K_i = {0}); otherwise -INFINITY /
 * +INFINITY marks an absent side and each finite side is one inequality
 * (two-sided rows read their row of G once per product).  Multipliers of
 * equality rows are free; the multiplier returned per row is
 * lambda+ - lambda- (positive: the upper side binds).  Row bounds are
 * available on duq_setup / duq_solve (not in batches or the serving loop). */
typedef struct duq_problem {
    int32_t n;            /* variables, n >= 1                                  */
    int32_t p;            /* constraint rows, p >= 0                            */
    int32_t dtype;        /* DUQ_F64 or DUQ_F32: element type of Q and G        */
    int32_t memspace;     /* DUQ_HOST (copied) or DUQ_DEVICE (borrowed)         */
    const void *Q;        /* n x n row-major, symmetric                          */
    const void *G;        /* p x n row-major (may be NULL when p == 0)           */
    const double *q;      /* n                                                   */
    const double *g;      /* p                                                   */
    const double *lb;     /* n, lb <= ub                                         */
    const double *ub;     /* n                                                   */
    const double *rlo;    /* p or NULL: lower row bounds (-INFINITY: none)      */
    const double *rhi;    /* p or NULL: upper row bounds (+INFINITY: none)      */
} duq_problem;

/* ---- solver options ----------------------------------------------------- *
 * Initialise with duq_default_options().  Spectral constants lam_min(Q),
 * lam_max(Q) and ||G||^2 set to a value <= 0 are estimated on the device by
 * an FP64 Lanczos process (k steps), inflated by `safety`.  With row bounds
 * ||G||^2 is that of the rows in cone form (a two-sided row counts twice:
 * lambda_max(G^T W G), W_ii = number of finite sides).  From them:
 *   L_d = ||G||^2/(lam_min + rho ||G||^2)   (Sec. 2 eq. Ld), outer step 1/(2 L_d)
 *   L_in = lam_max + rho ||G||^2, sigma_in = lam_min       (Sec. 3, Step 1)
 *   k_in cap of Sec. 5 (natural log, rounded up) unless max_inner > 0.
 * sigma_in > 0 overrides the strong convexity of the inner problem; when it
 * is <= 0 and every row is an equality with rho > 0 it is lambda_min(Q + rho
 * G^T G) (Sec. 3, Step 1, K = {0}), estimated on the formed matrix.         */
typedef struct duq_options {
    int32_t method;         /* DUQ_DGM | DUQ_DFGM                                */
    int32_t output;         /* DUQ_LAST | DUQ_AVG                                */
    int32_t inner_rule;     /* DUQ_CERT | DUQ_FIXED                              */
    int32_t inner_variant;  /* DUQ_INNER_*                                       */
    int32_t accumulate;     /* DUQ_ACC_F64 | DUQ_ACC_F32 (first phase only)      */
    int32_t engine;         /* DUQ_ENGINE_*                                      */
    int32_t max_outer;      /* outer iteration cap (>= 1)                         */
    int32_t max_inner;      /* inner cap; 0 = k_in of Sec. 5                      */
    int32_t lanczos_steps;  /* Krylov steps for estimated constants (0 = 96)     */
    int32_t trace_outer;    /* record the first trace_outer outer iterations     */
    double eps_out;         /* outer accuracy (relative, see duq_result)         */
    double eps_in;          /* inner accuracy, eq. duquad_in                     */
    double rho;             /* augmented Lagrangian parameter, rho >= 0          */
    double lam_min;         /* lambda_min(Q) or <= 0 to estimate                 */
    double lam_max;         /* lambda_max(Q) or <= 0 to estimate                 */
    double G_norm2;         /* ||G||_2^2 or <= 0 to estimate                     */
    double safety;          /* inflation of estimated constants (default 1.02)   */
    double switch_factor;   /* DUQ_ACC_F32: switch to F64 at switch_factor*eps_out */
    int32_t switch_stall;   /* ... or after this many non-improving iterations   */
    int32_t serve_slice;    /* serving loop: outer iterations per round (0 = 16)  */
    int32_t out_memspace;   /* duq_solve_batch: X_out / Lam_out are DUQ_HOST
                               (default) or DUQ_DEVICE buffers                  */
    int32_t batch_wpc;      /* per-instance batches: workgroups per CU (1..3), or
                               0 = the tuned value (duq_tune_batch) if one is
                               known for the batch's sizes, else the most that fit */
    double sigma_in;        /* strong convexity of L_rho(., mu), or <= 0 (above) */
    int32_t sparse_x;       /* duq_setup_csr: where products read x: DUQ_SPX_AUTO
                               (in place on the grid engine; staged in LDS on
                               the block engine when it fits), DUQ_SPX_LDS,
                               DUQ_SPX_IN_PLACE (device memory)               */
    int32_t lb_cert;        /* inner gap that enters the dual lower bound LB:
                               DUQ_LB_SIGMA (= AUTO): min(FW, ||pi||^2/(2 sigma)),
                               as the stopping test; valid when sigma is at
                               most the true strong convexity (an estimated
                               lambda_min is a Ritz value / safety: a margin,
                               not a bound).  DUQ_LB_SIGMA_FREE: the FW gap (or
                               the gradient-mapping bound without its sigma
                               term), valid for any sigma; linear in the
                               gradient, so LB converges more slowly       */
} duq_options;

/* ---- per-solve result --------------------------------------------------- *
 * The outer test (evaluated on the device every outer iteration) accepts a
 * candidate x (last iterate ubar(lambda^k), eq. last_primal, or the
 * theta-weighted average, eq. average_primal) when
 *    ||[Gx+g]_+|| <= eps_out max(1,||g||),  F(x) - LB <= eps_out max(1,|F(x)|),
 *    ||lambda^k|| ||[Gx+g]_+|| <= eps_out max(1,|F(x)|)
 * with LB a certified lower bound on F* (weak duality minus the inner
 * certificate).                                                              */
typedef struct duq_result {
    int32_t status;         /* DUQ_OK, DUQ_EMAXITER, DUQ_ENUMERIC, DUQ_EINFEASIBLE */
    int32_t outer_iters;
    int64_t inner_iters;    /* total inner FOM steps (products with Q)           */
    int64_t gt_rows;        /* rows of G touched by G^T v products (sparsity)    */
    double f;               /* F(x)                                              */
    double lb_dual;         /* LB                                                */
    double gap;             /* F(x) - LB                                         */
    double feas;            /* ||[Gx+g]_+||_2                                    */
    double time_ms;         /* device time of the solve (hipEvent)               */
    int32_t f64_outer_iters;/* outer iterations run with FP64 accumulation       */
    int32_t engine;         /* engine that ran                                   */
    double lam_min, lam_max, G_norm2;  /* constants used                         */
    double reserved[4];
} duq_result;

typedef struct duq_handle duq_handle;

/* Fill `o` with defaults: DFGM, LAST, CERT, AUTO inner, ACC_F64, eps_out 1e-4,
 * eps_in 1e-6, rho 0, max_outer 100000, constants estimated, safety 1.02.   */
void duq_default_options(duq_options *o);

/* Validate the problem (Sec. 2), move/borrow it to the device, derive the
 * constants (a1) and allocate the workspace.  On success *out owns all
 * device memory of the solve.  Errors: DUQ_EINVAL, DUQ_ENOMEM, DUQ_EDEVICE.
 * Size limit: every workgroup stages the whole iterate x in LDS (FP64), so n
 * is bounded by the LDS of one workgroup less the engine's scratch: on the
 * grid engine n <= 18 234 for 0 < p <= 256 with 160 KiB of LDS (one less per
 * further 256 rows of G); the block engine also holds the p multipliers.  A
 * larger n is DUQ_EINVAL (before any data is read or copied), and
 * duq_last_error() states the exact bound; duq_max_n gives it in advance. */
int duq_setup(const duq_problem *prob, const duq_options *opts, void *stream,
              duq_handle **out);

/* ---- sparse Q and G (Sec. 5.1) ------------------------------------------ *
 * The inner gradient Q u + q + G^T w and the dual gradient G u + g are the
 * bottleneck of both stages (Sec. 5.1); with sparse Q and G they cost their
 * nonzeros instead of n^2 and n p.  A matrix in compressed-row form:       */
typedef struct duq_csr {
    int32_t rows, cols;
    const int64_t *rowptr;  /* rows + 1 offsets: rowptr[0] = 0, nondecreasing    */
    const int32_t *col;     /* rowptr[rows] column indices, each in [0, cols);    */
                            /* any order inside a row; a repeated index adds     */
    const void *val;        /* rowptr[rows] values of the problem's dtype        */
} duq_csr;

/* duq_setup for sparse data: Q (n x n, symmetric, both triangles stored) and
 * G (p x n) in compressed-row form.  prob->Q and prob->G are not read (may be
 * NULL); every array (the CSR arrays included) is host memory and is copied
 * (prob->memspace must be DUQ_HOST); G^T is formed on the host once so that
 * the transposed product gathers along rows.  Everything else is as
 * duq_setup: row bounds, options, constants estimated by Lanczos on the
 * sparse operators, block or grid engine, duq_solve / duq_get_trace /
 * duq_solve_planned on the handle.  Every row an equality with rho > 0: the inner
 * products stay Q u and G^T (G u) (no formed Q + rho G^T G) and the inner
 * strong convexity is lambda_min(Q) unless opts->sigma_in is given.  Each
 * product row is summed by 2^k lanes in a fixed order (k per matrix from its
 * mean row length), so a solve is reproducible run to run.  The products
 * read x from a copy staged in LDS (the LDS bound on n of duq_setup) or,
 * with opts->sparse_x IN_PLACE (AUTO on the grid engine or when the copy
 * does not fit), from device memory, which leaves n bounded by device
 * memory only; the LDS then holds the engine's share of the p rows (block
 * engine: all p).
 * Errors: DUQ_EINVAL (null arrays, shapes other than n x n and p x n,
 * offsets, an index out of range, a non-finite value, memspace),
 * DUQ_ENOMEM, DUQ_EDEVICE.                                                  */
int duq_setup_csr(const duq_problem *prob, const duq_csr *Q, const duq_csr *G,
                  const duq_options *opts, void *stream, duq_handle **out);

/* Largest n that duq_setup accepts for a problem with p rows of G on
 * `engine` (DUQ_ENGINE_BLOCK or DUQ_ENGINE_GRID; AUTO is answered for GRID,
 * which AUTO uses above n = 1536) on the current device; the bound is the
 * LDS of one workgroup, which holds the staged iterate x (Sec. 5.1 products,
 * one double per variable) and the engine's reduction scratch.  Writes
 * *n_max.  Errors: DUQ_EINVAL (null n_max, p < 0, other engine),
 * DUQ_EDEVICE (no device). */
int duq_max_n(int32_t p, int32_t engine, int32_t *n_max);

/* Run Algorithm DFOM (Sec. 3) to the outer test.  x0 (n) warm-starts the
 * inner solver and lam0 (p) the multipliers (both host, may be NULL:
 * x0 = projection of 0 onto the box, lam0 = 0, Sec. 4; lam0 must be NULL
 * with row bounds).  Every row an equality with rho > 0: duq_setup forms
 * Q + rho G^T G once (the constant inner Hessian of Sec. 5.1), so an inner
 * step reads one n x n matrix as with rho = 0.  x_out (n) and
 * lam_out (p) are host buffers (may be NULL).  Returns the result status
 * (DUQ_OK, DUQ_EMAXITER with the last iterate written, DUQ_ENUMERIC,
 * DUQ_EINFEASIBLE with the certificate in lam_out) or an error code.  With
 * rho = 0, before the inner solve of outer iterations k = 1, 9, 17, ... the
 * multipliers mu^k (when all >= 0) are tested as a certificate of
 * infeasibility; the paper assumes a finite
 * optimal multiplier (Sec. 2), i.e. a feasible problem, and this test ends
 * the run early when there is none.                                         */
int duq_solve(duq_handle *h, const double *x0, const double *lam0,
              double *x_out, double *lam_out, duq_result *res);

/* Per-outer-iteration trace of the last duq_solve for the first
 * opts.trace_outer iterations: record k (k = 0..) is
 *   [DUQ_TRACE_SCALARS doubles][lambda^k (p)][mu^k (p)][ubar^k (n)]
 * and with row bounds [..][lambda+ (p)][mu+ (p)][ubar (n)][lambda- (p)][mu- (p)]
 * (sides a row does not have read 0).
 * Scalars: k, t_k, gap_k, dbar_k, LB_k, theta_k, S_k, F(cand), feas(cand),
 * ||lambda^k||, passed, extra_t, extra_gap, F2, feas2, passed2.
 * `out` holds max_records*(DUQ_TRACE_SCALARS+2p+n) doubles (+2p with row
 * bounds); *n_records gets the number written.                              */
#define DUQ_TRACE_SCALARS 16
int duq_get_trace(duq_handle *h, double *out, int32_t max_records, int32_t *n_records);

/* ---- parameter planning (Sec. 3.1 eq. choose_ein, Sec. 5) --------------- *
 * duq_plan_params: for a target accuracy eps of the dual function and
 * R_d = min ||lambda* - lambda^0|| (Sec. 2), the inner accuracy and outer
 * iteration count of eq. choose_ein that make both terms of the rate bound
 * of Theorem lemma_sublin_dfg_inexact at most about eps/2:
 *   DGM:  eps_in = eps/4,                        k_out = ceil(8 L_d R_d^2/eps)
 *   DFGM: eps_in = eps^(3/2)/(8 R_d sqrt(2 L_d)), k_out = ceil(sqrt(8 L_d R_d^2/eps))
 * the penalty rho* = 8 R_d^2/eps of Theorem in:th_last, and (when L_in > 0
 * and D_U > 0 are given) the inner count k_in of Sec. 5 at that eps_in
 * (sigma_in > 0: linear rate, else sublinear) with k_total = k_out k_in.
 * Errors: DUQ_EINVAL (method, eps <= 0, L_d <= 0, R_d <= 0, null out).     */
typedef struct duq_plan {
    double eps_in;
    int64_t k_out;
    double rho_star;
    int64_t k_in;        /* 0 when L_in or D_U was not given */
    int64_t k_total;
} duq_plan;
int duq_plan_params(int32_t method, double eps, double Ld, double Rd, double L_in, double sigma_in,
                    double D_U, duq_plan *out);

/* duq_solve_planned: Algorithm DFOM with eps_in and max_outer planned from a
 * guess R of R_d (the paper leaves a search on R_d open): the outer test runs
 * at eps; when it has not passed after k_out(R) outer iterations the guess
 * doubles and the next round starts from the last x (and lambda, without row
 * bounds).  R0 > 0 is the first guess, max_rounds >= 1 the number of rounds.
 * x_out (n) and lam_out (p) are host buffers (required); res sums the outer
 * and inner iterations of all rounds; *R_out (may be NULL) gets the last
 * guess and *rounds_out (may be NULL) the rounds run.  The handle's options
 * are restored afterwards.  Returns as duq_solve.                          */
int duq_solve_planned(duq_handle *h, double eps, double R0, int32_t max_rounds, double *x_out,
                      double *lam_out, duq_result *res, double *R_out, int32_t *rounds_out);

/* Constants in use: lambda_min(Q), lambda_max(Q), ||G||^2, L_d, L_in, sigma_in. */
int duq_get_constants(duq_handle *h, double *lam_min, double *lam_max,
                      double *G_norm2, double *Ld, double *L_in, double *sigma_in);

/* ---- batches (no batching in the paper; the instances are independent) -- *
 * DUQ_BATCH_UNEVEN: B independent QPs of different sizes, packed.  Instance
 *   i has n[i] variables and p[i] rows; Q_i starts at element qoff[i] of Q
 *   (n_i x n_i row-major), G_i at goff[i] of G (p_i x n_i), q_i / lb_i / ub_i
 *   at voff[i] of q / lb / ub, g_i at coff[i] of g.
 * DUQ_BATCH_SHARED: B QPs sharing Q (n x n), G (p x n), lb, ub; q is B x n
 *   and g is B x p (row b belongs to instance b); voff/coff are unused.
 * HOST data are checked (finite, lb <= ub) and copied; DEVICE data are
 *   borrowed for the call and not scanned (the caller vouches for them).
 * lam_min / lam_max / G_norm2: per-instance constants (B each) or NULL to
 *   estimate them on the device (one value each for SHARED).               */
enum { DUQ_BATCH_UNEVEN = 0, DUQ_BATCH_SHARED = 1 };
typedef struct duq_batch {
    int32_t kind;               /* DUQ_BATCH_UNEVEN | DUQ_BATCH_SHARED            */
    int32_t B;                  /* number of instances, B >= 1                    */
    int32_t dtype;              /* DUQ_F64 | DUQ_F32 storage of Q and G           */
    int32_t memspace;           /* DUQ_HOST (copied) | DUQ_DEVICE (borrowed)      */
    int32_t n_shared, p_shared; /* sizes for DUQ_BATCH_SHARED                     */
    const int32_t *n, *p;       /* B sizes (UNEVEN)                               */
    const int64_t *qoff, *goff, *voff, *coff;   /* element offsets (UNEVEN)      */
    const void *Q, *G;
    const double *q, *g, *lb, *ub;
    const double *lam_min, *lam_max, *G_norm2;  /* optional constants (NULL)      */
} duq_batch;

/* Solve every instance of the batch in one persistent launch: workgroups take
 * work from a device queue and run Algorithm DFOM on each instance with the
 * same options (max_outer, eps and rho apply per instance; tracing is not
 * available).  opts.engine selects the kernel:
 *   DUQ_ENGINE_AUTO   SHARED with rho = 0 and n <= 128: DUQ_ENGINE_TILE;
 *                     otherwise DUQ_ENGINE_BLOCK;
 *   DUQ_ENGINE_BLOCK  one workgroup per instance (largest first), products
 *                     as GEMVs (DUQ_ENGINE_GRID is taken as BLOCK here);
 *   DUQ_ENGINE_TILE   SHARED only: one workgroup per 16 instances in
 *                     lockstep, Q X, G U and G^T M as FP64 MFMA GEMMs with Q
 *                     held in registers (rho = 0, n <= 128).
 * Both accumulate in FP64 and give each instance the iterates it has alone.
 * With opts.out_memspace = DUQ_DEVICE the kernels write X_out / Lam_out
 * (device buffers) directly and nothing crosses PCIe but `res`.  X_out (sum n_i, or B x n) and
 * Lam_out (sum p_i, or B x p) are host buffers laid out like q and g; res has
 * B entries (time_ms is the batch's device time).  Returns DUQ_OK when every
 * instance passed its outer test, DUQ_EMAXITER / DUQ_ENUMERIC /
 * DUQ_EINFEASIBLE when one did not (see res[i].status), or an error code.
 * The device workspace of a call is kept for the next one on the same device
 * (a larger call replaces it, a concurrent call allocates its own); it is
 * held until the process ends.                                              */
int duq_solve_batch(const duq_batch *batch, const duq_options *opts, void *stream,
                    double *X_out, double *Lam_out, duq_result *res);

/* ---- launch-shape tuning for per-instance batches ----------------------- *
 * duq_tune_batch solves an UNEVEN batch (a representative sample of the
 * batches to come) once per candidate launch shape -- 1, 2 and 3 workgroups
 * per CU, as far as they fit -- timing each launch with events on `stream`.
 * The shape only decides how many instances run at once: every candidate
 * must give bitwise the same X, multipliers and counts (checked; DUQ_EDEVICE
 * if not).  The fastest is recorded in a table of this process keyed by
 * (dtype, row class, largest n rounded up to 64) and used by later
 * duq_solve_batch calls whose opts.batch_wpc is 0.  *best_wpc gets it;
 * ms_out (3 doubles, may be NULL) the device time per candidate (0 when a
 * shape does not fit).  duq_tune_save / duq_tune_load write and read the
 * table as text ("dtype short_rows n_bucket wpc" per line).                */
int duq_tune_batch(const duq_batch *batch, const duq_options *opts, void *stream, int32_t *best_wpc,
                   double *ms_out);
int duq_tune_save(const char *path);
int duq_tune_load(const char *path);

/* ---- serving loop (the paper has none; requests are independent QPs) ---- *
 * A server owns a device arena of hbm_budget_bytes (0 = 4 GiB), one HIP
 * stream and one host thread.  The thread works in rounds:
 *   1. admit pending requests in arrival order while their device footprint
 *      (matrices, vectors, solver state) fits the arena, and upload them
 *      (a large request's solver workspace is allocated beside the arena,
 *      its estimated size counted against the budget);
 *   2. run one launch of the batch kernel over every admitted request with
 *      n <= DUQ_SERVE_BATCH_NMAX; each runs a slice of outer iterations
 *      worth about opts.serve_slice iterations at n = 256,
 *      max(1, round(serve_slice (256^2 + 128^2) / (n^2 + 128^2))), and keeps
 *      its whole state (iterates and their products) in the arena for the
 *      next round;
 *   3. run opts.serve_slice outer iterations of the admitted larger request
 *      (one at a time, arrival order) on the single-QP engine (block or
 *      grid, as duq_setup picks);
 *   4. retire requests whose outer test passed (or that reached max_outer or
 *      failed), free their memory, and go back to 1.
 * Slicing changes no arithmetic: a request's iterates are those of the same
 * request solved in one piece (duq_solve_batch for small requests), alone or
 * in any mix.
 * The options (fixed at creation) apply to every request; accumulate must be
 * DUQ_ACC_F64 and tracing is not available.  All server calls are safe to
 * make from several threads.                                               */
#define DUQ_SERVE_BATCH_NMAX 1536
typedef struct duq_server duq_server;

typedef struct duq_request {
    int32_t shared_id;      /* -1: the problem in `prob`; otherwise an id returned
                               by duq_register_shared                           */
    int32_t reserved;
    duq_problem prob;       /* own problem: every field, memspace DUQ_HOST (the
                               data are copied by duq_submit).  Registered system:
                               only prob.q (n) and prob.g (p), host, are read.  */
} duq_request;

/* Create a server.  Errors: DUQ_EINVAL (options), DUQ_ENOMEM (the arena does
 * not fit the free device memory), DUQ_EDEVICE.                            */
int duq_server_create(size_t hbm_budget_bytes, const duq_options *opts, duq_server **out);

/* Keep Q, G, lb, ub of one system resident (HOST copied, DEVICE copied into
 * the arena) for requests that supply only q and g, e.g. an MPC problem
 * whose linear terms follow the measured state.  Its constants come from the
 * options or a device Lanczos estimate made here.  *id receives the id.
 * Errors: DUQ_EINVAL, DUQ_ENOMEM (arena full), DUQ_EDEVICE.               */
int duq_register_shared(duq_server *s, const duq_problem *shared_QG, int32_t *id);

/* Queue one request; *ticket identifies it for duq_poll.  The request data
 * are copied before the call returns.  Errors: DUQ_EINVAL (bad data,
 * unknown shared_id), DUQ_ENOMEM (its footprint exceeds the whole arena),
 * DUQ_EDEVICE (the server stopped after a device error).                   */
int duq_submit(duq_server *s, const duq_request *req, uint64_t *ticket);

/* DUQ_EAGAIN while the request is queued or running.  Once it has finished,
 * writes x_out (n), lam_out (p) and res (any may be NULL; res->time_ms is the
 * latency from duq_submit to completion), forgets the ticket and returns the
 * request's status (DUQ_OK, DUQ_EMAXITER, DUQ_ENUMERIC, DUQ_EINFEASIBLE or an
 * error code).
 * DUQ_ENOTFOUND for a ticket that is unknown or already collected.          */
int duq_poll(duq_server *s, uint64_t ticket, double *x_out, double *lam_out, duq_result *res);

/* Stop the server thread after its current round and free everything;
 * requests not yet collected are dropped (NULL is allowed).                */
void duq_server_destroy(duq_server *s);

/* ---- allocation-free solve ---------------------------------------------- *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * duq_solve_static runs one solve of Algorithm DFOM (as duq_setup + duq_solve
 * would, same kernels and engine choice) on a problem whose data are DEVICE
 * pointers (prob->memspace = DUQ_DEVICE, borrowed for the call), with the
 * spectral constants given in opts (lam_min > 0, or = 0 with rho > 0;
 * lam_max > 0; G_norm2 > 0 when p > 0: no Lanczos estimate runs).  x_out (n)
 * and lam_out (p) are DEVICE buffers.  x0 = projection of 0, lam0 = 0.
 * The workspace lives in a static device array of DUQ_STATIC_SCRATCH_BYTES
 * that each GPU the library runs on holds until the process ends; a problem
 * whose workspace does not fit (about 8 (14 n + 12 p) bytes on one
 * workgroup, plus 8 n bytes per workgroup of the grid engine) is DUQ_EINVAL.
 * The call makes no hipMalloc, hipFree or other allocating call; it clears
 * what must start at zero with a fill kernel, validates the data on the
 * device and synchronises `stream` twice (validation result, final state).
 * Every call on one GPU uses that GPU's one array: calls that overlap in time
 * on the same GPU (other threads, other streams) race and must be
 * serialised by the caller.  Not available: tracing (trace_outer must be 0),
 * the precision switch (accumulate must be DUQ_ACC_F64), warm starts.
 * res->time_ms is 0.  Returns as duq_solve.                                 */
#define DUQ_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int duq_solve_static(const duq_problem *prob, const duq_options *opts, void *stream,
                     double *x_out, double *lam_out, duq_result *res);

/* Release every resource of the handle (NULL is allowed).                  */
void duq_destroy(duq_handle *h);

/* Text of the last error on this thread (never NULL).                       */
const char *duq_last_error(void);
const char *duq_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* DUQ_H */
