/*
 * sstep.h -- C ABI of the MI355X (gfx950) s-step CG library.
 *
 * The library solves a sparse symmetric positive definite system A x = b with
 * the s-step conjugate-gradient outer iteration of S. Thomas and P. D'Ambra,
 * "Inexact Gauss-Seidel Coarse Solvers for AMG and s-step CG"
 * (arXiv:2512.09642), Sec. 2:
 *   1. r = b - A x, stop when ||r|| < tol ||r_0||            (Sec. 8, stopping rule)
 *   2. Chebyshev basis P = [p_0 .. p_{s-1}] of K_s(M^{-1}A, r)  (Sec. 2, Definition)
 *      by the three-term recurrence, keeping the products A P
 *   3. Gram system G = P^T (A P), c = P^T r as block reductions (Sec. 1, Sec. 2)
 *   4. column scaling d_i = (p_i^T A p_i)^{-1/2}, G <- S G S   (Sec. 2, column scaling)
 *      and nu forward Gauss-Seidel sweeps from alpha = 0      (Sec. 2, FGS iteration)
 *   5. x <- x + P alpha                                       (Sec. 2)
 * Every step runs in hand-written HIP kernels.  graph_chunk outer iterations
 * are captured in one HIP graph; the stopping test runs on the device right
 * after the residual kernel and, once it fires, every later kernel returns at
 * once.
 * The host synchronises once per graph replay: it waits for the copy of the
 * device's stop flag that follows replay r (replay r + 1 already queued
 * behind it) before deciding whether to queue replay r + 2.
 *
 * Conventions for every function below:
 *   - Vector arguments (b, x, g, lam, dA, P_out, AP_out, y) are DEVICE pointers
 *     to FP64 arrays on the GPU that was current at sstep_setup.  The matrix
 *     arrays of sstep_operator are host or device pointers (ptr_space).
 *   - Work is ordered after all work previously enqueued on options.stream
 *     (NULL = the legacy default stream) and the call returns after the
 *     library's own stream has finished, so outputs are ready on return.
 *   - Nothing allocates device memory after sstep_setup /
 *     sstep_setup_batched.
 *   - A context is used by one host thread at a time.
 *   - Errors are returned as sstep_status; sstep_last_error() gives a message.
 *     No exception crosses the ABI.
 */
#ifndef SSTEP_H
#define SSTEP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sstep_ctx sstep_ctx; /* opaque, library-owned */

typedef enum {
    SSTEP_OK = 0,
    SSTEP_E_ARG = 1,         /* invalid argument (sizes, bounds, pointers, malformed CSR, diagonal <= 0) */
    SSTEP_E_HIP = 2,         /* a HIP runtime call failed */
    SSTEP_E_NOMEM = 3,       /* device or pinned host allocation failed */
    SSTEP_E_BREAKDOWN = 4,   /* a basis column has p^T A p <= 0 or non-finite: scaling undefined */
    SSTEP_E_NOCONV = 5,      /* max_outer outer iterations without reaching tol */
    SSTEP_E_NONFINITE = 6,   /* the residual norm became NaN or Inf */
    SSTEP_E_UNSUPPORTED = 7  /* valid request the library does not provide */
} sstep_status;

typedef enum {
    SSTEP_OP_CSR = 0,       /* general sparse SPD matrix, CSR */
    SSTEP_OP_STENCIL7 = 1,  /* matrix-free 7-point operator on a 3D grid */
    SSTEP_OP_STENCIL27 = 2  /* matrix-free 27-point operator on a 3D grid (Sec. 8) */
} sstep_op_kind;

typedef enum {
    SSTEP_FP64 = 0,    /* every step in FP64 */
    SSTEP_FP32_IR = 1  /* basis, SpMV and Gram in FP32 with FP32 accumulation; residual, scaling,
                          FGS and x update in FP64 (one FP64 refinement per outer iteration) */
} sstep_precision;

/* Sparse SPD operator.
 *  CSR (kind = SSTEP_OP_CSR): n rows, nnz entries, 0-based int32 row_ptr[n+1]
 *     and col_idx[nnz] (columns strictly ascending within a row), FP64 val[nnz].
 *  Stencil (kind = SSTEP_OP_STENCIL7): interior grid nx x ny x nz, unknown
 *     (i,j,k) at i + nx*(j + ny*k) (x fastest), homogeneous Dirichlet boundary.
 *     (A u)_p = sum over the six faces f of p of k_f (u_p - u_q), u_q = 0 outside
 *     the grid, with face coefficients (boundary faces included, x fastest)
 *        kx[(k*ny + j)*(nx+1) + i]   face between cells i-1 and i,
 *        ky[(k*(ny+1) + j)*nx + i],  kz[(k*ny + j)*nx + i].
 *     kx = ky = kz = NULL selects the constant Poisson operator (every k_f = 1:
 *     diagonal 6, off-diagonal -1).  n and nnz are ignored.
 *  27-point stencil (kind = SSTEP_OP_STENCIL27): the Poisson operator of the
 *     paper's experiments (Sec. 8), interior grid nx x ny x nz numbered as
 *     above, homogeneous Dirichlet boundary: (A u)_p = 26 u_p - sum of u over
 *     the 26 other points of the 3 x 3 x 3 box around p (u = 0 outside), i.e.
 *     A = 27 I - T_x (x) T_y (x) T_z with T = tridiag(1, 1, 1).  Constant
 *     coefficients: kx, ky, kz must be NULL; n and nnz are ignored.
 *  ptr_space: 0 = the arrays are host memory, 1 = device memory.  They are
 *  copied into library memory; the caller may free them on return. */
typedef struct {
    int32_t kind;
    int32_t ptr_space;
    int64_t n, nnz;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
    int32_t nx, ny, nz;
    const double *kx, *ky, *kz;
} sstep_operator;

/* Gram formation.  STORED_AP: the basis steps write A p_j to an n x s array
 * AP and the Gram kernel reads P and AP.  APPLY_OP (stencil operators,
 * s <= 16, a basis column under 4 GiB, i.e. n < 2^29 in FP64): the Gram
 * kernel forms A p_j from P itself, so AP is neither written nor allocated
 * and the basis makes s - 1 launches per outer iteration; asking for it
 * otherwise gives SSTEP_E_UNSUPPORTED.  RECURRENCE (any operator, s <= 31):
 * the basis makes s launches, the last one computing p_s instead of A p_{s-1},
 * and the Gram kernel forms the M-weighted Gram H = P^T M P of the s + 1
 * columns p_0 .. p_s; the basis recurrence (Sec. 2, Definition) turns it into
 * G_raw = P^T A P exactly: M^{-1} A p_j = (p_{j+1} + p_{j-1}) / (2 theta)
 * + sigma p_j (j >= 1), M^{-1} A p_0 = p_1 / theta + sigma p_0 (monomial
 * basis: M^{-1} A p_j = p_{j+1}).  AP is neither written nor allocated and A
 * is not applied in the Gram kernel.  MOMENTS (FP64, Chebyshev basis,
 * s <= 31, p_0 = M^{-1} r or no preconditioner; batched contexts with an even
 * s and two basis steps per launch): as
 * RECURRENCE, but no kernel reads the basis back.  While the basis kernels
 * form p_i, they sum d_i = <p_i, M p_i> and e_i = <p_i, M p_{i-1}>
 * (fixed-order block partials).  With X = theta (M^{-1} A - sigma I),
 * p_i = T_i(X) p_0 and M X symmetric, the product rule
 * T_i T_j = (T_{i+j} + T_{|i-j|}) / 2 gives
 * H_ij = (mu_{i+j} + mu_{|i-j|}) / 2 with mu_0 = d_0, mu_1 = e_1,
 * mu_2i = 2 d_i - mu_0, mu_{2i-1} = 2 e_i - mu_1, and c_i = <p_i, r> = mu_i.
 * The FGS kernel forms H and then G_raw as for RECURRENCE.  Equal to the
 * directly formed Gram matrix up to rounding; asking for it otherwise gives
 * SSTEP_E_UNSUPPORTED. */
typedef enum {
    SSTEP_GRAM_AUTO = 0,
    SSTEP_GRAM_STORED_AP = 1,
    SSTEP_GRAM_APPLY_OP = 2,
    SSTEP_GRAM_RECURRENCE = 3,
    SSTEP_GRAM_MOMENTS = 4
} sstep_gram_kind;

typedef struct {
    int32_t precision;      /* sstep_precision, default SSTEP_FP64 */
    int32_t precond;        /* 1 = Jacobi M = diag(A) (default), 0 = none */
    int32_t p0_mode;        /* 0 = p_0 = M^{-1} r (default), 1 = p_0 = r as printed in Sec. 2 */
    int32_t max_outer;      /* outer-iteration limit, default 10000 */
    int32_t graph_chunk;    /* outer iterations per graph replay, default 4 */
    int32_t record_history; /* 1 = keep per-iteration relative residual and delta on the device */
    int32_t autotune;       /* 1 (default) = at setup, time the Gram kernel's schedules (blocks, row
                               slabs) on the context's buffers and keep the fastest, cached in
                               $SSTEP_TUNE_CACHE or ~/.cache/sstep/tune.json; systems under 2^20
                               unknowns use the defaults; 0 = defaults */
    int32_t gram;           /* sstep_gram_kind: how G = P^T A P (Sec. 2) is formed.  SSTEP_GRAM_AUTO
                               (default) = SSTEP_GRAM_MOMENTS where it applies (FP64), else
                               SSTEP_GRAM_RECURRENCE for s <= 31 (FP32+IR, p_0 = r with Jacobi,
                               the monomial basis, the allocation-free solve), SSTEP_GRAM_STORED_AP
                               at s = 32.  Batched contexts take AUTO (= MOMENTS where it applies,
                               else RECURRENCE for s <= 31), MOMENTS, RECURRENCE or STORED_AP
                               (SSTEP_E_UNSUPPORTED for APPLY_OP) */
    int32_t basis;          /* 0 = Chebyshev basis (default, Sec. 2); 1 = monomial basis
                               p_{j+1} = M^{-1} A p_j of the same Krylov space, the comparison of
                               Sec. 4 (a diagnostic: its Gram matrix is badly conditioned; the
                               bounds are then unused; not for batched contexts) */
    int32_t basis_steps;    /* 0 (default) = two basis steps per launch where the kernels allow it
                               (constant 7-point operator, or batched stencil systems, when AP is
                               not stored); 1 = one step per launch everywhere.  Both give the
                               same basis bit for bit */
    void *stream;           /* hipStream_t the caller's data is ordered on (NULL = default) */
} sstep_options;

typedef struct {
    int32_t outer_iters;  /* completed outer updates */
    int32_t status;       /* sstep_status of the solve */
    double rel_res;       /* ||b - A x|| / ||b - A x_0|| of the returned x */
    double res0;          /* ||b - A x_0|| */
    double *hist_relres;  /* (host, optional) relative residual for k = 0..outer_iters */
    double *hist_delta;   /* (host, optional) ||ctil - G atil|| / ||ctil|| per update (Sec. 7) */
    int32_t hist_cap;     /* capacity of each history array (0 = none) */
    double *hist_lnorm;   /* (host, optional) ||L||_F per update, L the strictly lower part of the
                             scaled Gram matrix G = I + L + L^T (Sec. 4) */
} sstep_stats;

/* Fills *opt with the defaults listed above. */
void sstep_default_options(sstep_options *opt);

/* Creates a context for operator A, basis width s in [1, 32], nu >= 1 FGS sweeps
 * (Sec. 2), and Chebyshev bounds 0 <= lambda_min < lambda_max enclosing the
 * spectrum of M^{-1} A (Sec. 2, Definition).  Copies A to the device,
 * allocates every workspace (basis P and, unless the Gram kernel forms the
 * products itself, AP: n x s each, column-major,
 * partial sums, device state) and captures the outer-iteration graph.
 * opt may be NULL (defaults).  Returns SSTEP_E_ARG for invalid sizes, bounds,
 * a malformed CSR pattern or, with Jacobi, a non-positive diagonal. */
sstep_status sstep_setup(sstep_ctx **out, const sstep_operator *A, int32_t s, int32_t nu,
                         double lambda_min, double lambda_max, const sstep_options *opt);

/* Replaces the coefficients of the operator (same kind, same sizes, same CSR
 * pattern): val for CSR, kx/ky/kz for stencils. */
sstep_status sstep_update_coefficients(sstep_ctx *ctx, const sstep_operator *A);

/* y = A x (FP64). x and y: n doubles, distinct. */
sstep_status sstep_apply(sstep_ctx *ctx, const double *x, double *y);

/* Solves A x = b.  x holds the initial guess on entry and the result on exit.
 * Stops at the first k with ||b - A x_k|| < tol ||b - A x_0|| (tol in (0, 1));
 * returns immediately if ||b - A x_0|| = 0.  On SSTEP_E_NOCONV, _BREAKDOWN or
 * _NONFINITE, x holds the last completed iterate.  st may be NULL. */
sstep_status sstep_solve(sstep_ctx *ctx, const double *b, double *x, double tol, sstep_stats *st);

/* Adjoint solve A^T lam = g.  A is symmetric, so this is the same s-step
 * iteration applied to g; lam holds the initial guess on entry. */
sstep_status sstep_solve_adjoint(sstep_ctx *ctx, const double *g, double *lam, double tol, sstep_stats *st);

/* Gradient of a loss through x = A^{-1} b with respect to the operator's
 * coefficients, given x and the adjoint solution lam: dL/dA = -lam x^T, i.e.
 *   CSR:      dA[k] = -lam_i x_j for stored entry k = (i, j)        (nnz values)
 *   stencil:  interior face f between p and q: -(lam_p - lam_q)(x_p - x_q),
 *             boundary face of p: -lam_p x_p; dA = [dkx | dky | dkz] concatenated
 *             ((nx+1)ny nz + nx(ny+1)nz + nx ny(nz+1) values, layouts as in
 *             sstep_operator; also for the constant Poisson operator, whose faces are 1).
 * accumulate = 1 adds to dA instead of overwriting it. */
sstep_status sstep_grad_operator(sstep_ctx *ctx, const double *lam, const double *x, double *dA, int32_t accumulate);

/* Number of values sstep_grad_operator writes (0 for the 27-point operator,
 * which has no coefficients: sstep_grad_operator gives SSTEP_E_UNSUPPORTED). */
int64_t sstep_grad_size(const sstep_ctx *ctx);

/* Number of unknowns n. */
int64_t sstep_n(const sstep_ctx *ctx);

/* ONE outer iteration from x (no stopping test, no graph): x <- x + P alpha.
 * Host outputs (each may be NULL): alpha_tilde[s] (scaled FGS solution),
 * G[s*s] (scaled Gram matrix, row-major), ctil[s] (scaled right-hand side),
 * rnorm[1] (||b - A x|| before the update).  Device outputs (may be NULL):
 * P_out, AP_out: n x s FP64 column-major (leading dimension n).  When AP is
 * not kept (SSTEP_GRAM_APPLY_OP), AP_out is formed by the basis kernels' product
 * step into a buffer allocated on the first such call.  Used by the lockstep
 * parity tests. */
sstep_status sstep_step(sstep_ctx *ctx, const double *b, double *x, double *alpha_tilde, double *G, double *ctil,
                        double *rnorm, double *P_out, double *AP_out);

/* Lanczos estimate of the spectrum of M^{-1}A, the interval the Chebyshev
 * basis needs (Sec. 2, Definition: [lambda_min, lambda_max] must enclose it;
 * Sec. 8, setup: a few Lanczos steps give the extreme eigenvalues).  M^{-1}A
 * is self-adjoint in the M-inner product, so the recurrence runs on
 * M-orthonormal vectors from the start vector u (device, n doubles, not
 * modified):
 *   z_0 = u / ||u||_M;  alpha_j = z_j^T A z_j;
 *   w = M^{-1} A z_j - alpha_j z_j - beta_j z_{j-1};  beta_{j+1} = ||w||_M;
 *   z_{j+1} = w / beta_{j+1}
 * for up to steps in [1, 64] steps, no reorthogonalisation, stopping early
 * when beta_{j+1} <= 1e-13 max |alpha_i| or is not finite (m steps done).
 * The Ritz values are the eigenvalues of T_m = tridiag(beta; alpha; beta),
 * computed on the device by bisection.  Host outputs (each may be NULL),
 * steps entries each, zero beyond m: alpha, beta (beta[i] = beta_{i+1}, below
 * row i of T_m), ritz (ascending); m_out = m.  Runs on the context's stream;
 * the vectors use the basis storage P when it holds 3n doubles (P is scratch
 * between solves), otherwise 3n doubles allocated on the first call and kept
 * until sstep_destroy.  SSTEP_E_ARG for a zero start vector. */
sstep_status sstep_lanczos(sstep_ctx *ctx, const double *u, int32_t steps, double *alpha, double *beta,
                           double *ritz, int32_t *m_out);

/* Replaces the Chebyshev bounds 0 <= lambda_min < lambda_max of the context
 * (the outer-iteration graph is captured again). */
sstep_status sstep_set_bounds(sstep_ctx *ctx, double lambda_min, double lambda_max);

/* sstep_lanczos from u, then the bounds with a relative safety margin in
 * [0, 1) (Sec. 8: 10%): lambda_min = max(0, (1 - margin) theta_min),
 * lambda_max = (1 + margin) theta_max for the extreme Ritz values, set on the
 * context as by sstep_set_bounds and returned (host, may be NULL). */
sstep_status sstep_lanczos_bounds(sstep_ctx *ctx, const double *u, int32_t steps, double margin,
                                  double *lambda_min, double *lambda_max);

/* Diagnostics of the last outer iteration of the last sstep_step or solve on
 * ctx (host outputs, each may be NULL): rnorm = ||b - A x_k|| of its residual,
 * delta = ||ctil - G atil|| / ||ctil|| of its Gram solve (Sec. 7), lnorm =
 * ||L||_F of its scaled Gram matrix G = I + L + L^T (Sec. 4).  After a solve
 * that stopped, rnorm is the final residual and delta, lnorm belong to the
 * last update. */
sstep_status sstep_last_iteration(sstep_ctx *ctx, double *rnorm, double *delta, double *lnorm);

/* Kernel classes timed by sstep_kernel_times, in this order. */
enum { SSTEP_KT_RESIDUAL = 0, SSTEP_KT_BASIS = 1, SSTEP_KT_GRAM = 2, SSTEP_KT_FGS = 3, SSTEP_KT_UPDATE = 4,
       SSTEP_KT_COUNT = 5 };

/* Average duration in milliseconds of one launch of each kernel class of the
 * outer iteration (the same kernels, grids and arguments a solve uses),
 * measured with HIP events on the library stream over reps repetitions of
 * the class; the basis figure is the average over the launches of one basis
 * (sstep_basis_launches of them).  b is read; x is used as scratch and
 * overwritten. */
sstep_status sstep_kernel_times(sstep_ctx *ctx, const double *b, double *x, int32_t reps, double *ms_out);

/* The sstep_gram_kind a context uses (SSTEP_GRAM_STORED_AP,
 * SSTEP_GRAM_APPLY_OP or SSTEP_GRAM_RECURRENCE), batched contexts included;
 * -1 for a NULL context. */
int32_t sstep_gram_mode(const sstep_ctx *ctx);

/* Kernel launches that form the basis p_1 .. p_m of one outer iteration
 * (Sec. 2, Definition; m = s - 1 with SSTEP_GRAM_APPLY_OP, else s).  With
 * basis_steps = 0, for the constant 7-point operator with the Chebyshev basis
 * and AP not stored, and for batched stencil systems with the recurrence Gram
 * kind, one launch forms two consecutive columns (p_{j+1} and p_{j+2} from
 * p_{j-1} and p_j, exactly as two single steps would), and *pairs (if pairs
 * is not NULL) receives how many launches do so; an odd m ends with a single
 * step.  Otherwise every launch forms one column and *pairs is 0.  A batched
 * context takes two steps per launch only when every system's grid row fits
 * a third of a 1024-thread block (or its whole plane fits one block).
 * Returns -1 for a NULL context. */
int32_t sstep_basis_launches(const sstep_ctx *ctx, int32_t *pairs);

/* Batched solves: nsys independent operators (each its own size), nrhs
 * right-hand sides per operator, one shared s and nu, per-system bounds
 * lmin[q] < lmax[q] (host arrays).  The outer iteration of every
 * (system, rhs) pair advances together: each step of it (residual, the basis
 * steps, Gram, FGS, update) is one launch over all pairs, at most s + 4
 * launches per outer iteration (fewer when basis launches form two columns,
 * see sstep_basis_launches), graph_chunk outer iterations per graph replay; a
 * pair that has stopped is skipped by every launch. */
sstep_status sstep_setup_batched(sstep_ctx **out, int32_t nsys, const sstep_operator *A, int32_t nrhs, int32_t s,
                                 int32_t nu, const double *lmin, const double *lmax, const sstep_options *opt);

/* The tile schedule a batched context runs (chosen by the autotuner at set-up,
 * or the defaults): rows per chunk tile of the residual, Gram and update
 * launches, and the persistent grid in blocks per compute unit (host outputs,
 * each may be NULL).  SSTEP_E_ARG for a NULL or non-batched context. */
sstep_status sstep_batched_tiles(const sstep_ctx *ctx, int64_t *rows_per_tile, int32_t *grid_factor);

/* The bands a batched context's two-step basis launches run over (host
 * outputs, each may be NULL): *bands, the blocks per right-hand side of the
 * band table chosen for the whole batch (z-ranges as long as still give four
 * blocks per compute unit; 0 when every basis launch forms one column);
 * *tail_bands, those of a second table with ranges of 16 planes, which a
 * solve switches to once the pairs still running would start fewer than four
 * blocks per compute unit from the first table (0 when the two tables are the
 * same); *tail_replays, the graph replays of the last sstep_solve_batched that
 * ran on the second table.  The basis columns do not depend on the table; the
 * moments Gram kind sums its per-band partials in a different order.
 * SSTEP_E_ARG for a NULL or non-batched context. */
sstep_status sstep_batched_bands(const sstep_ctx *ctx, int32_t *bands, int32_t *tail_bands, int32_t *tail_replays);

/* b[q], x[q] (host arrays of nsys device pointers): n_q x nrhs FP64,
 * column-major (right-hand side r at offset r*n_q).  st: host array of
 * nsys*nrhs entries (pair (q, r) at q*nrhs + r), may be NULL.  Returns the
 * first non-OK pair status, or SSTEP_OK. */
sstep_status sstep_solve_batched(sstep_ctx *ctx, const double *const *b, double *const *x, double tol,
                                 sstep_stats *st);

/* Coarse-grid solve of a two-level hierarchy (Sec. 6, Proposition "AMG
 * Convergence" and the streaming remark; Sec. 8, "AMG and performance"):
 * Af is a 7-point stencil operator (constant or face coefficients) on a fine
 * grid of (2 ncx + 1) x (2 ncy + 1) x (2 ncz + 1) points; P is the trilinear
 * prolongation from the ncx x ncy x ncz coarse grid (coarse point (I, J, K) on
 * fine point (2I+1, 2J+1, 2K+1), hat weights 1, 1/2 per axis); the coarse
 * operator is A_c = P^T Af P.  formed = 0: A_c is never formed (streamed:
 * each Gauss-Seidel update forms p_j^T Af (P u) on the fly from the fine
 * coefficients; the library keeps a_jj, a wavefront table and the fine
 * vector P u); formed = 1: the 27 entries of each row of A_c are formed on
 * the device at setup.  SSTEP_E_ARG for even fine sides. */
sstep_status sstep_coarse_setup(sstep_ctx **out, const sstep_operator *Af, int32_t formed, const sstep_options *opt);

/* u = nu forward Gauss-Seidel sweeps on A_c u = f from u = 0, unknowns in
 * natural order (x fastest), each update u_j = (f_j - sum_{i != j} a_ji u_i)
 * / a_jj with the updated values of the lower-numbered unknowns (Sec. 6: nu =
 * 10-30 sweeps; Sec. 8: nu_coarse = 20).  f, u: device, n_c doubles each.
 * The sweep runs in wavefronts I + 2J + 4K, which gives exactly the
 * sequential order's values. */
sstep_status sstep_coarse_fgs(sstep_ctx *ctx, const double *f, double *u, int32_t nu);

/* Number of coarse unknowns and the library's device workspace in bytes for
 * the context's variant (streamed or formed; the fine coefficients
 * excluded). */
sstep_status sstep_coarse_info(const sstep_ctx *ctx, int64_t *n_coarse, int64_t *workspace_bytes);

/* For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc/hipFree): sstep_setup + sstep_solve +
 * sstep_destroy in one call that allocates nothing.  The whole workspace
 * (basis P, products AP when kept, partial sums, solve state, Jacobi
 * diagonals) lives in one static device array of 64 MiB per GPU, held from
 * the library's first use on that GPU until the process ends; a problem whose
 * workspace does not fit (about 128-256 bytes per unknown at s = 16, so up to
 * some 250k-500k unknowns) gets SSTEP_E_ARG with the sizes in the message.
 * Same arguments and results as sstep_setup / sstep_solve, with these limits:
 * FP64 only (SSTEP_E_UNSUPPORTED otherwise); operator arrays (CSR, face
 * coefficients) must be device memory (ptr_space = 1) and are used in place,
 * the CSR pattern is validated on the device; the Gram schedule is the
 * default one (no autotuning); no history is recorded (st->hist_* ignored);
 * the outer iterations are launched directly on opt->stream, graph_chunk at a
 * time, with a wait for the stop flag after each group, so the call cannot be
 * captured into a graph.  Every call on a GPU uses that GPU's one array:
 * calls that overlap on one GPU (other host threads, other streams) race and
 * give wrong results.  Errors: sstep_last_error(NULL). */
sstep_status sstep_solve_noalloc(const sstep_operator *A, int32_t s, int32_t nu, double lambda_min,
                                 double lambda_max, const sstep_options *opt, const double *b, double *x, double tol,
                                 sstep_stats *st);

const char *sstep_last_error(const sstep_ctx *ctx);
const char *sstep_status_string(sstep_status s);
void sstep_destroy(sstep_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SSTEP_H */
