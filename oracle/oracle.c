/*
 * Plain FP64 CPU oracle of the s-step CG outer iteration with forward
 * Gauss-Seidel (FGS) Gram solves, written from S. Thomas and P. D'Ambra,
 * "Inexact Gauss-Seidel Coarse Solvers for AMG and s-step CG"
 * (arXiv:2512.09642).
 *
 * TEST INFRASTRUCTURE -- NOT PART OF THE PRODUCT.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load this library.  It
 * shares no code, header, table or helper with the HIP library, and it never
 * consumes values produced by the HIP library.
 *
 * Style: plain loops, one step of the method after another in the order the
 * paper states them, FP64 throughout, long reductions (over the n unknowns)
 * with Neumaier compensated summation, built with -O2 -ffp-contract=off and no
 * fast-math.  Nothing is blocked, fused or reordered.
 *
 * Layout: vectors have n entries; an n x s block (the basis P, the products
 * AP) is column-major with leading dimension n (column j at offset j*n); an
 * s x s matrix is row-major.  Sparse matrices are CSR with int32 indices,
 * 0-based, columns strictly ascending within a row.
 *
 * Readings taken where the paper is silent (each is repeated at the place it
 * is used):
 *   - the outer iteration is the memoryless projection the paper writes down
 *     (solve G alpha = P^T r, x += P alpha), without block conjugation;
 *   - the basis starts from p_0 = M^{-1} r (p0_mode 0) or p_0 = r (p0_mode 1);
 *   - the residual r = b - A x is recomputed from x at every outer iteration;
 *   - the Gram matrix is formed from its lower triangle and mirrored, and the
 *     scaled diagonal is set to exactly one;
 *   - every Gram solve starts FGS from alpha = 0 and a sweep visits the
 *     unknowns in ascending order;
 *   - stopping uses the 2-norm of the true residual, strict "<", relative to
 *     the initial residual.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum {
    ORACLE_OK = 0,
    ORACLE_E_ARG = 1,
    ORACLE_E_NOMEM = 3,
    ORACLE_E_BREAKDOWN = 4,
    ORACLE_E_NOCONV = 5,
    ORACLE_E_NONFINITE = 6,
};

/* ---------------------------------------------------------------------------
 * Neumaier compensated summation (improved Kahan-Babuska).
 * ------------------------------------------------------------------------- */
typedef struct {
    double sum;
    double comp;
} nsum_t;

static void nsum_add(nsum_t *a, double v)
{
    double t = a->sum + v;
    if (fabs(a->sum) >= fabs(v))
        a->comp += (a->sum - t) + v;
    else
        a->comp += (v - t) + a->sum;
    a->sum = t;
}

static double nsum_value(const nsum_t *a) { return a->sum + a->comp; }

/* Compensated dot product sum_m u[m] * v[m].  The timing build with OpenMP
 * (oracle/build.py, CPU baseline only) sums contiguous per-thread ranges with
 * the same compensated sum and combines the per-thread sums and corrections in
 * thread order; the reference build used by the tests is sequential. */
double oracle_dot(int64_t n, const double *u, const double *v)
{
#ifdef _OPENMP
    if (n >= 65536 && omp_get_max_threads() > 1) {
        double sums[512], comps[512];
        int used = 1;
        const int nt = omp_get_max_threads() < 512 ? omp_get_max_threads() : 512;
#pragma omp parallel num_threads(nt)
        {
            const int t = omp_get_thread_num(), T = omp_get_num_threads();
            const int64_t lo = n * t / T, hi = n * (t + 1) / T;
            nsum_t a = {0.0, 0.0};
            for (int64_t m = lo; m < hi; ++m)
                nsum_add(&a, u[m] * v[m]);
            sums[t] = a.sum;
            comps[t] = a.comp;
            if (t == 0)
                used = T;
        }
        nsum_t acc = {0.0, 0.0};
        for (int t = 0; t < used; ++t) {
            nsum_add(&acc, sums[t]);
            nsum_add(&acc, comps[t]);
        }
        return nsum_value(&acc);
    }
#endif
    nsum_t acc = {0.0, 0.0};
    for (int64_t m = 0; m < n; ++m)
        nsum_add(&acc, u[m] * v[m]);
    return nsum_value(&acc);
}

/* ---------------------------------------------------------------------------
 * Sparse operator (Sec. 2: A is sparse SPD).
 * ------------------------------------------------------------------------- */

/* 0 if (row_ptr, col_idx) is a well-formed CSR pattern of an n x n matrix
 * with strictly ascending columns, 1 otherwise. */
int oracle_csr_validate(int64_t n, const int32_t *row_ptr, const int32_t *col_idx)
{
    if (n < 1 || !row_ptr || !col_idx || row_ptr[0] != 0)
        return 1;
    for (int64_t i = 0; i < n; ++i) {
        if (row_ptr[i + 1] < row_ptr[i])
            return 1;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            if (col_idx[k] < 0 || col_idx[k] >= n)
                return 1;
            if (k > row_ptr[i] && col_idx[k] <= col_idx[k - 1])
                return 1;
        }
    }
    return 0;
}

/* y = A x, each row summed left to right in stored (ascending column) order. */
void oracle_spmv(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                 const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            acc += val[k] * x[col_idx[k]];
        y[i] = acc;
    }
}

/* Number of stored entries of the 7-point operator on an nx x ny x nz grid. */
int64_t oracle_stencil7_nnz(int32_t nx, int32_t ny, int32_t nz)
{
    int64_t n = (int64_t)nx * ny * nz;
    return n + 2 * ((int64_t)(nx - 1) * ny * nz + (int64_t)nx * (ny - 1) * nz + (int64_t)nx * ny * (nz - 1));
}

/* Assemble the 7-point Dirichlet operator of an nx x ny x nz interior grid
 * (x fastest) as CSR.  Face coefficients kx[(k*ny + j)*(nx+1) + i] (face
 * between cells i-1 and i), ky[(k*(ny+1) + j)*nx + i], kz[(k*ny + j)*nx + i]
 * with boundary faces included; A_pp is the sum of the six faces of p (taken in
 * the order west, east, south, north, bottom, top) and A_pq = -k_f.  All three
 * pointers NULL selects the constant Poisson operator (every k_f = 1, so
 * diagonal 6 and off-diagonal -1).  Returns nnz; the caller sizes the arrays
 * with oracle_stencil7_nnz. */
int64_t oracle_assemble_stencil7(int32_t nx, int32_t ny, int32_t nz, const double *kx, const double *ky,
                                 const double *kz, int32_t *row_ptr, int32_t *col_idx, double *val)
{
    const int64_t nxy = (int64_t)nx * ny;
    int64_t nnz = 0;
    row_ptr[0] = 0;
    for (int32_t k = 0; k < nz; ++k)
        for (int32_t j = 0; j < ny; ++j)
            for (int32_t i = 0; i < nx; ++i) {
                const int64_t p = i + nx * ((int64_t)j + (int64_t)ny * k);
                double fw = 1.0, fe = 1.0, fs = 1.0, fn = 1.0, fb = 1.0, ft = 1.0;
                if (kx) {
                    fw = kx[((int64_t)k * ny + j) * (nx + 1) + i];
                    fe = kx[((int64_t)k * ny + j) * (nx + 1) + i + 1];
                    fs = ky[((int64_t)k * (ny + 1) + j) * nx + i];
                    fn = ky[((int64_t)k * (ny + 1) + j + 1) * nx + i];
                    fb = kz[((int64_t)k * ny + j) * nx + i];
                    ft = kz[((int64_t)(k + 1) * ny + j) * nx + i];
                }
                const double diag = ((((fw + fe) + fs) + fn) + fb) + ft;
                if (k > 0) { col_idx[nnz] = (int32_t)(p - nxy); val[nnz++] = -fb; }
                if (j > 0) { col_idx[nnz] = (int32_t)(p - nx); val[nnz++] = -fs; }
                if (i > 0) { col_idx[nnz] = (int32_t)(p - 1); val[nnz++] = -fw; }
                col_idx[nnz] = (int32_t)p; val[nnz++] = diag;
                if (i < nx - 1) { col_idx[nnz] = (int32_t)(p + 1); val[nnz++] = -fe; }
                if (j < ny - 1) { col_idx[nnz] = (int32_t)(p + nx); val[nnz++] = -fn; }
                if (k < nz - 1) { col_idx[nnz] = (int32_t)(p + nxy); val[nnz++] = -ft; }
                row_ptr[p + 1] = (int32_t)nnz;
            }
    return nnz;
}

/* Number of stored entries of the 27-point operator on an nx x ny x nz grid:
 * every point couples to the in-grid points of its 3 x 3 x 3 box. */
int64_t oracle_stencil27_nnz(int32_t nx, int32_t ny, int32_t nz)
{
    /* per axis, the number of (point, offset in {-1, 0, 1}) pairs in the grid */
    const int64_t px = 3 * (int64_t)nx - 2, py = 3 * (int64_t)ny - 2, pz = 3 * (int64_t)nz - 2;
    return px * py * pz;
}

/* Assemble the 27-point Dirichlet operator of an nx x ny x nz interior grid
 * (x fastest) as CSR: A = 27 I - (T_x (x) T_y (x) T_z) with T = tridiag(1, 1, 1)
 * on each axis, i.e. diagonal 26 and -1 for each of the 26 neighbours of the
 * 3 x 3 x 3 box that lie in the grid (Sec. 8: a 27-point finite-difference
 * Poisson operator on the unit cube; this is the stencil with those
 * coefficients).  Columns ascending.  Returns nnz; size the arrays with
 * oracle_stencil27_nnz. */
int64_t oracle_assemble_stencil27(int32_t nx, int32_t ny, int32_t nz, int32_t *row_ptr, int32_t *col_idx,
                                  double *val)
{
    int64_t nnz = 0;
    row_ptr[0] = 0;
    for (int32_t k = 0; k < nz; ++k)
        for (int32_t j = 0; j < ny; ++j)
            for (int32_t i = 0; i < nx; ++i) {
                const int64_t p = i + nx * ((int64_t)j + (int64_t)ny * k);
                for (int dk = -1; dk <= 1; ++dk)
                    for (int dj = -1; dj <= 1; ++dj)
                        for (int di = -1; di <= 1; ++di) {
                            const int32_t a = i + di, b = j + dj, c = k + dk;
                            if (a < 0 || a >= nx || b < 0 || b >= ny || c < 0 || c >= nz)
                                continue;
                            col_idx[nnz] = (int32_t)(a + nx * ((int64_t)b + (int64_t)ny * c));
                            val[nnz++] = (di == 0 && dj == 0 && dk == 0) ? 26.0 : -1.0;
                        }
                row_ptr[p + 1] = (int32_t)nnz;
            }
    return nnz;
}

/* Preconditioner M (Sec. 2): Jacobi M = diag(A) when precond = 1, identity
 * when precond = 0.  Writes invd = M^{-1} diagonal and dvec = M diagonal.
 * Returns ORACLE_E_ARG if a diagonal entry is missing or not positive. */
int oracle_jacobi(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val, int precond,
                  double *invd, double *dvec)
{
    for (int64_t i = 0; i < n; ++i) {
        double aii = 0.0;
        int found = 0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col_idx[k] == i) {
                aii = val[k];
                found = 1;
            }
        if (!found || !(aii > 0.0) || !isfinite(aii))
            return ORACLE_E_ARG;
        if (precond) {
            invd[i] = 1.0 / aii;
            if (dvec)
                dvec[i] = aii;
        } else {
            invd[i] = 1.0;
            if (dvec)
                dvec[i] = 1.0;
        }
    }
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------------
 * Chebyshev basis (Sec. 2, Definition "Chebyshev Polynomial Basis"):
 *   theta = 2 / (lmax - lmin), sigma = (lmax + lmin) / 2,
 *   p_1     = theta (M^{-1}A - sigma I) p_0,
 *   p_{j+1} = 2 theta (M^{-1}A - sigma I) p_j - p_{j-1},  j >= 1.
 * Column 0 of P must already hold p_0.  AP[:, j] = A p_j for j = 0..s-1 (the
 * products the recurrence needs are kept, and the last one is formed as well,
 * since the Gram matrix needs A p_{s-1}).  y is n doubles of scratch.
 * ------------------------------------------------------------------------- */
void oracle_chebyshev_basis(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                            const double *invd, int s, double theta, double sigma, double *P, double *AP)
{
    for (int j = 0; j < s; ++j) {
        const double *pj = P + (int64_t)j * n;
        double *y = AP + (int64_t)j * n;
        oracle_spmv(n, row_ptr, col_idx, val, pj, y); /* y = A p_j */
        if (j + 1 >= s)
            break;
        double *pnext = P + (int64_t)(j + 1) * n;
        if (j == 0) {
#pragma omp parallel for schedule(static)
            for (int64_t m = 0; m < n; ++m)
                pnext[m] = theta * (invd[m] * y[m] - sigma * pj[m]);
        } else {
            const double *pprev = P + (int64_t)(j - 1) * n;
            const double two_theta = 2.0 * theta;
#pragma omp parallel for schedule(static)
            for (int64_t m = 0; m < n; ++m)
                pnext[m] = two_theta * (invd[m] * y[m] - sigma * pj[m]) - pprev[m];
        }
    }
}

/* Monomial basis of the same Krylov space (the comparison of Sec. 4):
 *   p_{j+1} = M^{-1} A p_j,
 * with AP[:, j] = A p_j for j = 0..s-1 as above.  Column 0 of P must hold p_0. */
void oracle_monomial_basis(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                           const double *invd, int s, double *P, double *AP)
{
    for (int j = 0; j < s; ++j) {
        const double *pj = P + (int64_t)j * n;
        double *y = AP + (int64_t)j * n;
        oracle_spmv(n, row_ptr, col_idx, val, pj, y); /* y = A p_j */
        if (j + 1 >= s)
            break;
        double *pnext = P + (int64_t)(j + 1) * n;
#pragma omp parallel for schedule(static)
        for (int64_t m = 0; m < n; ++m)
            pnext[m] = invd[m] * y[m];
    }
}

/* ---------------------------------------------------------------------------
 * Gram system (Sec. 1 and Sec. 2): G_raw = P^T (A P) and c = P^T r.
 * The lower triangle i >= j is summed and mirrored, so G_raw is exactly
 * symmetric.  Graw is s x s row-major.
 * ------------------------------------------------------------------------- */
void oracle_gram(int64_t n, int s, const double *P, const double *AP, const double *r, double *Graw, double *c)
{
    for (int i = 0; i < s; ++i) {
        for (int j = 0; j <= i; ++j) {
            const double g = oracle_dot(n, P + (int64_t)i * n, AP + (int64_t)j * n);
            Graw[i * s + j] = g;
            Graw[j * s + i] = g;
        }
        c[i] = oracle_dot(n, P + (int64_t)i * n, r);
    }
}

/* Column scaling (Sec. 2, "Column scaling", after Ruhe): d_i = (p_i^T A p_i)^{-1/2},
 * G = S G_raw S with S = diag(d), so diag(G) = I (set to exactly 1), and the
 * scaled right-hand side ctil = S c = P~^T r.  Returns ORACLE_E_BREAKDOWN if a
 * diagonal entry of G_raw is not positive or not finite. */
int oracle_column_scale(int s, const double *Graw, const double *c, double *G, double *ctil, double *d)
{
    for (int i = 0; i < s; ++i) {
        const double gii = Graw[i * s + i];
        if (!(gii > 0.0) || !isfinite(gii))
            return ORACLE_E_BREAKDOWN;
        d[i] = 1.0 / sqrt(gii);
    }
    for (int i = 0; i < s; ++i) {
        G[i * s + i] = 1.0;
        for (int j = 0; j < i; ++j) {
            /* scaled from the lower triangle and mirrored: G stays exactly symmetric */
            const double g = (d[i] * Graw[i * s + j]) * d[j];
            G[i * s + j] = g;
            G[j * s + i] = g;
        }
        ctil[i] = d[i] * c[i];
    }
    return ORACLE_OK;
}

/* Forward Gauss-Seidel on G a = ctil with G = I + L + L^T (Sec. 2, FGS
 * iteration; Sec. 3): start from a = 0 and run nu sweeps; a sweep visits
 * j = 0..s-1 in ascending order and sets
 *     a_j = ctil_j - sum_{i != j} G_ji a_i
 * using the already-updated a_i for i < j (the forward substitution with I+L)
 * and the previous sweep's a_i for i > j (the L^T term). */
void oracle_fgs(int s, const double *G, const double *ctil, int nu, double *a)
{
    for (int j = 0; j < s; ++j)
        a[j] = 0.0;
    for (int sweep = 0; sweep < nu; ++sweep)
        for (int j = 0; j < s; ++j) {
            double acc = ctil[j];
            for (int i = 0; i < s; ++i)
                if (i != j)
                    acc -= G[j * s + i] * a[i];
            a[j] = acc;
        }
}

/* ---------------------------------------------------------------------------
 * One outer iteration (Sec. 2: build P on K_s(M^{-1}A, r), solve
 * G alpha = P^T r with nu FGS sweeps in the scaled basis, x += P alpha).
 * ------------------------------------------------------------------------- */
typedef struct {
    int64_t n;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
    const double *invd;
    int s, nu, p0_mode, basis; /* basis: 0 Chebyshev, 1 monomial */
    double theta, sigma;
    double *P, *AP, *r; /* n*s, n*s, n */
} oracle_ws;

/* r = b - A x and its 2-norm (compensated sum of squares). */
static double residual(const oracle_ws *w, const double *b, const double *x, double *r)
{
    oracle_spmv(w->n, w->row_ptr, w->col_idx, w->val, x, r);
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < w->n; ++m)
        r[m] = b[m] - r[m];
    return sqrt(oracle_dot(w->n, r, r));
}

/* Basis, Gram, scaling, FGS and update for residual w->r of iterate x (in
 * place: x becomes x + P alpha).  Optional outputs may be NULL. */
static int outer_update(const oracle_ws *w, double *x, double *atil_out, double *G_out, double *ctil_out,
                        double *Graw_out, double *d_out, double *delta_out, double *lnorm_out)
{
    const int64_t n = w->n;
    const int s = w->s;
    double Graw[64 * 64], G[64 * 64], c[64], ctil[64], d[64], atil[64], alpha[64];

    /* p_0 = M^{-1} r (p0_mode 0) or r (p0_mode 1) */
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < n; ++m)
        w->P[m] = w->p0_mode ? w->r[m] : w->invd[m] * w->r[m];
    if (w->basis == 1)
        oracle_monomial_basis(n, w->row_ptr, w->col_idx, w->val, w->invd, s, w->P, w->AP);
    else
        oracle_chebyshev_basis(n, w->row_ptr, w->col_idx, w->val, w->invd, s, w->theta, w->sigma, w->P, w->AP);
    oracle_gram(n, s, w->P, w->AP, w->r, Graw, c);
    const int st = oracle_column_scale(s, Graw, c, G, ctil, d);
    if (Graw_out)
        memcpy(Graw_out, Graw, sizeof(double) * s * s);
    if (st != ORACLE_OK)
        return st;
    oracle_fgs(s, G, ctil, w->nu, atil);

    /* alpha = S atil (coefficients of the unscaled basis), x += P alpha */
    for (int i = 0; i < s; ++i)
        alpha[i] = d[i] * atil[i];
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < n; ++m) {
        double acc = 0.0;
        for (int i = 0; i < s; ++i)
            acc += w->P[(int64_t)i * n + m] * alpha[i];
        x[m] += acc;
    }

    if (atil_out)
        memcpy(atil_out, atil, sizeof(double) * s);
    if (G_out)
        memcpy(G_out, G, sizeof(double) * s * s);
    if (ctil_out)
        memcpy(ctil_out, ctil, sizeof(double) * s);
    if (d_out)
        memcpy(d_out, d, sizeof(double) * s);
    if (delta_out) {
        /* relative Gram-solve residual || ctil - G atil || / || ctil || (Sec. 7) */
        double num = 0.0, den = 0.0;
        for (int i = 0; i < s; ++i) {
            double ri = ctil[i];
            for (int j = 0; j < s; ++j)
                ri -= G[i * s + j] * atil[j];
            num += ri * ri;
            den += ctil[i] * ctil[i];
        }
        *delta_out = den > 0.0 ? sqrt(num / den) : 0.0;
    }
    if (lnorm_out) {
        /* ||L||_F of the strictly lower part of G (Sec. 4) */
        double acc = 0.0;
        for (int i = 0; i < s; ++i)
            for (int j = 0; j < i; ++j)
                acc += G[i * s + j] * G[i * s + j];
        *lnorm_out = sqrt(acc);
    }
    return ORACLE_OK;
}

static int check_common(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val, int s,
                        int nu, double lmin, double lmax)
{
    if (n < 1 || !row_ptr || !col_idx || !val)
        return ORACLE_E_ARG;
    if (s < 1 || s > 64 || nu < 1)
        return ORACLE_E_ARG;
    if (!isfinite(lmin) || !isfinite(lmax) || lmin < 0.0 || !(lmax > lmin))
        return ORACLE_E_ARG;
    if (oracle_csr_validate(n, row_ptr, col_idx))
        return ORACLE_E_ARG;
    return ORACLE_OK;
}

static int ws_init(oracle_ws *w, int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                   int s, int nu, double lmin, double lmax, int precond, int p0_mode, int basis, double **invd_store)
{
    memset(w, 0, sizeof(*w));
    w->n = n;
    w->row_ptr = row_ptr;
    w->col_idx = col_idx;
    w->val = val;
    w->s = s;
    w->nu = nu;
    w->p0_mode = p0_mode;
    w->basis = basis;
    w->theta = 2.0 / (lmax - lmin);
    w->sigma = (lmax + lmin) / 2.0;
    double *invd = (double *)malloc(sizeof(double) * n);
    w->P = (double *)malloc(sizeof(double) * n * s);
    w->AP = (double *)malloc(sizeof(double) * n * s);
    w->r = (double *)malloc(sizeof(double) * n);
    *invd_store = invd;
    if (!invd || !w->P || !w->AP || !w->r)
        return ORACLE_E_NOMEM;
    const int st = oracle_jacobi(n, row_ptr, col_idx, val, precond, invd, NULL);
    w->invd = invd;
    return st;
}

static void ws_free(oracle_ws *w, double *invd)
{
    free(invd);
    free(w->P);
    free(w->AP);
    free(w->r);
}

/* One outer iteration from x_k (no stopping test): xnext = x_k + P alpha.
 * Outputs: atil (s), G (s*s scaled), ctil (s), Graw (s*s), d (s), rnorm
 * (||b - A x_k||), delta (the Gram-solve residual of Sec. 7), lnorm (||L||_F
 * of Sec. 4), and optionally the basis P and AP (n*s each, column-major); any
 * output pointer may be NULL. */
int oracle_sstep_step(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                      const double *b, const double *xk, double *xnext, int s, int nu, double lmin, double lmax,
                      int precond, int p0_mode, int basis, double *atil, double *G, double *ctil, double *Graw,
                      double *d,
                      double *rnorm, double *delta, double *lnorm, double *P_out, double *AP_out)
{
    int st = check_common(n, row_ptr, col_idx, val, s, nu, lmin, lmax);
    if (st != ORACLE_OK || !b || !xk || !xnext || (basis != 0 && basis != 1))
        return st != ORACLE_OK ? st : ORACLE_E_ARG;
    oracle_ws w;
    double *invd = NULL;
    st = ws_init(&w, n, row_ptr, col_idx, val, s, nu, lmin, lmax, precond, p0_mode, basis, &invd);
    if (st == ORACLE_OK) {
        const double rho = residual(&w, b, xk, w.r);
        if (rnorm)
            *rnorm = rho;
        if (xnext != xk)
            memcpy(xnext, xk, sizeof(double) * n);
        st = outer_update(&w, xnext, atil, G, ctil, Graw, d, delta, lnorm);
        if (P_out)
            memcpy(P_out, w.P, sizeof(double) * n * s);
        if (AP_out)
            memcpy(AP_out, w.AP, sizeof(double) * n * s);
    }
    ws_free(&w, invd);
    return st;
}

/* s-step CG solve of A x = b from the initial guess in x (overwritten).
 * For k = 0, 1, ...: r_k = b - A x_k; stop with k iterations when
 * ||r_k|| < tol ||r_0|| (Sec. 8 stopping rule, strict) -- immediately when
 * ||r_0|| = 0; fail with ORACLE_E_NOCONV when k reaches max_outer; otherwise do
 * one outer update.  hist_* (capacity hist_cap, may be NULL) receive
 * ||r_k||/||r_0|| for k = 0..iters and, per update, delta_k (Sec. 7) and
 * ||L||_F (Sec. 4).  On an error x holds the last completed iterate. */
int oracle_sstep_solve(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                       const double *b, double *x, int s, int nu, double lmin, double lmax, double tol,
                       int max_outer, int precond, int p0_mode, int basis, int *iters, double *relres, double *res0,
                       double *hist_relres, double *hist_delta, double *hist_lnorm, int hist_cap)
{
    int st = check_common(n, row_ptr, col_idx, val, s, nu, lmin, lmax);
    if (st != ORACLE_OK)
        return st;
    if (!b || !x || !(tol > 0.0) || !(tol < 1.0) || max_outer < 0 || (basis != 0 && basis != 1))
        return ORACLE_E_ARG;
    oracle_ws w;
    double *invd = NULL;
    st = ws_init(&w, n, row_ptr, col_idx, val, s, nu, lmin, lmax, precond, p0_mode, basis, &invd);
    double rho0 = 0.0;
    int k = 0;
    if (iters)
        *iters = 0;
    if (relres)
        *relres = 0.0;
    for (; st == ORACLE_OK; ++k) {
        const double rho = residual(&w, b, x, w.r);
        if (k == 0) {
            rho0 = rho;
            if (res0)
                *res0 = rho0;
            if (rho0 == 0.0)
                break;
        }
        if (!isfinite(rho)) {
            st = ORACLE_E_NONFINITE;
            break;
        }
        if (relres)
            *relres = rho / rho0;
        if (hist_relres && k < hist_cap)
            hist_relres[k] = rho / rho0;
        if (rho < tol * rho0)
            break;
        if (k == max_outer) {
            st = ORACLE_E_NOCONV;
            break;
        }
        double delta = 0.0, lnorm = 0.0;
        st = outer_update(&w, x, NULL, NULL, NULL, NULL, NULL, &delta, &lnorm);
        if (st != ORACLE_OK)
            break;
        if (hist_delta && k < hist_cap)
            hist_delta[k] = delta;
        if (hist_lnorm && k < hist_cap)
            hist_lnorm[k] = lnorm;
    }
    if (iters)
        *iters = k;
    ws_free(&w, invd);
    return st;
}

/* ---------------------------------------------------------------------------
 * Gradient of a loss L(x) through x = A^{-1} b, given the adjoint
 * lam = A^{-T} dL/dx = A^{-1} dL/dx (A symmetric): dL/dA = -lam x^T, hence
 *   CSR entry (i, j):   -lam_i x_j;
 *   face f between p and q (A_pp += k_f, A_qq += k_f, A_pq = A_qp -= k_f):
 *                       -(lam_p - lam_q)(x_p - x_q);
 *   boundary face of p: -lam_p x_p.
 * ------------------------------------------------------------------------- */
void oracle_grad_csr(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *lam,
                     const double *x, double *dval)
{
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            dval[k] = -lam[i] * x[col_idx[k]];
}

void oracle_grad_faces(int32_t nx, int32_t ny, int32_t nz, const double *lam, const double *x, double *dkx,
                       double *dky, double *dkz)
{
    const int64_t nxy = (int64_t)nx * ny;
    for (int32_t k = 0; k < nz; ++k)
        for (int32_t j = 0; j < ny; ++j)
            for (int32_t i = 0; i <= nx; ++i) {
                const int64_t p = i + nx * ((int64_t)j + (int64_t)ny * k); /* cell east of the face */
                double g;
                if (i == 0)
                    g = -lam[p] * x[p];
                else if (i == nx)
                    g = -lam[p - 1] * x[p - 1];
                else
                    g = -(lam[p - 1] - lam[p]) * (x[p - 1] - x[p]);
                dkx[((int64_t)k * ny + j) * (nx + 1) + i] = g;
            }
    for (int32_t k = 0; k < nz; ++k)
        for (int32_t j = 0; j <= ny; ++j)
            for (int32_t i = 0; i < nx; ++i) {
                const int64_t p = i + nx * ((int64_t)j + (int64_t)ny * k);
                double g;
                if (j == 0)
                    g = -lam[p] * x[p];
                else if (j == ny)
                    g = -lam[p - nx] * x[p - nx];
                else
                    g = -(lam[p - nx] - lam[p]) * (x[p - nx] - x[p]);
                dky[((int64_t)k * (ny + 1) + j) * nx + i] = g;
            }
    for (int32_t k = 0; k <= nz; ++k)
        for (int32_t j = 0; j < ny; ++j)
            for (int32_t i = 0; i < nx; ++i) {
                const int64_t p = i + nx * ((int64_t)j + (int64_t)ny * k);
                double g;
                if (k == 0)
                    g = -lam[p] * x[p];
                else if (k == nz)
                    g = -lam[p - nxy] * x[p - nxy];
                else
                    g = -(lam[p - nxy] - lam[p]) * (x[p - nxy] - x[p]);
                dkz[((int64_t)k * ny + j) * nx + i] = g;
            }
}

/* ---------------------------------------------------------------------------
 * Spectrum bounds for the Chebyshev basis by Lanczos (Sec. 8, setup of the
 * experiments: a few Lanczos steps give the extreme eigenvalues of M^{-1}A,
 * widened by a safety margin).
 *
 * M^{-1}A is self-adjoint in the M-inner product <u, v>_M = u^T M v, so the
 * Lanczos recurrence runs on M-orthonormal vectors z_j:
 *     z_0     = u / ||u||_M,                    beta_0 = 0, z_{-1} = 0,
 *     y       = A z_j,            alpha_j = z_j^T y  (= <z_j, M^{-1}A z_j>_M),
 *     w       = M^{-1} y - alpha_j z_j - beta_j z_{j-1},
 *     beta_{j+1} = ||w||_M,       z_{j+1} = w / beta_{j+1}.
 * T_m = tridiag(beta_1..beta_{m-1}; alpha_0..alpha_{m-1}; beta_1..beta_{m-1})
 * is the projection of M^{-1}A on the Krylov space; its eigenvalues (Ritz
 * values) approximate the spectrum from inside.  No reorthogonalisation.
 * The recurrence stops early (m = j + 1) when beta_{j+1} is not above
 * 1e-13 max_{i <= j} |alpha_i| (an invariant subspace, to rounding) or not
 * finite.  Writes alpha[0..m), beta[0..m) (beta[i] = beta_{i+1}, the
 * off-diagonal below row i; beta[m-1] is the value that stopped it or the
 * last one), returns m (0 for invalid arguments or a zero start vector).
 * ------------------------------------------------------------------------- */
int oracle_lanczos(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val, int precond,
                   const double *u, int steps, double *alpha, double *beta)
{
    if (n < 1 || !u || steps < 1 || !alpha || !beta)
        return 0;
    double *invd = (double *)malloc(sizeof(double) * n);
    double *dvec = (double *)malloc(sizeof(double) * n);
    double *zprev = (double *)calloc((size_t)n, sizeof(double));
    double *z = (double *)malloc(sizeof(double) * n);
    double *y = (double *)malloc(sizeof(double) * n);
    int m = 0;
    if (!invd || !dvec || !zprev || !z || !y)
        goto out;
    if (oracle_jacobi(n, row_ptr, col_idx, val, precond, invd, dvec) != ORACLE_OK)
        goto out;
    {
        /* z_0 = u / ||u||_M */
        nsum_t acc = {0.0, 0.0};
        for (int64_t i = 0; i < n; ++i)
            nsum_add(&acc, dvec[i] * u[i] * u[i]);
        const double un = sqrt(nsum_value(&acc));
        if (!(un > 0.0) || !isfinite(un))
            goto out;
        for (int64_t i = 0; i < n; ++i)
            z[i] = u[i] / un;
    }
    double bj = 0.0, amax = 0.0;
    for (int j = 0; j < steps; ++j) {
        oracle_spmv(n, row_ptr, col_idx, val, z, y); /* y = A z_j */
        const double aj = oracle_dot(n, z, y);
        alpha[j] = aj;
        if (fabs(aj) > amax)
            amax = fabs(aj);
        nsum_t acc = {0.0, 0.0};
        for (int64_t i = 0; i < n; ++i) {
            y[i] = invd[i] * y[i] - aj * z[i] - bj * zprev[i]; /* w */
            nsum_add(&acc, dvec[i] * y[i] * y[i]);
        }
        const double bn = sqrt(nsum_value(&acc));
        beta[j] = bn;
        m = j + 1;
        if (!(bn > 1e-13 * amax) || !isfinite(bn))
            break;
        for (int64_t i = 0; i < n; ++i) {
            zprev[i] = z[i];
            z[i] = y[i] / bn;
        }
        bj = bn;
    }
out:
    free(invd);
    free(dvec);
    free(zprev);
    free(z);
    free(y);
    return m;
}

/* ---------------------------------------------------------------------------
 * Coarse-grid solve of a two-level hierarchy (Sec. 6; Sec. 8, "AMG and
 * performance"): A_c = P^T A_f P with a geometric prolongation P, solved by
 * nu forward Gauss-Seidel sweeps from zero.
 * ------------------------------------------------------------------------- */

/* Trilinear prolongation from an ncx x ncy x ncz coarse grid to the fine grid
 * of (2 ncx + 1) x (2 ncy + 1) x (2 ncz + 1) points (both x fastest, zero
 * Dirichlet boundary): coarse point (I, J, K) sits on fine point
 * (2I+1, 2J+1, 2K+1), and its basis function is the product over the axes of
 * the 1D hat 1, 1/2, 0 at fine distance 0, 1, >= 2.  Writes P as CSR
 * (n_f rows, up to 8 entries per row, columns ascending); sizes: row_ptr
 * n_f + 1, col_idx and val 27 n_c.  Returns nnz. */
int64_t oracle_prolongation_trilinear(int32_t ncx, int32_t ncy, int32_t ncz, int32_t *row_ptr, int32_t *col_idx,
                                      double *val)
{
    const int32_t nx = 2 * ncx + 1, ny = 2 * ncy + 1, nz = 2 * ncz + 1;
    int64_t nnz = 0;
    row_ptr[0] = 0;
    for (int32_t z = 0; z < nz; ++z)
        for (int32_t y = 0; y < ny; ++y)
            for (int32_t x = 0; x < nx; ++x) {
                const int64_t row = x + (int64_t)nx * (y + (int64_t)ny * z);
                /* coarse parents per axis: odd fine index 2I+1 -> I (weight 1);
                   even fine index 2I -> I-1 and I (weight 1/2 each, when inside) */
                int32_t pk[2], pj[2], pi[2];
                double wk[2], wj[2], wi[2];
                int nk = 0, nj = 0, ni = 0;
                if (z % 2) { pk[nk] = (z - 1) / 2; wk[nk++] = 1.0; }
                else {
                    if (z / 2 - 1 >= 0) { pk[nk] = z / 2 - 1; wk[nk++] = 0.5; }
                    if (z / 2 < ncz) { pk[nk] = z / 2; wk[nk++] = 0.5; }
                }
                if (y % 2) { pj[nj] = (y - 1) / 2; wj[nj++] = 1.0; }
                else {
                    if (y / 2 - 1 >= 0) { pj[nj] = y / 2 - 1; wj[nj++] = 0.5; }
                    if (y / 2 < ncy) { pj[nj] = y / 2; wj[nj++] = 0.5; }
                }
                if (x % 2) { pi[ni] = (x - 1) / 2; wi[ni++] = 1.0; }
                else {
                    if (x / 2 - 1 >= 0) { pi[ni] = x / 2 - 1; wi[ni++] = 0.5; }
                    if (x / 2 < ncx) { pi[ni] = x / 2; wi[ni++] = 0.5; }
                }
                for (int a = 0; a < nk; ++a)
                    for (int b = 0; b < nj; ++b)
                        for (int c = 0; c < ni; ++c) {
                            col_idx[nnz] = (int32_t)(pi[c] + (int64_t)ncx * (pj[b] + (int64_t)ncy * pk[a]));
                            val[nnz++] = (wk[a] * wj[b]) * wi[c];
                        }
                row_ptr[row + 1] = (int32_t)nnz;
            }
    return nnz;
}

/* nu forward Gauss-Seidel sweeps on A u = f from u = 0, unknowns in ascending
 * order, each update
 *     u_j = (f_j - sum_{i != j} A_ji u_i) / A_jj
 * with the already-updated u_i for i < j (Sec. 6: FGS as the coarse-grid
 * solver, nu = 10-30).  Returns ORACLE_E_ARG if a diagonal entry is missing
 * or not positive. */
int oracle_gs(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val, const double *f, int nu,
              double *u)
{
    if (n < 1 || nu < 0 || !row_ptr || !col_idx || !val || !f || !u)
        return ORACLE_E_ARG;
    for (int64_t j = 0; j < n; ++j)
        u[j] = 0.0;
    for (int sweep = 0; sweep < nu; ++sweep)
        for (int64_t j = 0; j < n; ++j) {
            double acc = f[j], diag = 0.0;
            for (int32_t k = row_ptr[j]; k < row_ptr[j + 1]; ++k) {
                if (col_idx[k] == j)
                    diag = val[k];
                else
                    acc -= val[k] * u[col_idx[k]];
            }
            if (!(diag > 0.0))
                return ORACLE_E_ARG;
            u[j] = acc / diag;
        }
    return ORACLE_OK;
}
