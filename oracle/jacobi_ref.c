/*
 * Plain FP64 CPU oracle for synchronous Jacobi on a CSR matrix.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or constant with the GPU path.
 *
 * Written for obviousness, not speed: every loop follows the definition it
 * cites, summations run in ascending index order starting from 0.0, and the
 * file is built with -ffp-contract=off so that no multiply-add is fused.
 * The optional thread count only splits the independent per-row loops into
 * fixed static chunks; each row is computed the same way whatever the count,
 * and every reduction (norms) is a serial loop in row order, so results are
 * bit-identical for any thread count.
 *
 * Paper references (Cheik Ahamed & Magoules, "On the stability and
 * performance of the solution of sparse linear systems by partitioned
 * procedures"):
 *   - Jacobi splitting M = D, N = -(L+U) (section 3, splitting and
 *     component-form equations);
 *   - correction form u^{k+1} = u^k + D^{-1}(b - A u^k) (section 3, second
 *     Jacobi iteration equation);
 *   - vectorial Jacobi algorithm (section 3, algorithm "Jacobi method:
 *     vectorial version"): D^{-1} computed once, then per iteration
 *     q = A u, r = b - q, norm of r, stop test, update;
 *   - CSR storage AA/JA/IA (section 4.1 and its CSR figure).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum {
    REF_OK = 0,
    REF_NOT_CONVERGED = 1,
    REF_E_INVALID = -1,
    REF_E_ZERO_DIAG = -2,
    REF_E_NOMEM = -3,
    REF_E_DIVERGED = -6
};

enum { REF_NORM_L2_REL = 0, REF_NORM_INF_ABS = 1 };

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Structural checks of a 0-based CSR matrix: row_ptr starts at 0 and never
 * decreases, columns lie in [0,n) and strictly increase within a row, every
 * row holds its diagonal, and that diagonal is nonzero. */
int ref_check_csr(int32_t n, const int32_t *rp, const int32_t *ci, const double *v)
{
    if (n < 0 || rp == NULL || (n > 0 && (ci == NULL || v == NULL))) return REF_E_INVALID;
    if (rp[0] != 0) return REF_E_INVALID;
    for (int32_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return REF_E_INVALID;
        int have_diag = 0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] < 0 || ci[p] >= n) return REF_E_INVALID;
            if (p > rp[i] && ci[p] <= ci[p - 1]) return REF_E_INVALID;
            if (ci[p] == i) {
                have_diag = 1;
                if (v[p] == 0.0) return REF_E_ZERO_DIAG;
            }
        }
        if (!have_diag) return REF_E_ZERO_DIAG;
    }
    return REF_OK;
}

/* D^{-1}: one division per row, done once before the iterations. */
static void inverse_diagonal(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, double *invd)
{
    for (int32_t i = 0; i < n; ++i)
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] == i) invd[i] = 1.0 / v[p];
}

/* r = b - A x, row by row; q_i accumulates a_ij x_j over ascending j from 0. */
static void residual(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                     const double *b, const double *x, double *r)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        double q = 0.0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) q += v[p] * x[ci[p]];
        r[i] = b[i] - q;
    }
}

static double norm2(int32_t n, const double *r)
{
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += r[i] * r[i];
    return sqrt(s);
}

static double norminf(int32_t n, const double *r)
{
    double m = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double a = fabs(r[i]);
        if (a > m || a != a) m = a;
    }
    return m;
}

/* x_new = x + D^{-1} r: every component of the new iterate comes from the old
 * one (synchronous update into a separate buffer). */
static void update(int32_t n, const double *invd, const double *x, const double *r, double *xn)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) xn[i] = x[i] + invd[i] * r[i];
}

/*
 * K fixed sweeps from x0 (NULL = zeros).  hist[k] (if not NULL) receives the
 * 2-norm of r_k = b - A x_k for k = 0..K-1; xout receives x_K.
 */
int ref_sweeps(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, const double *b,
               const double *x0, int32_t K, double *xout, double *hist, int nthreads)
{
    int st = ref_check_csr(n, rp, ci, v);
    if (st != REF_OK) return st;
    if (K < 0) return REF_E_INVALID;
    set_threads(nthreads);
    double *invd = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *x = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *xn = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *r = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!invd || !x || !xn || !r) { free(invd); free(x); free(xn); free(r); return REF_E_NOMEM; }
    inverse_diagonal(n, rp, ci, v, invd);
    for (int32_t i = 0; i < n; ++i) x[i] = x0 ? x0[i] : 0.0;
    for (int32_t k = 0; k < K; ++k) {
        residual(n, rp, ci, v, b, x, r);
        if (hist) hist[k] = norm2(n, r);
        update(n, invd, x, r, xn);
        double *t = x; x = xn; xn = t;
    }
    memcpy(xout, x, sizeof(double) * (size_t)n);
    free(invd); free(x); free(xn); free(r);
    return REF_OK;
}

/*
 * Solve with the vectorial algorithm's stop test.  For k = 0, 1, ...:
 * compute r_k; nrm = ||r_k||_2 (relative mode) or max|r_k,i| (absolute
 * infinity mode); stop when nrm <= tol*||b||_2 (relative; absolute when
 * ||b|| = 0) or nrm <= tol (infinity mode) and return x_k with sweeps = k;
 * when k reaches maxit return x_maxit and REF_NOT_CONVERGED; a non-finite
 * norm or one beyond 1e150*max(||b||,1) returns REF_E_DIVERGED.  Otherwise
 * update.  relres receives nrm/||b||_2 (or nrm when ||b|| = 0, and always
 * nrm in infinity mode) of the returned iterate.
 */
int ref_solve(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, const double *b,
              const double *x0, double tol, int32_t maxit, int normkind, double *xout,
              int32_t *sweeps, double *relres, int nthreads)
{
    int st = ref_check_csr(n, rp, ci, v);
    if (st != REF_OK) return st;
    if (maxit < 0 || !(tol >= 0.0) || (normkind != REF_NORM_L2_REL && normkind != REF_NORM_INF_ABS))
        return REF_E_INVALID;
    set_threads(nthreads);
    double *invd = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *x = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *xn = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *r = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!invd || !x || !xn || !r) { free(invd); free(x); free(xn); free(r); return REF_E_NOMEM; }
    inverse_diagonal(n, rp, ci, v, invd);
    for (int32_t i = 0; i < n; ++i) x[i] = x0 ? x0[i] : 0.0;
    double bn = norm2(n, b);
    double scale = (normkind == REF_NORM_L2_REL && bn > 0.0) ? bn : 1.0;
    double bigref = bn > 1.0 ? bn : 1.0;
    int result = REF_NOT_CONVERGED;
    int32_t k = 0;
    double nrm = 0.0;
    for (k = 0;; ++k) {
        residual(n, rp, ci, v, b, x, r);
        nrm = (normkind == REF_NORM_L2_REL) ? norm2(n, r) : norminf(n, r);
        if (!isfinite(nrm) || nrm > 1e150 * bigref) { result = REF_E_DIVERGED; break; }
        if (nrm <= tol * scale) { result = REF_OK; break; }
        if (k == maxit) { result = REF_NOT_CONVERGED; break; }
        update(n, invd, x, r, xn);
        double *t = x; x = xn; xn = t;
    }
    memcpy(xout, x, sizeof(double) * (size_t)n);
    *sweeps = k;
    *relres = nrm / scale;
    free(invd); free(x); free(xn); free(r);
    return result;
}

/*
 * Reverse-mode derivative of K sweeps from x_0 = 0 with full storage of the
 * iterates x_0..x_K (no checkpointing).
 *
 * One sweep is x_{k+1,i} = x_{k,i} + (b_i - sum_j a_ij x_{k,j}) / a_ii.  With
 * lambda_K = g = dL/dx_K and mu = D^{-1} lambda_{k+1}, the chain rule gives,
 * for k = K-1 down to 0:
 *   dL/db_i    += mu_i
 *   dL/da_ij   -= mu_i * x_{k,j}       (j != i)
 *   dL/da_ii   -= mu_i * x_{k+1,i}     (derivative of both the diagonal term of
 *                                       A x_k and of 1/a_ii)
 *   lambda_k    = lambda_{k+1} - A^T mu
 * A^T mu is formed by scattering each row's entries (a_ij mu_i added into
 * component j).  gb and gvals (CSR entry order) are overwritten.
 */
int ref_adjoint(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, const double *b,
                int32_t K, const double *g, double *gb, double *gvals, double *xK)
{
    int st = ref_check_csr(n, rp, ci, v);
    if (st != REF_OK) return st;
    if (K < 0) return REF_E_INVALID;
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t nnz = rp[n];
    double *invd = malloc(sizeof(double) * nn);
    double *xs = malloc(sizeof(double) * nn * (size_t)(K + 1));
    double *r = malloc(sizeof(double) * nn);
    double *lam = malloc(sizeof(double) * nn);
    double *lamn = malloc(sizeof(double) * nn);
    double *mu = malloc(sizeof(double) * nn);
    if (!invd || !xs || !r || !lam || !lamn || !mu) {
        free(invd); free(xs); free(r); free(lam); free(lamn); free(mu);
        return REF_E_NOMEM;
    }
    inverse_diagonal(n, rp, ci, v, invd);
    for (int32_t i = 0; i < n; ++i) xs[i] = 0.0;
    for (int32_t k = 0; k < K; ++k) {
        const double *x = xs + (size_t)k * nn;
        double *xn = xs + (size_t)(k + 1) * nn;
        residual(n, rp, ci, v, b, x, r);
        update(n, invd, x, r, xn);
    }
    if (xK) memcpy(xK, xs + (size_t)K * nn, sizeof(double) * (size_t)n);
    for (int32_t i = 0; i < n; ++i) { lam[i] = g[i]; gb[i] = 0.0; }
    for (int32_t p = 0; p < nnz; ++p) gvals[p] = 0.0;
    for (int32_t k = K - 1; k >= 0; --k) {
        const double *x = xs + (size_t)k * nn;
        const double *xn = xs + (size_t)(k + 1) * nn;
        for (int32_t i = 0; i < n; ++i) mu[i] = invd[i] * lam[i];
        for (int32_t i = 0; i < n; ++i) gb[i] += mu[i];
        for (int32_t i = 0; i < n; ++i)
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
                gvals[p] -= mu[i] * (ci[p] == i ? xn[i] : x[ci[p]]);
        for (int32_t i = 0; i < n; ++i) lamn[i] = lam[i];
        for (int32_t i = 0; i < n; ++i)
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p) lamn[ci[p]] -= v[p] * mu[i];
        double *t = lam; lam = lamn; lamn = t;
    }
    free(invd); free(xs); free(r); free(lam); free(lamn); free(mu);
    return REF_OK;
}

/* One sweep's value at the listed rows only: for each i in rows,
 * out[t] = x_i + (1/a_ii) (b_i - sum_j a_ij x_j).  Lets a test check sampled
 * components of a late sweep of a large system without replaying it. */
int ref_sweep_rows(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, const double *b,
                   const double *x, int32_t nrows, const int32_t *rows, double *out, double *res)
{
    for (int32_t t = 0; t < nrows; ++t) {
        int32_t i = rows[t];
        if (i < 0 || i >= n) return REF_E_INVALID;
        double q = 0.0, d = 0.0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            q += v[p] * x[ci[p]];
            if (ci[p] == i) d = v[p];
        }
        if (d == 0.0) return REF_E_ZERO_DIAG;
        double rr = b[i] - q;
        double invd = 1.0 / d;
        if (res) res[t] = rr;
        out[t] = x[i] + invd * rr;
    }
    return REF_OK;
}
