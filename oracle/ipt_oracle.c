/*
 * Reference (oracle) implementation of Iterative Perturbation Theory, plain FP64.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct CPU checker
 * that the HIP path is compared against.  It shares no code, header, table or
 * helper with the product library; only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.
 *
 * What it computes (Kenmoe, Kriemann, Smerlak, Zadorin, "A fast iterative
 * algorithm for near-diagonal eigenvalue problems"):
 *   M = D + Delta, theta = diag(D) pairwise distinct (Sec. 3, "partition").
 *   For a requested index i, g_i = (1/(theta_j - theta_i))_{j != i}, (g_i)_i = 0
 *   (Alg. 1, step computing g_i; inverse-gap matrix G_jk = 1/(theta_j - theta_k)).
 *   The map f_i(z) = e_i + g_i o (z (Delta z)_i - Delta z)   (eq. single_line_dyn)
 *   is iterated from z = e_i (or a supplied warm start) while
 *   |z - f_i(z)| / |z| > eta  (Alg. 1 loop test), the eigenvalue is
 *   lambda_i = (M z)_i = theta_i + (Delta z)_i          (Alg. 1 return step).
 *   Applying f_{idx[c]} to every requested column c is exactly the matrix map
 *   F(Z) = I + G o (Z D(Delta Z) - Delta Z) restricted to those columns
 *   (eq. dyn, Alg. 2), because each column is an independent fixed-point problem.
 *
 * Readings taken where the paper is silent (each is listed in the design notes):
 *   - the norm in the stopping test is the Euclidean norm of the column
 *     (per-column relative step s_c);
 *   - the returned eigenvector is the iterate z that passed the test, and
 *     lambda uses (Delta z)_i of that same z (no extra product);
 *   - a column is DIVERGED when any entry of f_i(z) or s is non-finite, when
 *     |f_i(z) - e_i| exceeds div_norm, or when s grew on div_growth consecutive
 *     sweeps; it is NOT_CONVERGED when max_iter sweeps end without a decision.
 *     In both cases the last computed iterate f_i(z) is returned, with lambda from
 *     the (Delta z)_i of that sweep.
 *   - a warm start has its entry i overwritten with 1 (chart z_i = 1).
 *   - non-autonomous continuation: the paper's sequence of scales 1 - alpha^k
 *     starts at k = 0 (scale 0, the identity map); here sweep t uses 1 - alpha^t,
 *     the same iterates one sweep earlier.  The paper leaves the stopping rule
 *     open; here a column certifies only once the scale is exactly 1.
 *
 * Arithmetic: FP64, every dot product summed in ascending index order, compiled
 * with -ffp-contract=off so no fused multiply-add changes the rounding.  OpenMP
 * runs independent columns in parallel; a column's arithmetic does not depend on
 * the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_CONVERGED = 0, OR_NOT_CONVERGED = 1, OR_DIVERGED = 2 };

/* y = Delta z for a dense row-major Delta (leading dimension lda). */
static void dense_apply(int64_t n, const double *delta, int64_t lda, const double *z, double *y) {
    for (int64_t j = 0; j < n; ++j) {
        const double *row = delta + j * lda;
        double acc = 0.0;
        for (int64_t l = 0; l < n; ++l) acc += row[l] * z[l];
        y[j] = acc;
    }
}

/* y = Delta z for a CSR Delta (entries of a row summed in storage order). */
static void csr_apply(int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                      const double *z, double *y) {
    for (int64_t j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int64_t p = row_ptr[j]; p < row_ptr[j + 1]; ++p) acc += val[p] * z[col[p]];
        y[j] = acc;
    }
}

typedef struct {
    int64_t n;
    /* dense */
    const double *delta;
    int64_t lda;
    /* csr */
    const int32_t *row_ptr;
    const int32_t *col;
    const double *val;
} op_t;

static void op_apply(const op_t *A, const double *z, double *y) {
    if (A->delta) dense_apply(A->n, A->delta, A->lda, z, y);
    else csr_apply(A->n, A->row_ptr, A->col, A->val, z, y);
}

/* One application of f_i (eq. single_line_dyn): w = e_i + g o (z d - y), with
 * y = Delta z and d = y_i.  Returns d. */
static double map_once(const op_t *A, const double *theta, int64_t i, const double *g,
                       const double *z, double *y, double *w) {
    const int64_t n = A->n;
    op_apply(A, z, y);
    const double d = y[i];
    for (int64_t j = 0; j < n; ++j) w[j] = (j == i) ? 1.0 : g[j] * (z[j] * d - y[j]);
    (void)theta;
    return d;
}

static void inverse_gaps(int64_t n, const double *theta, int64_t i, double *g) {
    for (int64_t j = 0; j < n; ++j) g[j] = (j == i) ? 0.0 : 1.0 / (theta[j] - theta[i]);
}

/* Alg. 1 for one column.  z (length n) holds the start on entry and the returned
 * vector on exit. */
static void solve_column(const op_t *A, const double *theta, int64_t i, double tol, int max_iter,
                         double div_norm, int div_growth, double *z, double *g, double *y, double *w,
                         double *lambda, int32_t *status, int32_t *sweeps, double *step) {
    const int64_t n = A->n;
    inverse_gaps(n, theta, i, g);
    z[i] = 1.0;
    double prev_s = INFINITY;
    int grow = 0;
    double d = 0.0, s = INFINITY;
    for (int t = 1; t <= max_iter; ++t) {
        d = map_once(A, theta, i, g, z, y, w);
        double num = 0.0, den = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double e = w[j] - z[j];
            num += e * e;
            den += z[j] * z[j];
        }
        s = sqrt(num) / sqrt(den);
        if (s <= tol) {               /* z passed the test: return it */
            *lambda = theta[i] + d;
            *status = OR_CONVERGED;
            *sweeps = t;
            *step = s;
            return;
        }
        int finite = isfinite(s);
        double dist2 = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double e = w[j] - (j == i ? 1.0 : 0.0);
            if (!isfinite(w[j])) finite = 0;
            dist2 += e * e;
        }
        grow = (s > prev_s) ? grow + 1 : 0;
        prev_s = s;
        memcpy(z, w, (size_t)n * sizeof(double));
        if (!finite || !(sqrt(dist2) <= div_norm) || grow >= div_growth) {
            *lambda = theta[i] + d;
            *status = OR_DIVERGED;
            *sweeps = t;
            *step = s;
            return;
        }
    }
    *lambda = theta[i] + d;
    *status = OR_NOT_CONVERGED;
    *sweeps = max_iter;
    *step = s;
}

/* Non-autonomous continuation (concluding discussion of the 3 x 3 example): sweep t
 * applies f_i with the perturbation scaled by 1 - alpha^t, alpha^t formed by
 * repeated multiplication in FP64, so that the scale tends to 1 and reaches it
 * exactly once alpha^t drops below half an ulp of 1.  (The paper counts from a
 * scale of 1 - alpha^0 = 0, the identity map; that sweep is not counted here.)  A
 * column can pass the stopping test only on a sweep whose scale is exactly 1; while
 * the scale is below 1 only the non-finite and div_norm rules apply and the growth
 * count restarts.  lambda = theta_i + (scale Delta z)_i of the last sweep. */
static void solve_column_cont(const op_t *A, const double *theta, int64_t i, double alpha, double tol,
                              int max_iter, double div_norm, int div_growth, double *z, double *g, double *y,
                              double *w, double *lambda, int32_t *status, int32_t *sweeps, double *step) {
    const int64_t n = A->n;
    inverse_gaps(n, theta, i, g);
    z[i] = 1.0;
    double prev_s = INFINITY, apow = 1.0;
    int grow = 0;
    double d = 0.0, s = INFINITY;
    for (int t = 1; t <= max_iter; ++t) {
        apow *= alpha;
        const double scale = 1.0 - apow;
        op_apply(A, z, y);
        for (int64_t j = 0; j < n; ++j) y[j] *= scale; /* (scale Delta) z */
        d = y[i];
        for (int64_t j = 0; j < n; ++j) w[j] = (j == i) ? 1.0 : g[j] * (z[j] * d - y[j]);
        double num = 0.0, den = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double e = w[j] - z[j];
            num += e * e;
            den += z[j] * z[j];
        }
        s = sqrt(num) / sqrt(den);
        if (scale == 1.0 && s <= tol) {
            *lambda = theta[i] + d;
            *status = OR_CONVERGED;
            *sweeps = t;
            *step = s;
            return;
        }
        int finite = isfinite(s);
        double dist2 = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double e = w[j] - (j == i ? 1.0 : 0.0);
            if (!isfinite(w[j])) finite = 0;
            dist2 += e * e;
        }
        if (scale == 1.0) {
            grow = (s > prev_s) ? grow + 1 : 0;
            prev_s = s;
        } else {
            grow = 0;
            prev_s = INFINITY;
        }
        memcpy(z, w, (size_t)n * sizeof(double));
        if (!finite || !(sqrt(dist2) <= div_norm) || grow >= div_growth) {
            *lambda = theta[i] + d;
            *status = OR_DIVERGED;
            *sweeps = t;
            *step = s;
            return;
        }
    }
    *lambda = theta[i] + d;
    *status = OR_NOT_CONVERGED;
    *sweeps = max_iter;
    *step = s;
}

/* IPT-ACX for one column: Alg. 1 with its update replaced by alternating cyclic
 * extrapolation (Alg. 3), orders 3, 2, 3, 2, ...  Each extrapolation cycle of order
 * p takes F(z), ..., F^p(z) and moves to
 *     z + sum_{q=1..p} binom(p, q) sigma^q D^q,
 *     D^q = q-th forward difference (D^1 = F(z) - z, D^2 = F^2(z) - 2F(z) + z,
 *           D^3 = F^3(z) - 3F^2(z) + 3F(z) - z),
 *     sigma = |<D^p, D^(p-1)>| / |D^p|^2.
 * Readings of the printed listing (whose update line omits the leading z term and
 * whose sigma has an unsquared norm): with these, sigma = 1 gives F^p(z) and an
 * affine map x -> r x + b with r < 1 reaches its fixed point in one cycle.  When
 * |D^p| = 0, sigma = 1.  The stopping and divergence tests of Alg. 1 are made on
 * the first application of each cycle (the listing's loop test), with growth
 * counted from cycle to cycle.  max_iter bounds the applications of F: a test at
 * application u whose cycle could not be followed by another test within the
 * budget (u + p > max_iter) ends the column as NOT_CONVERGED with F(z) returned --
 * for p = 1 this is the plain rule u = max_iter.  Returned values otherwise as in
 * solve_column. */
static void solve_column_acx(const op_t *A, const double *theta, int64_t i, double tol, int max_iter,
                             double div_norm, int div_growth, double *z, double *g, double *y, double *f1,
                             double *f2, double *f3, double *lambda, int32_t *status, int32_t *sweeps,
                             double *step) {
    const int64_t n = A->n;
    inverse_gaps(n, theta, i, g);
    z[i] = 1.0;
    double prev_s = INFINITY, s = INFINITY, d = 0.0;
    int grow = 0, used = 0;
    for (int cycle = 0;; ++cycle) {
        const int p = (cycle % 2 == 0) ? 3 : 2;
        d = map_once(A, theta, i, g, z, y, f1);
        ++used;
        double num = 0.0, den = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double e = f1[j] - z[j];
            num += e * e;
            den += z[j] * z[j];
        }
        s = sqrt(num) / sqrt(den);
        if (s <= tol) {
            *lambda = theta[i] + d;
            *status = OR_CONVERGED;
            *sweeps = used;
            *step = s;
            return;
        }
        int finite = isfinite(s);
        double dist2 = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double e = f1[j] - (j == i ? 1.0 : 0.0);
            if (!isfinite(f1[j])) finite = 0;
            dist2 += e * e;
        }
        grow = (s > prev_s) ? grow + 1 : 0;
        prev_s = s;
        const int diverged = !finite || !(sqrt(dist2) <= div_norm) || grow >= div_growth;
        if (diverged || used + p > max_iter) {
            memcpy(z, f1, (size_t)n * sizeof(double));
            *lambda = theta[i] + d;
            *status = diverged ? OR_DIVERGED : OR_NOT_CONVERGED;
            *sweeps = used;
            *step = s;
            return;
        }
        map_once(A, theta, i, g, f1, y, f2);
        ++used;
        if (p == 3) {
            map_once(A, theta, i, g, f2, y, f3);
            ++used;
        }
        /* sigma from the two highest differences, summed in ascending j */
        double dot = 0.0, nrm = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double d1 = f1[j] - z[j];
            const double d2 = (f2[j] - 2.0 * f1[j]) + z[j];
            if (p == 2) {
                dot += d2 * d1;
                nrm += d2 * d2;
            } else {
                const double d3 = ((f3[j] - 3.0 * f2[j]) + 3.0 * f1[j]) - z[j];
                dot += d3 * d2;
                nrm += d3 * d3;
            }
        }
        const double sg = (nrm > 0.0) ? fabs(dot) / nrm : 1.0;
        for (int64_t j = 0; j < n; ++j) {
            const double d1 = f1[j] - z[j];
            const double d2 = (f2[j] - 2.0 * f1[j]) + z[j];
            if (p == 2) {
                z[j] = (z[j] + 2.0 * sg * d1) + (sg * sg) * d2;
            } else {
                const double d3 = ((f3[j] - 3.0 * f2[j]) + 3.0 * f1[j]) - z[j];
                z[j] = ((z[j] + 3.0 * sg * d1) + 3.0 * (sg * sg) * d2) + (sg * sg * sg) * d3;
            }
        }
    }
}

/* rho = |M z - lambda z|_2 / |z|_2 with M z = theta o z + Delta z (plain definition). */
static double eigen_residual(const op_t *A, const double *theta, const double *z, double lambda, double *y) {
    const int64_t n = A->n;
    op_apply(A, z, y);
    double r2 = 0.0, z2 = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        const double r = theta[j] * z[j] + y[j] - lambda * z[j];
        r2 += r * r;
        z2 += z[j] * z[j];
    }
    return sqrt(r2) / sqrt(z2);
}

static int solve_columns(const op_t *A, const double *theta, int64_t k, const int32_t *idx,
                         const double *z0, int64_t ldz0, double tol, int max_iter, double div_norm,
                         int div_growth, double *z_out, int64_t ldz, double *lambda_out, int32_t *status_out,
                         int32_t *sweeps_out, double *step_out, double *resid_out, int acx, double alpha) {
    const int64_t n = A->n;
    int fail = 0;
#pragma omp parallel
    {
        double *buf = (double *)malloc((size_t)n * 6 * sizeof(double));
        if (!buf) {
#pragma omp atomic write
            fail = 1;
        } else {
            double *z = buf, *g = buf + n, *y = buf + 2 * n, *w = buf + 3 * n, *w2 = buf + 4 * n, *w3 = buf + 5 * n;
#pragma omp for schedule(dynamic, 1)
            for (int64_t c = 0; c < k; ++c) {
                const int64_t i = idx ? idx[c] : c;
                for (int64_t j = 0; j < n; ++j) z[j] = z0 ? z0[j * ldz0 + c] : (j == i ? 1.0 : 0.0);
                double lam, st;
                int32_t stat, sw;
                if (alpha > 0.0)
                    solve_column_cont(A, theta, i, alpha, tol, max_iter, div_norm, div_growth, z, g, y, w, &lam,
                                      &stat, &sw, &st);
                else if (acx)
                    solve_column_acx(A, theta, i, tol, max_iter, div_norm, div_growth, z, g, y, w, w2, w3, &lam,
                                     &stat, &sw, &st);
                else
                    solve_column(A, theta, i, tol, max_iter, div_norm, div_growth, z, g, y, w, &lam, &stat, &sw,
                                 &st);
                for (int64_t j = 0; j < n; ++j) z_out[j * ldz + c] = z[j];
                lambda_out[c] = lam;
                status_out[c] = stat;
                if (sweeps_out) sweeps_out[c] = sw;
                if (step_out) step_out[c] = st;
                if (resid_out) resid_out[c] = eigen_residual(A, theta, z, lam, y);
            }
            free(buf);
        }
    }
    return fail ? -1 : 0;
}

/* ---------------------------------------------------------- complex field */
/* The paper states IPT over C^n (Sec. 2): theta, Delta and z complex, the same map
 * f_i(z) = e_i + g_i o (z (Delta z)_i - Delta z), g_j = 1/(theta_j - theta_i), the same
 * stopping test on the Euclidean norm of C^n and lambda_i = theta_i + (Delta z)_i.
 * Arithmetic written out on (re, im) pairs: products (ac - bd, ad + bc), sums in
 * ascending index order, 1/x by Smith's method (so a real input gives the real
 * oracle's numbers bit for bit). */
typedef struct {
    double re, im;
} cplx;

static cplx c_mul(cplx a, cplx b) {
    cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}

static cplx c_sub(cplx a, cplx b) {
    cplx r = {a.re - b.re, a.im - b.im};
    return r;
}

static cplx c_add(cplx a, cplx b) {
    cplx r = {a.re + b.re, a.im + b.im};
    return r;
}

static double c_abs2(cplx a) { return a.re * a.re + a.im * a.im; }

/* 1/x (Smith): divide by the larger component first. */
static cplx c_inv(cplx x) {
    cplx r;
    if (fabs(x.re) >= fabs(x.im)) {
        const double q = x.im / x.re, den = x.re + x.im * q;
        r.re = 1.0 / den;
        r.im = -q / den;
    } else {
        const double q = x.re / x.im, den = x.im + x.re * q;
        r.re = q / den;
        r.im = -1.0 / den;
    }
    return r;
}

/* One column of complex IPT (solve_column over C^n). */
static void solve_column_z(int64_t n, const cplx *theta, const cplx *delta, int64_t lda, int64_t i, double tol,
                           int max_iter, double div_norm, int div_growth, cplx *z, cplx *g, cplx *y, cplx *w,
                           cplx *lambda, int32_t *status, int32_t *sweeps, double *step) {
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) {
            g[j].re = 0.0;
            g[j].im = 0.0;
        } else {
            g[j] = c_inv(c_sub(theta[j], theta[i]));
        }
    }
    z[i].re = 1.0;
    z[i].im = 0.0;
    double prev_s = INFINITY, s = INFINITY;
    int grow = 0;
    cplx d = {0.0, 0.0};
    for (int t = 1; t <= max_iter; ++t) {
        for (int64_t j = 0; j < n; ++j) {
            const cplx *row = delta + j * lda;
            cplx acc = {0.0, 0.0};
            for (int64_t l = 0; l < n; ++l) acc = c_add(acc, c_mul(row[l], z[l]));
            y[j] = acc;
        }
        d = y[i];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) {
                w[j].re = 1.0;
                w[j].im = 0.0;
            } else {
                w[j] = c_mul(g[j], c_sub(c_mul(z[j], d), y[j]));
            }
        }
        double num = 0.0, den = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            num += c_abs2(c_sub(w[j], z[j]));
            den += c_abs2(z[j]);
        }
        s = sqrt(num) / sqrt(den);
        if (s <= tol) {
            *lambda = c_add(theta[i], d);
            *status = OR_CONVERGED;
            *sweeps = t;
            *step = s;
            return;
        }
        int finite = isfinite(s);
        double dist2 = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            cplx e = w[j];
            if (j == i) e.re -= 1.0;
            if (!isfinite(w[j].re) || !isfinite(w[j].im)) finite = 0;
            dist2 += c_abs2(e);
        }
        grow = (s > prev_s) ? grow + 1 : 0;
        prev_s = s;
        memcpy(z, w, (size_t)n * sizeof(cplx));
        if (!finite || !(sqrt(dist2) <= div_norm) || grow >= div_growth) {
            *lambda = c_add(theta[i], d);
            *status = OR_DIVERGED;
            *sweeps = t;
            *step = s;
            return;
        }
    }
    *lambda = c_add(theta[i], d);
    *status = OR_NOT_CONVERGED;
    *sweeps = max_iter;
    *step = s;
}

/* ---------------------------------------------------------------- public */

void oracle_set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Dense IPT on the requested columns.  Delta: n x n row-major (lda).  idx: k
 * requested diagonal indices (NULL means 0..k-1).  z0: optional n x k row-major
 * warm start (ldz0).  Outputs z_out (n x k row-major, ldz), lambda_out[k],
 * status_out[k], and optional sweeps_out / step_out / resid_out. */
int oracle_ipt_dense(int64_t n, const double *theta, const double *delta, int64_t lda, int64_t k,
                     const int32_t *idx, const double *z0, int64_t ldz0, double tol, int max_iter,
                     double div_norm, int div_growth, double *z_out, int64_t ldz, double *lambda_out,
                     int32_t *status_out, int32_t *sweeps_out, double *step_out, double *resid_out) {
    op_t A = {n, delta, lda, NULL, NULL, NULL};
    return solve_columns(&A, theta, k, idx, z0, ldz0, tol, max_iter, div_norm, div_growth, z_out, ldz,
                         lambda_out, status_out, sweeps_out, step_out, resid_out, 0, 0.0);
}

/* Non-autonomous continuation (solve_column_cont) with 0 < alpha < 1, otherwise as
 * oracle_ipt_dense. */
int oracle_ipt_dense_cont(int64_t n, const double *theta, const double *delta, int64_t lda, int64_t k,
                          const int32_t *idx, const double *z0, int64_t ldz0, double alpha, double tol,
                          int max_iter, double div_norm, int div_growth, double *z_out, int64_t ldz,
                          double *lambda_out, int32_t *status_out, int32_t *sweeps_out, double *step_out,
                          double *resid_out) {
    if (!(alpha > 0.0 && alpha < 1.0)) return -2;
    op_t A = {n, delta, lda, NULL, NULL, NULL};
    return solve_columns(&A, theta, k, idx, z0, ldz0, tol, max_iter, div_norm, div_growth, z_out, ldz,
                         lambda_out, status_out, sweeps_out, step_out, resid_out, 0, alpha);
}

/* IPT-ACX (Alg. 3 in place of the plain update), otherwise as oracle_ipt_dense;
 * sweeps_out counts applications of F. */
int oracle_ipt_dense_acx(int64_t n, const double *theta, const double *delta, int64_t lda, int64_t k,
                         const int32_t *idx, const double *z0, int64_t ldz0, double tol, int max_iter,
                         double div_norm, int div_growth, double *z_out, int64_t ldz, double *lambda_out,
                         int32_t *status_out, int32_t *sweeps_out, double *step_out, double *resid_out) {
    op_t A = {n, delta, lda, NULL, NULL, NULL};
    return solve_columns(&A, theta, k, idx, z0, ldz0, tol, max_iter, div_norm, div_growth, z_out, ldz,
                         lambda_out, status_out, sweeps_out, step_out, resid_out, 1, 0.0);
}

/* Same with a CSR Delta (row_ptr[n+1], col[nnz], val[nnz]). */
int oracle_ipt_csr(int64_t n, const double *theta, const int32_t *row_ptr, const int32_t *col,
                   const double *val, int64_t k, const int32_t *idx, const double *z0, int64_t ldz0,
                   double tol, int max_iter, double div_norm, int div_growth, double *z_out, int64_t ldz,
                   double *lambda_out, int32_t *status_out, int32_t *sweeps_out, double *step_out,
                   double *resid_out) {
    op_t A = {n, NULL, 0, row_ptr, col, val};
    return solve_columns(&A, theta, k, idx, z0, ldz0, tol, max_iter, div_norm, div_growth, z_out, ldz,
                         lambda_out, status_out, sweeps_out, step_out, resid_out, 0, 0.0);
}

/* IPT-ACX with a CSR Delta. */
int oracle_ipt_csr_acx(int64_t n, const double *theta, const int32_t *row_ptr, const int32_t *col,
                       const double *val, int64_t k, const int32_t *idx, const double *z0, int64_t ldz0,
                       double tol, int max_iter, double div_norm, int div_growth, double *z_out, int64_t ldz,
                       double *lambda_out, int32_t *status_out, int32_t *sweeps_out, double *step_out,
                       double *resid_out) {
    op_t A = {n, NULL, 0, row_ptr, col, val};
    return solve_columns(&A, theta, k, idx, z0, ldz0, tol, max_iter, div_norm, div_growth, z_out, ldz,
                         lambda_out, status_out, sweeps_out, step_out, resid_out, 1, 0.0);
}

/* The iterates z^(0..t) of f_i from a start z (no stopping test): out is
 * (t+1) x n row-major, out[0] = start with entry i set to 1. */
int oracle_ipt_trace(int64_t n, const double *theta, const double *delta, int64_t lda, int64_t i,
                     const double *z_start, int t, double *out) {
    op_t A = {n, delta, lda, NULL, NULL, NULL};
    double *g = (double *)malloc((size_t)n * 2 * sizeof(double));
    if (!g) return -1;
    double *y = g + n;
    inverse_gaps(n, theta, i, g);
    for (int64_t j = 0; j < n; ++j) out[j] = z_start ? z_start[j] : (j == i ? 1.0 : 0.0);
    out[i] = 1.0;
    for (int s = 1; s <= t; ++s) map_once(&A, theta, i, g, out + (int64_t)(s - 1) * n, y, out + (int64_t)s * n);
    free(g);
    return 0;
}

/* One application of f_i to z (dense Delta); returns d = (Delta z)_i. */
double oracle_ipt_map(int64_t n, const double *theta, const double *delta, int64_t lda, int64_t i,
                      const double *z, double *w) {
    op_t A = {n, delta, lda, NULL, NULL, NULL};
    double *g = (double *)malloc((size_t)n * 2 * sizeof(double));
    if (!g) return NAN;
    double *y = g + n;
    inverse_gaps(n, theta, i, g);
    const double d = map_once(&A, theta, i, g, z, y, w);
    free(g);
    return d;
}

/* Batched dense IPT: problem b has size ns[b], theta at theta_pool + theta_off[b],
 * row-major Delta at delta_pool + delta_off[b], and its full spectrum is written to
 * z_pool + z_off[b] (n_b x n_b row-major), lambda_pool + theta_off[b],
 * status_pool + theta_off[b].  Problems are independent; this is a loop. */
int oracle_ipt_batched(int32_t count, const int32_t *ns, const int64_t *theta_off, const int64_t *delta_off,
                       const int64_t *z_off, const double *theta_pool, const double *delta_pool, double tol,
                       int max_iter, double div_norm, int div_growth, double *z_pool, double *lambda_pool,
                       int32_t *status_pool, int32_t *sweeps_pool) {
    for (int32_t b = 0; b < count; ++b) {
        const int64_t n = ns[b];
        int rc = oracle_ipt_dense(n, theta_pool + theta_off[b], delta_pool + delta_off[b], n, n, NULL, NULL, 0, tol,
                                  max_iter, div_norm, div_growth, z_pool + z_off[b], n, lambda_pool + theta_off[b],
                                  status_pool + theta_off[b], sweeps_pool ? sweeps_pool + theta_off[b] : NULL, NULL,
                                  NULL);
        if (rc) return rc;
    }
    return 0;
}

/* Complex dense IPT (solve_column_z per requested column).  theta: n complex,
 * Delta: n x n row-major complex (lda complex elements), z0 / z_out: n x k row-major
 * complex; complex numbers are (re, im) pairs of doubles.  Otherwise as
 * oracle_ipt_dense (resid_out: |M z - lambda z| / |z|). */
int oracle_ipt_dense_z(int64_t n, const double *theta, const double *delta, int64_t lda, int64_t k,
                       const int32_t *idx, const double *z0, int64_t ldz0, double tol, int max_iter, double div_norm,
                       int div_growth, double *z_out, int64_t ldz, double *lambda_out, int32_t *status_out,
                       int32_t *sweeps_out, double *step_out, double *resid_out) {
    const cplx *th = (const cplx *)theta, *A = (const cplx *)delta, *Z0 = (const cplx *)z0;
    cplx *Zo = (cplx *)z_out, *L = (cplx *)lambda_out;
    int fail = 0;
#pragma omp parallel
    {
        cplx *buf = (cplx *)malloc((size_t)n * 4 * sizeof(cplx));
        if (!buf) {
#pragma omp atomic write
            fail = 1;
        } else {
            cplx *z = buf, *g = buf + n, *y = buf + 2 * n, *w = buf + 3 * n;
#pragma omp for schedule(dynamic, 1)
            for (int64_t c = 0; c < k; ++c) {
                const int64_t i = idx ? idx[c] : c;
                for (int64_t j = 0; j < n; ++j) {
                    if (Z0) {
                        z[j] = Z0[j * ldz0 + c];
                    } else {
                        z[j].re = (j == i) ? 1.0 : 0.0;
                        z[j].im = 0.0;
                    }
                }
                cplx lam;
                int32_t stat, sw;
                double st;
                solve_column_z(n, th, A, lda, i, tol, max_iter, div_norm, div_growth, z, g, y, w, &lam, &stat, &sw,
                               &st);
                for (int64_t j = 0; j < n; ++j) Zo[j * ldz + c] = z[j];
                L[c] = lam;
                status_out[c] = stat;
                if (sweeps_out) sweeps_out[c] = sw;
                if (step_out) step_out[c] = st;
                if (resid_out) {
                    double r2 = 0.0, z2 = 0.0;
                    for (int64_t j = 0; j < n; ++j) {
                        cplx acc = {0.0, 0.0};
                        for (int64_t l = 0; l < n; ++l) acc = c_add(acc, c_mul(A[j * lda + l], z[l]));
                        const cplx r = c_sub(c_add(c_mul(th[j], z[j]), acc), c_mul(lam, z[j]));
                        r2 += c_abs2(r);
                        z2 += c_abs2(z[j]);
                    }
                    resid_out[c] = sqrt(r2) / sqrt(z2);
                }
            }
            free(buf);
        }
    }
    return fail ? -1 : 0;
}
