/* Exercises every public entry point of the C oracle on small inputs, for builds with
 * the address and undefined-behaviour sanitizers (test infrastructure, like the
 * oracle itself).  The inputs are a fixed pseudo-random near-diagonal family; the
 * program checks only that every call returns and that the outputs are finite or
 * carry a failure status, and exits non-zero otherwise.  The sanitizers report any
 * out-of-bounds access, use after free or undefined operation on the way. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_ipt_dense(int64_t, const double *, const double *, int64_t, int64_t, const int32_t *, const double *,
                     int64_t, double, int, double, int, double *, int64_t, double *, int32_t *, int32_t *, double *,
                     double *);
int oracle_ipt_dense_cont(int64_t, const double *, const double *, int64_t, int64_t, const int32_t *,
                          const double *, int64_t, double, double, int, double, int, double *, int64_t, double *,
                          int32_t *, int32_t *, double *, double *);
int oracle_ipt_dense_acx(int64_t, const double *, const double *, int64_t, int64_t, const int32_t *, const double *,
                         int64_t, double, int, double, int, double *, int64_t, double *, int32_t *, int32_t *,
                         double *, double *);
int oracle_ipt_csr(int64_t, const double *, const int32_t *, const int32_t *, const double *, int64_t,
                   const int32_t *, const double *, int64_t, double, int, double, int, double *, int64_t, double *,
                   int32_t *, int32_t *, double *, double *);
int oracle_ipt_csr_acx(int64_t, const double *, const int32_t *, const int32_t *, const double *, int64_t,
                       const int32_t *, const double *, int64_t, double, int, double, int, double *, int64_t,
                       double *, int32_t *, int32_t *, double *, double *);
int oracle_ipt_trace(int64_t, const double *, const double *, int64_t, int64_t, const double *, int, double *);
double oracle_ipt_map(int64_t, const double *, const double *, int64_t, int64_t, const double *, double *);
int oracle_ipt_batched(int32_t, const int32_t *, const int64_t *, const int64_t *, const int64_t *, const double *,
                       const double *, double, int, double, int, double *, double *, int32_t *, int32_t *);
int oracle_ipt_dense_z(int64_t, const double *, const double *, int64_t, int64_t, const int32_t *, const double *,
                       int64_t, double, int, double, int, double *, int64_t, double *, int32_t *, int32_t *, double *,
                       double *);
void oracle_set_threads(int);

static uint64_t rng = 88172645463325252ull;
static double urand(void) { /* xorshift64, uniform in [-1, 1) */
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static int failures = 0;
#define CHECK(cond, what)                                  \
    do {                                                   \
        if (!(cond)) {                                     \
            fprintf(stderr, "sanitize_driver: %s\n", what); \
            ++failures;                                    \
        }                                                  \
    } while (0)

/* theta_j = j + 1 (lda-strided Delta with a padded row: lda = n + 3) */
static void family(int64_t n, int64_t lda, double eps, double *theta, double *delta) {
    for (int64_t j = 0; j < n; ++j) theta[j] = (double)(j + 1);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t l = 0; l < lda; ++l) delta[j * lda + l] = (l < n) ? eps * urand() : NAN; /* padding never read */
}

static void outputs_ok(int64_t n, int64_t k, int64_t ldz, const double *z, const double *lam, const int32_t *st,
                       int complex_, const char *what) {
    for (int64_t c = 0; c < k; ++c) {
        if (st[c] != 0) continue; /* only converged columns must be finite */
        for (int64_t j = 0; j < n; ++j)
            for (int q = 0; q <= complex_; ++q)
                CHECK(isfinite(z[(j * ldz + c) * (complex_ + 1) + q]), what);
        CHECK(isfinite(lam[c * (complex_ + 1)]), what);
    }
}

int main(void) {
    oracle_set_threads(4);
    const int64_t sizes[] = {1, 2, 3, 17, 64};
    for (int s = 0; s < 5; ++s) {
        const int64_t n = sizes[s], lda = n + 3, k = n > 4 ? n - 2 : n, ldz = k + 1;
        double *theta = malloc(n * sizeof(double)), *delta = malloc(n * lda * sizeof(double));
        double *z = malloc(n * ldz * sizeof(double)), *z0 = malloc(n * ldz * sizeof(double));
        double *lam = malloc(k * sizeof(double)), *step = malloc(k * sizeof(double)), *res = malloc(k * sizeof(double));
        int32_t *st = malloc(k * sizeof(int32_t)), *sw = malloc(k * sizeof(int32_t)), *idx = malloc(k * sizeof(int32_t));
        family(n, lda, 0.05, theta, delta);
        for (int64_t c = 0; c < k; ++c) idx[c] = (int32_t)((c * 7 + 1) % n); /* distinct: 7 is prime to n here */
        if (n == 64 || n == 17) {
            for (int64_t c = 0; c < k; ++c) idx[c] = (int32_t)(n - 1 - c);
        }
        CHECK(oracle_ipt_dense(n, theta, delta, lda, k, idx, NULL, 0, 1e-12, 50, 1e3, 8, z, ldz, lam, st, sw, step,
                               res) == 0, "dense rc");
        outputs_ok(n, k, ldz, z, lam, st, 0, "dense outputs");
        for (int64_t j = 0; j < n * ldz; ++j) z0[j] = z[j];
        CHECK(oracle_ipt_dense(n, theta, delta, lda, k, idx, z0, ldz, 1e-12, 50, 1e3, 8, z, ldz, lam, st, NULL, NULL,
                               NULL) == 0, "dense warm rc");
        CHECK(oracle_ipt_dense_cont(n, theta, delta, lda, k, idx, NULL, 0, 0.5, 1e-10, 200, 1e3, 8, z, ldz, lam, st,
                                    sw, step, res) == 0, "cont rc");
        CHECK(oracle_ipt_dense_acx(n, theta, delta, lda, k, idx, NULL, 0, 1e-12, 60, 1e3, 8, z, ldz, lam, st, sw,
                                   step, res) == 0, "acx rc");
        outputs_ok(n, k, ldz, z, lam, st, 0, "acx outputs");
        /* CSR of the same Delta (without its padding), rows sorted */
        int32_t *rp = malloc((n + 1) * sizeof(int32_t)), *col = malloc(n * n * sizeof(int32_t));
        double *val = malloc(n * n * sizeof(double));
        int64_t nnz = 0;
        for (int64_t j = 0; j < n; ++j) {
            rp[j] = (int32_t)nnz;
            for (int64_t l = 0; l < n; ++l)
                if ((j + l) % 3 != 1) {
                    col[nnz] = (int32_t)l;
                    val[nnz++] = delta[j * lda + l];
                }
        }
        rp[n] = (int32_t)nnz;
        CHECK(oracle_ipt_csr(n, theta, rp, col, val, k, idx, NULL, 0, 1e-12, 50, 1e3, 8, z, ldz, lam, st, sw, step,
                             res) == 0, "csr rc");
        outputs_ok(n, k, ldz, z, lam, st, 0, "csr outputs");
        CHECK(oracle_ipt_csr_acx(n, theta, rp, col, val, k, idx, NULL, 0, 1e-12, 60, 1e3, 8, z, ldz, lam, st, sw,
                                 step, res) == 0, "csr acx rc");
        /* trace and one map application */
        double *tr = malloc((size_t)(n * 6) * sizeof(double)), *w = malloc(n * sizeof(double));
        CHECK(oracle_ipt_trace(n, theta, delta, lda, n - 1, NULL, 5, tr) == 0, "trace rc");
        CHECK(isfinite(oracle_ipt_map(n, theta, delta, lda, 0, tr + 5 * n, w)), "map value");
        /* complex: Hermitian perturbation of the same size */
        double *thz = malloc(2 * n * sizeof(double)), *dz = malloc(2 * n * n * sizeof(double));
        double *zz = malloc(2 * n * k * sizeof(double)), *lz = malloc(2 * k * sizeof(double));
        for (int64_t j = 0; j < n; ++j) {
            thz[2 * j] = theta[j];
            thz[2 * j + 1] = 0.0;
            for (int64_t l = 0; l <= j; ++l) {
                const double re = 0.05 * urand(), im = (l == j) ? 0.0 : 0.05 * urand();
                dz[2 * (j * n + l)] = re;
                dz[2 * (j * n + l) + 1] = im;
                dz[2 * (l * n + j)] = re;
                dz[2 * (l * n + j) + 1] = -im;
            }
        }
        CHECK(oracle_ipt_dense_z(n, thz, dz, n, k, idx, NULL, 0, 1e-12, 50, 1e3, 8, zz, k, lz, st, sw, step, res) == 0,
              "complex rc");
        outputs_ok(n, k, k, zz, lz, st, 1, "complex outputs");
        free(theta); free(delta); free(z); free(z0); free(lam); free(step); free(res); free(st); free(sw); free(idx);
        free(rp); free(col); free(val); free(tr); free(w); free(thz); free(dz); free(zz); free(lz);
    }
    /* a small batch of uneven sizes packed in pools */
    {
        const int32_t count = 5, ns[5] = {1, 9, 2, 33, 5};
        int64_t toff[5], doff[5], tt = 0, dd = 0;
        for (int b = 0; b < count; ++b) {
            toff[b] = tt;
            doff[b] = dd;
            tt += ns[b];
            dd += (int64_t)ns[b] * ns[b];
        }
        double *th = malloc(tt * sizeof(double)), *de = malloc(dd * sizeof(double)), *zp = malloc(dd * sizeof(double));
        double *lp = malloc(tt * sizeof(double));
        int32_t *sp = malloc(tt * sizeof(int32_t)), *swp = malloc(tt * sizeof(int32_t));
        for (int b = 0; b < count; ++b) family(ns[b], ns[b], 0.03, th + toff[b], de + doff[b]);
        CHECK(oracle_ipt_batched(count, ns, toff, doff, doff, th, de, 1e-12, 50, 1e3, 8, zp, lp, sp, swp) == 0,
              "batched rc");
        free(th); free(de); free(zp); free(lp); free(sp); free(swp);
    }
    if (failures) return 1;
    printf("sanitize_driver: all oracle entry points ran\n");
    return 0;
}
