// Drives the C ABI of libipt under the host address and undefined-behaviour
// sanitizers (the library's host code built with them, its kernels as usual).
//   abi_sanitize_driver          argument checks and calls that need no device
//   abi_sanitize_driver gpu      also a live handle: rejected arguments, then one small
//                                solve of every kind (dense FP64 / ladder / IPT-ACX /
//                                homotopy / no-allocation, complex, CSR, batched with and
//                                without the choice of D, the tile tuner, the
//                                Rayleigh-Schroedinger terms and the warm-start network)
// Exits 0 when every call returned what it should; the sanitizers abort on any
// host-side memory error or undefined operation.
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "ipt.h"

static int failures = 0;
#define EXPECT(cond)                                                             \
    do {                                                                         \
        if (!(cond)) {                                                           \
            fprintf(stderr, "abi_sanitize_driver:%d: failed: %s\n", __LINE__, #cond); \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double urand() {  // xorshift64 in [-1, 1)
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

template <typename T>
static T *dev_copy(const std::vector<T> &h) {
    T *d = nullptr;
    if (hipMalloc((void **)&d, h.size() * sizeof(T) + 16) != hipSuccess) return nullptr;
    if (hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    return d;
}
template <typename T>
static T *dev_alloc(size_t count) {
    T *d = nullptr;
    if (hipMalloc((void **)&d, count * sizeof(T) + 16) != hipSuccess) return nullptr;
    return d;
}
template <typename T>
static std::vector<T> host_copy(const T *d, size_t count) {
    std::vector<T> h(count);
    (void)hipMemcpy(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost);
    return h;
}

static void no_device_calls() {
    ipt_opts o;
    ipt_opts_default(&o);
    EXPECT(o.tol > 0.0 && o.max_iter >= 1);
    for (int s = 0; s <= 7; ++s) EXPECT(ipt_status_string((ipt_status)s) != nullptr);
    EXPECT(ipt_last_error(nullptr) != nullptr);
    EXPECT(ipt_create(nullptr, nullptr) == IPT_EINVAL);
    EXPECT(ipt_destroy(nullptr) == IPT_EINVAL);
    EXPECT(ipt_set_stream(nullptr, nullptr) == IPT_EINVAL);
    double x = 0.0;
    int32_t i = 0;
    EXPECT(ipt_solve_dense(nullptr, 1, &x, &x, 1, 1, &i, nullptr, 0, nullptr, &x, 1, &x, &i, nullptr, nullptr) ==
           IPT_EINVAL);
    EXPECT(ipt_solve_csr(nullptr, 1, &x, &i, &i, &x, 0, 1, &i, nullptr, 0, nullptr, &x, 1, &x, &i, nullptr,
                         nullptr) == IPT_EINVAL);
    EXPECT(ipt_solve_csr_z(nullptr, 1, &x, &i, &i, &x, 0, 1, &i, nullptr, 0, nullptr, &x, 1, &x, &i, nullptr,
                           nullptr) == IPT_EINVAL);
    EXPECT(ipt_solve_batched(nullptr, 1, &i, nullptr, nullptr, nullptr, &x, &x, nullptr, &x, &x, &i, nullptr) ==
           IPT_EINVAL);
    EXPECT(ipt_mlp_destroy(nullptr) == IPT_EINVAL);
    EXPECT(ipt_mlp_num_params(nullptr) == -1);
}

static void gpu_calls() {
    ipt_handle h = nullptr;
    if (ipt_create(&h, nullptr) != IPT_OK) {
        fprintf(stderr, "abi_sanitize_driver: no device\n");
        ++failures;
        return;
    }
    ipt_opts o;
    ipt_opts_default(&o);
    const int64_t n = 200, k = n;
    std::vector<double> th(n), de(n * n);
    for (int64_t j = 0; j < n; ++j) th[j] = (double)(j + 1);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t l = 0; l <= j; ++l) de[j * n + l] = de[l * n + j] = 0.02 * urand() / sqrt((double)n);
    double *dth = dev_copy(th), *dde = dev_copy(de), *dz = dev_alloc<double>(n * k), *dl = dev_alloc<double>(k);
    int32_t *dst = dev_alloc<int32_t>(k);
    ipt_info info;
    // rejected arguments on a live handle
    EXPECT(ipt_solve_dense(h, 0, dth, dde, n, k, nullptr, nullptr, 0, &o, dz, k, dl, dst, &info, nullptr) ==
           IPT_EINVAL);
    EXPECT(strlen(ipt_last_error(h)) > 0);
    EXPECT(ipt_solve_dense(h, n, dth, dde, n - 1, k, nullptr, nullptr, 0, &o, dz, k, dl, dst, &info, nullptr) ==
           IPT_EINVAL);
    EXPECT(ipt_solve_dense(h, n, dth, dde, n, k + 1, nullptr, nullptr, 0, &o, dz, k, dl, dst, &info, nullptr) ==
           IPT_EINVAL);
    ipt_opts bad = o;
    bad.tol = NAN;
    EXPECT(ipt_solve_dense(h, n, dth, dde, n, k, nullptr, nullptr, 0, &bad, dz, k, dl, dst, &info, nullptr) ==
           IPT_EINVAL);
    bad = o;
    bad.precision = 7;
    EXPECT(ipt_solve_dense(h, n, dth, dde, n, k, nullptr, nullptr, 0, &bad, dz, k, dl, dst, &info, nullptr) ==
           IPT_EINVAL);
    int32_t tiles_bad[IPT_TILE_BUCKETS];
    for (int q = 0; q < IPT_TILE_BUCKETS; ++q) tiles_bad[q] = 48;
    EXPECT(ipt_batched_set_tiles(h, tiles_bad) == IPT_EINVAL);
    // dense: FP64, ladder, IPT-ACX, homotopy, no-allocation, with column info
    std::vector<ipt_opts> variants(5, o);
    variants[1].precision = IPT_PREC_LADDER;
    variants[2].flags = IPT_FLAG_ACX;
    variants[3].homotopy_q = 2;
    for (int v = 0; v < 5; ++v) {
        int32_t *csw = dev_alloc<int32_t>(k);
        double *cst = dev_alloc<double>(k), *cre = dev_alloc<double>(k);
        ipt_colinfo ci = {csw, cst, cre};
        const ipt_status st =
            v < 4 ? ipt_solve_dense(h, n, dth, dde, n, k, nullptr, nullptr, 0, &variants[v], dz, k, dl, dst, &info, &ci)
                  : ipt_solve_dense_noalloc(h, n, dth, dde, n, k, nullptr, nullptr, 0, &o, dz, k, dl, dst, &info, &ci);
        EXPECT(st == IPT_OK);
        EXPECT(info.converged == k);
        (void)hipFree(csw);
        (void)hipFree(cst);
        (void)hipFree(cre);
    }
    // warm start from the last answer, a subset of columns in any order
    {
        const int64_t kk = 37;
        std::vector<int32_t> idx(kk);
        for (int64_t c = 0; c < kk; ++c) idx[c] = (int32_t)((c * 53 + 11) % n);
        int32_t *didx = dev_copy(idx);
        double *dz2 = dev_alloc<double>(n * kk), *dl2 = dev_alloc<double>(kk);
        int32_t *dst2 = dev_alloc<int32_t>(kk);
        EXPECT(ipt_solve_dense(h, n, dth, dde, n, kk, didx, nullptr, 0, &o, dz2, kk, dl2, dst2, &info, nullptr) ==
               IPT_OK);
        EXPECT(ipt_solve_dense(h, n, dth, dde, n, kk, didx, dz2, kk, &o, dz2, kk, dl2, dst2, &info, nullptr) == IPT_OK);
        (void)hipFree(didx);
        (void)hipFree(dz2);
        (void)hipFree(dl2);
        (void)hipFree(dst2);
    }
    // complex Hermitian
    {
        std::vector<double> thz(2 * n), dzm(2 * n * n);
        for (int64_t j = 0; j < n; ++j) {
            thz[2 * j] = th[j];
            thz[2 * j + 1] = 0.0;
            for (int64_t l = 0; l <= j; ++l) {
                const double re = de[j * n + l], im = (l == j) ? 0.0 : 0.01 * urand() / sqrt((double)n);
                dzm[2 * (j * n + l)] = re;
                dzm[2 * (j * n + l) + 1] = im;
                dzm[2 * (l * n + j)] = re;
                dzm[2 * (l * n + j) + 1] = -im;
            }
        }
        double *dthz = dev_copy(thz), *ddz = dev_copy(dzm), *dzz = dev_alloc<double>(2 * n * k);
        double *dlz = dev_alloc<double>(2 * k);
        EXPECT(ipt_solve_dense_z(h, n, dthz, ddz, n, k, nullptr, nullptr, 0, &o, dzz, k, dlz, dst, &info, nullptr) ==
               IPT_OK);
        (void)hipFree(dthz);
        (void)hipFree(ddz);
        (void)hipFree(dzz);
        (void)hipFree(dlz);
    }
    // CSR: tridiagonal plus a few long-range pairs, 8 lowest columns, FP64 and ladder
    {
        const int64_t m = 3000, kk = 8;
        std::vector<std::vector<std::pair<int32_t, double>>> rows(m);
        for (int64_t j = 0; j + 1 < m; ++j) {
            const double v = 0.05 * urand();
            rows[j].push_back({(int32_t)(j + 1), v});
            rows[j + 1].push_back({(int32_t)j, v});
        }
        for (int64_t j = 0; j + 97 < m; j += 13) {
            const double v = 0.05 * urand();
            rows[j].push_back({(int32_t)(j + 97), v});
            rows[j + 97].push_back({(int32_t)j, v});
        }
        std::vector<int32_t> rp(m + 1), col, idx(kk);
        std::vector<double> val, ths(m);
        for (int64_t j = 0; j < m; ++j) {
            rp[j] = (int32_t)col.size();
            for (auto &e : rows[j]) {
                col.push_back(e.first);
                val.push_back(e.second);
            }
            ths[j] = (double)j;
        }
        rp[m] = (int32_t)col.size();
        for (int64_t c = 0; c < kk; ++c) idx[c] = (int32_t)c;
        int32_t *drp = dev_copy(rp), *dcol = dev_copy(col), *didx = dev_copy(idx), *dst2 = dev_alloc<int32_t>(kk);
        double *dval = dev_copy(val), *dths = dev_copy(ths), *dz2 = dev_alloc<double>(m * kk),
               *dl2 = dev_alloc<double>(kk);
        for (int prec : {IPT_PREC_FP64, IPT_PREC_LADDER}) {
            ipt_opts oc = o;
            oc.precision = prec;
            EXPECT(ipt_solve_csr(h, m, dths, drp, dcol, dval, (int64_t)col.size(), kk, didx, nullptr, 0, &oc, dz2, kk,
                                 dl2, dst2, &info, nullptr) == IPT_OK);
        }
        // the same pattern over C^n: imaginary parts on the off-diagonal pairs (Hermitian)
        {
            std::vector<double> valz(2 * val.size()), thz(2 * m);
            for (int64_t j = 0; j < m; ++j) {
                thz[2 * j] = ths[j];
                thz[2 * j + 1] = 0.0;
                for (int32_t p = rp[j]; p < rp[j + 1]; ++p) {
                    valz[2 * p] = val[p];
                    valz[2 * p + 1] = (col[p] > j ? 0.01 : -0.01) * val[p];
                }
            }
            double *dvz = dev_copy(valz), *dtz = dev_copy(thz), *dzz = dev_alloc<double>(2 * m * kk),
                   *dlz = dev_alloc<double>(2 * kk);
            EXPECT(ipt_solve_csr_z(h, m, dtz, drp, dcol, dvz, (int64_t)col.size(), kk, didx, nullptr, 0, &o, dzz, kk,
                                   dlz, dst2, &info, nullptr) == IPT_OK);
            ipt_opts ol = o;
            ol.precision = IPT_PREC_LADDER;
            EXPECT(ipt_solve_csr_z(h, m, dtz, drp, dcol, dvz, (int64_t)col.size(), kk, didx, nullptr, 0, &ol, dzz, kk,
                                   dlz, dst2, &info, nullptr) == IPT_EINVAL);
            (void)hipFree(dvz);
            (void)hipFree(dtz);
            (void)hipFree(dzz);
            (void)hipFree(dlz);
        }
        (void)hipFree(drp);
        (void)hipFree(dcol);
        (void)hipFree(didx);
        (void)hipFree(dst2);
        (void)hipFree(dval);
        (void)hipFree(dths);
        (void)hipFree(dz2);
        (void)hipFree(dl2);
    }
    // batched: uneven sizes in pools; ladder, choice of D, the tuner
    {
        const int32_t count = 9;
        const int32_t ns[count] = {1, 2, 31, 64, 65, 100, 129, 200, 3};
        std::vector<int64_t> toff(count), doff(count);
        int64_t tt = 0, dd = 0;
        for (int b = 0; b < count; ++b) {
            toff[b] = tt;
            doff[b] = dd;
            tt += ns[b];
            dd += (int64_t)ns[b] * ns[b];
        }
        std::vector<double> thp(tt), dep(dd);
        for (int b = 0; b < count; ++b) {
            const int64_t nb = ns[b];
            for (int64_t j = 0; j < nb; ++j) thp[toff[b] + j] = (double)j + 0.5 * (urand() + 1.0) * 0.9;
            for (int64_t j = 0; j < nb; ++j)
                for (int64_t l = 0; l <= j; ++l)
                    dep[doff[b] + j * nb + l] = dep[doff[b] + l * nb + j] = 0.02 * urand() / sqrt((double)nb);
        }
        double *dthp = dev_copy(thp), *ddep = dev_copy(dep), *dzp = dev_alloc<double>(dd), *dlp = dev_alloc<double>(tt);
        int32_t *dsp = dev_alloc<int32_t>(tt);
        ipt_opts ob = o;
        ob.precision = IPT_PREC_LADDER;
        ob.max_iter = 64;
        EXPECT(ipt_solve_batched(h, count, ns, toff.data(), doff.data(), doff.data(), dthp, ddep, &ob, dzp, dlp, dsp,
                                 &info) <= IPT_ENOTCONV);
        ob.flags = IPT_FLAG_CHOOSE_D;
        EXPECT(ipt_solve_batched(h, count, ns, toff.data(), doff.data(), doff.data(), dthp, ddep, &ob, dzp, dlp, dsp,
                                 &info) <= IPT_ENOTCONV);
        int32_t tiles[IPT_TILE_BUCKETS];
        EXPECT(ipt_batched_tune(h, count, ns, toff.data(), doff.data(), doff.data(), dthp, ddep, dzp, dlp, dsp, tiles) ==
               IPT_OK);
        EXPECT(ipt_batched_get_tiles(h, tiles) == IPT_OK);
        EXPECT(ipt_batched_set_tiles(h, tiles) == IPT_OK);
        (void)hipFree(dthp);
        (void)hipFree(ddep);
        (void)hipFree(dzp);
        (void)hipFree(dlp);
        (void)hipFree(dsp);
    }
    // Rayleigh-Schroedinger terms and the warm-start network on 8 family members
    {
        const int64_t kk = 4, order = 2, out = n * kk;
        const int32_t batch = 8;
        std::vector<int32_t> idx(kk);
        for (int64_t c = 0; c < kk; ++c) idx[c] = (int32_t)c;
        std::vector<double> eps(batch);
        std::vector<float> x(batch * 2);
        for (int p = 0; p < batch; ++p) {
            eps[p] = 0.01 * (p + 1);
            x[2 * p] = (float)(eps[p] / 0.08);
            x[2 * p + 1] = 1.0f;
        }
        int32_t *didx = dev_copy(idx);
        double *deps = dev_copy(eps), *terms = dev_alloc<double>(order * n * kk), *z0 = dev_alloc<double>(batch * n * kk);
        float *dx = dev_copy(x), *tg = dev_alloc<float>(batch * out), *mu = dev_alloc<float>(out),
              *sg = dev_alloc<float>(out), *y = dev_alloc<float>(batch * out);
        EXPECT(ipt_rs_terms(h, n, dth, dde, n, kk, didx, (int32_t)order, terms) == IPT_OK);
        EXPECT(ipt_rs_start(h, deps, batch, (int32_t)order, terms, n, kk, didx, z0, kk, n * kk) == IPT_OK);
        EXPECT(ipt_mlp_targets(h, z0, batch, n, kk, kk, n * kk, didx, deps, (int32_t)order, terms, nullptr, tg, mu, sg) ==
               IPT_OK);
        ipt_mlp m = nullptr;
        EXPECT(ipt_mlp_create(h, 2, 64, 2, (int32_t)out, 7, &m) == IPT_OK);
        if (m) {
            const int64_t np = ipt_mlp_num_params(m);
            EXPECT(np > 0);
            float *params = dev_alloc<float>(np), *grad = dev_alloc<float>(np);
            float loss = 0.f;
            EXPECT(ipt_mlp_get_params(m, params) == IPT_OK);
            EXPECT(ipt_mlp_set_params(m, params) == IPT_OK);
            EXPECT(ipt_mlp_forward(m, dx, batch, y) == IPT_OK);
            EXPECT(ipt_mlp_loss_grad(m, dx, tg, nullptr, batch, &loss, grad) == IPT_OK && isfinite(loss));
            EXPECT(ipt_mlp_train(m, dx, tg, nullptr, batch, 5, 1e-3f, &loss) == IPT_OK && isfinite(loss));
            EXPECT(ipt_mlp_predict_z0(m, dx, batch, mu, sg, deps, (int32_t)order, terms, n, kk, didx, z0, kk, n * kk) ==
                   IPT_OK);
            EXPECT(ipt_mlp_destroy(m) == IPT_OK);
            (void)hipFree(params);
            (void)hipFree(grad);
        }
        (void)hipFree(didx);
        (void)hipFree(deps);
        (void)hipFree(terms);
        (void)hipFree(z0);
        (void)hipFree(dx);
        (void)hipFree(tg);
        (void)hipFree(mu);
        (void)hipFree(sg);
        (void)hipFree(y);
    }
    std::vector<int32_t> st = host_copy(dst, k);
    (void)st;
    (void)hipFree(dth);
    (void)hipFree(dde);
    (void)hipFree(dz);
    (void)hipFree(dl);
    (void)hipFree(dst);
    EXPECT(ipt_destroy(h) == IPT_OK);
}

int main(int argc, char **argv) {
    no_device_calls();
    if (argc > 1 && strcmp(argv[1], "gpu") == 0) gpu_calls();
    if (failures) {
        fprintf(stderr, "abi_sanitize_driver: %d check(s) failed\n", failures);
        return 1;
    }
    printf("abi_sanitize_driver: ok (%s)\n", argc > 1 ? argv[1] : "no device");
    return 0;
}
