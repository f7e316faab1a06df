// Rayleigh-Schroedinger corrections of M = D + Delta on requested columns (App. B,
// eq. ARS-alpha): with Z^[0] = E (the unit columns e_i, i = idx[c]) and
// d^[s]_c = (Delta Z^[s])_{i c},
//   Z^[l] = G o ( sum_{s=0}^{l-1} Z^[l-1-s] d^[s] - Delta Z^[l-1] ),   G_jc = 1/(theta_j - theta_i),
// so that Z_RS(eps) = sum_l eps^l Z^[l] is the perturbation series of D + eps Delta (the
// series IPT contains, App. C).  Each column is independent.  These terms are computed
// once for a family and give warm starts at no cost per member.  FP64 throughout.
#include "ipt_internal.h"

namespace ipt {

namespace {

__global__ void k_rs_clear(int32_t *err) { *err = 0; }

// a / b and a % b for non-negative a, b > 0, in 32 bits when both fit
__device__ inline void divmod_nn(int64_t a, int64_t b, int64_t &q, int64_t &r) {
    if (((a | b) >> 31) == 0) {
        const uint32_t qa = (uint32_t)a / (uint32_t)b;
        q = qa;
        r = a - (int64_t)qa * b;
    } else {
        q = a / b;
        r = a - q * b;
    }
}

// Y^[0] = Delta E: y[j, c] = Delta[j, idx[c]].
__global__ void k_rs_gather(const double *delta, int64_t lda, const int32_t *idx, int64_t n, int64_t k, double *y,
                            int32_t *err) {
    const int64_t total = n * k;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < total; u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = u / k, c = u - j * k;
        const int32_t i = idx[c];
        if (i < 0 || i >= n) {
            atomicOr(err, 1);
            y[u] = 0.0;
            continue;
        }
        y[u] = delta[j * lda + i];
    }
}

// y = Delta z (n x n times n x k, row-major): a wave per row j; lane l sums the
// columns l, l + 64, ... of that row for 16 columns of z at a time, then the wave
// adds its lanes in a fixed order.
constexpr int RS_COLS = 16;
__global__ __launch_bounds__(256) void k_rs_product(const double *delta, int64_t lda, const double *z, int64_t n,
                                                    int64_t k, double *y) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= n) return;
    const double *row = delta + j * lda;
    for (int64_t c0 = 0; c0 < k; c0 += RS_COLS) {
        double acc[RS_COLS];
#pragma unroll
        for (int q = 0; q < RS_COLS; ++q) acc[q] = 0.0;
        for (int64_t l = lane; l < n; l += 64) {
            const double a = row[l];
            const double *zr = z + l * k + c0;
#pragma unroll
            for (int q = 0; q < RS_COLS; ++q)
                if (c0 + q < k) acc[q] = fma(a, zr[q], acc[q]);
        }
#pragma unroll
        for (int q = 0; q < RS_COLS; ++q) {
            double v = acc[q];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0 && c0 + q < k) y[j * k + c0 + q] = v;
        }
    }
}

// d[l-1] = the diagonal entries of y = Delta Z^[l-1]; then Z^[l] (written as term l
// at terms + (l-1) n k); terms 1..l-1 are already there, Z^[0] = E contributes only on
// the diagonal, where G is zero.
__global__ void k_rs_term(const double *theta, const int32_t *idx, const double *y, double *terms, double *d,
                          int32_t l, int64_t n, int64_t k, int32_t *err) {
    const int64_t total = n * k;
    const int64_t nk = n * k;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < total; u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = u / k, c = u - j * k;
        const int32_t i = idx[c];
        if (i < 0 || i >= n) {
            terms[(int64_t)(l - 1) * nk + u] = 0.0;
            continue;
        }
        // d^[s] for s < l - 1 were stored by the earlier terms; d^[l-1] is read from y
        const double dl = y[(int64_t)i * k + c];
        if (j == i) {
            d[(int64_t)(l - 1) * k + c] = dl;
            terms[(int64_t)(l - 1) * nk + u] = 0.0;
            continue;
        }
        double acc = 0.0;
        for (int s = 0; s + 1 < l; ++s)  // s = l - 1 pairs with Z^[0] = E, zero off the diagonal
            acc += terms[(int64_t)(l - 2 - s) * nk + u] * d[(int64_t)s * k + c];
        const double gap = theta[j] - theta[i];
        if (!(gap != 0.0) || !isfinite(gap)) atomicOr(err, 2);
        const double g = 1.0 / gap;
        terms[(int64_t)(l - 1) * nk + u] = g * (acc - y[u]);
    }
}

// Z0_p = E + sum_{l=1..order} eps_p^l T_l for problems p < count.
__global__ void k_rs_start(const double *eps, int32_t count, int32_t order, const double *terms, int64_t n, int64_t k,
                           const int32_t *idx, double *z0, int64_t ldz0, int64_t pstride) {
    const int64_t nk = n * k, total = (int64_t)count * nk;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < total; u += (int64_t)gridDim.x * blockDim.x) {
        int64_t p, q, j, c;
        divmod_nn(u, nk, p, q);
        divmod_nn(q, k, j, c);
        double v = 1.0;
        if (j != idx[c]) {
            const double ep = eps[p];
            double pw = 1.0;
            v = 0.0;
            for (int l = 1; l <= order; ++l) {
                pw *= ep;
                v += pw * terms[(int64_t)(l - 1) * nk + q];
            }
        }
        z0[p * pstride + j * ldz0 + c] = v;
    }
}

inline int grid_for(int64_t count) {
    int64_t b = (count + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

}  // namespace

hipError_t rs_clear(hipStream_t s, int32_t *err) {
    k_rs_clear<<<1, 1, 0, s>>>(err);
    return hipGetLastError();
}

hipError_t rs_gather(hipStream_t s, const double *delta, int64_t lda, const int32_t *idx, int64_t n, int64_t k,
                     double *y, int32_t *err) {
    k_rs_gather<<<grid_for(n * k), 256, 0, s>>>(delta, lda, idx, n, k, y, err);
    return hipGetLastError();
}

hipError_t rs_product(hipStream_t s, const double *delta, int64_t lda, const double *z, int64_t n, int64_t k,
                      double *y) {
    k_rs_product<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(delta, lda, z, n, k, y);
    return hipGetLastError();
}

hipError_t rs_term(hipStream_t s, const double *theta, const int32_t *idx, const double *y, double *terms, double *d,
                   int32_t l, int64_t n, int64_t k, int32_t *err) {
    k_rs_term<<<grid_for(n * k), 256, 0, s>>>(theta, idx, y, terms, d, l, n, k, err);
    return hipGetLastError();
}

hipError_t rs_start(hipStream_t s, const double *eps, int32_t count, int32_t order, const double *terms, int64_t n,
                    int64_t k, const int32_t *idx, double *z0, int64_t ldz0, int64_t pstride) {
    k_rs_start<<<grid_for((int64_t)count * n * k), 256, 0, s>>>(eps, count, order, terms, n, k, idx, z0, ldz0,
                                                                pstride);
    return hipGetLastError();
}

}  // namespace ipt
