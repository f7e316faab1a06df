// IPT-ACX (Sec. 5, Alg. 3): the extrapolation step that ends each cycle of
// alternating cyclic extrapolation.  After a cycle of order p the slots hold the
// cycle's base iterate z and F(z), ..., F^p(z) for every active column; with the
// forward differences
//   D^1 = F(z) - z,  D^2 = F^2(z) - 2F(z) + z,  D^3 = F^3(z) - 3F^2(z) + 3F(z) - z,
// each active column moves to z + sum_{q=1..p} binom(p, q) sigma^q D^q with
// sigma = |<D^p, D^(p-1)>| / |D^p|^2 (1 when D^p = 0).  Entry i of every iterate is 1,
// so every difference vanishes there and the chart z_i = 1 is kept exactly.
//
// Three launches: row-range partials of the two sums (fixed split, rows of a split
// summed in order, splits added in order), sigma per column, the elementwise update
// of z in place.  Rows are the slow index of the row-major slots, so lanes run over
// consecutive columns.
#include <math.h>

#include "ipt_internal.h"

namespace ipt {

namespace {

constexpr int ACX_MAX_SPLITS = 64;

__device__ inline void diffs(int32_t p, double z, double a, double b, double c, double &d1, double &d2,
                             double &d3) {
    d1 = a - z;
    d2 = (b - 2.0 * a) + z;
    d3 = p == 3 ? ((c - 3.0 * b) + 3.0 * a) - z : 0.0;
}

// Block: cw columns x (256 / cw) row groups of one row split (cw = 64, or the
// next power of two >= kc for narrow solves, so that few columns still fill the
// block); partial (dot, norm) per split and column, row groups added in order.
__global__ __launch_bounds__(256) void k_acx_dots(const Ctrl *ctrl, const int32_t *state, const double *z,
                                                  const double *f1, const double *f2, const double *f3, int64_t ld,
                                                  int64_t n, int64_t kc, int32_t p, int32_t cw, int64_t rows_per,
                                                  double *part) {
    if (ctrl->error || ctrl->done) return;
    __shared__ double sh[2][256];
    const int cx = threadIdx.x % cw, g = threadIdx.x / cw, ng = 256 / cw;
    const int64_t c = (int64_t)blockIdx.x * cw + cx;
    const bool act = c < kc && state[c] == COL_ACTIVE;
    double dot = 0.0, nrm = 0.0;
    if (act) {
        const int64_t r0 = (int64_t)blockIdx.y * rows_per;
        const int64_t r1 = r0 + rows_per < n ? r0 + rows_per : n;
        for (int64_t j = r0 + g; j < r1; j += ng) {
            const int64_t e = j * ld + c;
            double d1, d2, d3;
            diffs(p, z[e], f1[e], f2[e], p == 3 ? f3[e] : 0.0, d1, d2, d3);
            const double hi = p == 3 ? d3 : d2, lo = p == 3 ? d2 : d1;
            dot += hi * lo;
            nrm += hi * hi;
        }
    }
    sh[0][threadIdx.x] = dot;
    sh[1][threadIdx.x] = nrm;
    __syncthreads();
    if (g == 0 && c < kc) {
        double sd = 0.0, sn = 0.0;
        for (int q = 0; q < ng; ++q) {
            sd += sh[0][q * cw + cx];
            sn += sh[1][q * cw + cx];
        }
        part[((int64_t)blockIdx.y * kc + c) * 2] = sd;
        part[((int64_t)blockIdx.y * kc + c) * 2 + 1] = sn;
    }
}

__global__ void k_acx_sigma(const Ctrl *ctrl, const int32_t *state, const double *part, int32_t splits, int64_t kc,
                            double *sigma) {
    if (ctrl->error || ctrl->done) return;
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= kc || state[c] != COL_ACTIVE) return;
    double dot = 0.0, nrm = 0.0;
    for (int q = 0; q < splits; ++q) {
        dot += part[((int64_t)q * kc + c) * 2];
        nrm += part[((int64_t)q * kc + c) * 2 + 1];
    }
    sigma[c] = nrm > 0.0 ? fabs(dot) / nrm : 1.0;
}

__global__ void k_acx_update(const Ctrl *ctrl, const int32_t *state, double *z, const double *f1, const double *f2,
                             const double *f3, int64_t ld, int64_t n, int64_t kc, int32_t p, const double *sigma) {
    if (ctrl->error || ctrl->done) return;
    const int64_t total = n * kc;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = t / kc, c = t - j * kc;
        if (state[c] != COL_ACTIVE) continue;
        const int64_t e = j * ld + c;
        const double sg = sigma[c];
        double d1, d2, d3;
        const double zz = z[e];
        diffs(p, zz, f1[e], f2[e], p == 3 ? f3[e] : 0.0, d1, d2, d3);
        z[e] = p == 3 ? ((zz + 3.0 * sg * d1) + 3.0 * (sg * sg) * d2) + (sg * sg * sg) * d3
                      : (zz + 2.0 * sg * d1) + (sg * sg) * d2;
    }
}

}  // namespace

static int acx_cw(int64_t kc) {
    int cw = 1;
    while (cw < kc && cw < 64) cw <<= 1;
    return cw;
}

// Row splits: enough blocks to fill the chip (about 1024), at least 64 rows each.
int acx_splits(int64_t n, int64_t kc) {
    const int64_t col_blocks = (kc + acx_cw(kc) - 1) / acx_cw(kc);
    int64_t s = (1024 + col_blocks - 1) / col_blocks;
    const int64_t by_rows = (n + 63) / 64;
    if (s > by_rows) s = by_rows;
    if (s > ACX_MAX_SPLITS) s = ACX_MAX_SPLITS;
    return (int)(s < 1 ? 1 : s);
}

hipError_t launch_acx(hipStream_t s, const Ctrl *ctrl, const int32_t *state, double *z, const double *f1,
                      const double *f2, const double *f3, int64_t ld, int64_t n, int64_t kc, int32_t p, double *part,
                      double *sigma) {
    const int splits = acx_splits(n, kc);
    const int64_t rows_per = (n + splits - 1) / splits;
    const int cw = acx_cw(kc);
    dim3 g1((unsigned)((kc + cw - 1) / cw), (unsigned)splits);
    k_acx_dots<<<g1, 256, 0, s>>>(ctrl, state, z, f1, f2, f3, ld, n, kc, p, cw, rows_per, part);
    k_acx_sigma<<<(unsigned)((kc + 255) / 256), 256, 0, s>>>(ctrl, state, part, splits, kc, sigma);
    const int64_t total = n * kc;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_acx_update<<<(unsigned)(blocks > 0 ? blocks : 1), 256, 0, s>>>(ctrl, state, z, f1, f2, f3, ld, n, kc, p, sigma);
    return hipGetLastError();
}

}  // namespace ipt
