// Sparse IPT over C^n: Delta in CSR form with complex entries (the few-eigenpairs use
// of Sec. 6.1 for a complex M; Sec. 2 states the method over C^n).  The map and its
// bookkeeping are those of the real CSR sweep and of the dense complex sweep:
//   W_jc = (Z_jc d_c - Y_jc) / (theta_j - theta_i)  (j != i),  W_ic = 1,  Y = Delta Z,
//   d_c = Y_ic                                                      (eq. dyn)
// with complex arithmetic on (re, im) pairs of doubles (the gap inverted by Smith's
// method), the per-column partial sums |W - Z|^2, |Z|^2, |gap (W - Z)|^2, |W - e|^2 of
// each block of rows for the real finalize, and lambda_c = theta_i + d_c.
//
// Layout: Z is row-major n x ldz complex (ldz = k), so the k entries of a gathered row
// Z[col[p], :] are contiguous (16 k bytes).  kg lanes serve one row (kg = k rounded up
// to a power of two, at most 64), a lane owns one column (c, c + 64, ... when k > 64),
// and the row's entries are taken four at a time so that their gathers are in flight
// together; sums run in storage order.  FP64 only.
#include <math.h>

#include "ipt_internal.h"

namespace ipt {

namespace {

constexpr int ZSP_ROWS = 64;   // rows per block (one partial-sum row block)
constexpr int ZSP_GATHER = 4;  // entries of a row whose gathers are issued together

__device__ inline double2 zc_mul(double2 a, double2 b) { return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// 1/x by Smith's method (the larger component divides first), as the dense complex sweep
__device__ inline double2 zc_inv(double2 x) {
    if (fabs(x.x) >= fabs(x.y)) {
        const double q = x.y / x.x, den = x.x + x.y * q;
        return double2{1.0 / den, -q / den};
    }
    const double q = x.x / x.y, den = x.y + x.x * q;
    return double2{q / den, -1.0 / den};
}

__device__ inline double zc_abs2(double2 a) { return a.x * a.x + a.y * a.y; }

struct ZSpArgs {
    const int32_t *row_ptr, *col;
    const double2 *val;
    const double *th_re, *th_im;
    const double2 *zin;
    double2 *zout;
    ColState cs;
    double *d_re, *d_im;  // read (d of this sweep), or written by the product-free sweep
    double *part;         // [row block][k][NPART]
    int64_t n, k, ldz;
    int32_t kg;
};

// The per-column sums of the block's rows: the rows_per_pass lanes of a column (fixed
// xor pattern), then the four waves in order.
__device__ inline void zsp_store_sums(const ZSpArgs &a, double (*red)[64][NPART], double s0, double s1, double s2,
                                      double s3, int64_t c0) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int off = a.kg; off < 64; off <<= 1) {
        s0 += __shfl_xor(s0, off);
        s1 += __shfl_xor(s1, off);
        s2 += __shfl_xor(s2, off);
        s3 += __shfl_xor(s3, off);
    }
    if (lane < a.kg) {
        red[wv][lane][0] = s0;
        red[wv][lane][1] = s1;
        red[wv][lane][2] = s2;
        red[wv][lane][3] = s3;
    }
    __syncthreads();
    if (threadIdx.x < a.kg) {
        const int t = threadIdx.x;
        const int64_t cc = c0 + t;
        if (cc < a.k) {
#pragma unroll
            for (int q = 0; q < NPART; ++q)
                a.part[((int64_t)blockIdx.x * a.k + cc) * NPART + q] =
                    ((red[0][t][q] + red[1][t][q]) + red[2][t][q]) + red[3][t][q];
        }
    }
    __syncthreads();
}

// One product sweep: Y = Delta Z by rows (gathered rows of Z), the update and the sums.
__global__ __launch_bounds__(256) void k_zspmm_sweep(const Ctrl *ctrl, ZSpArgs a) {
    if (ctrl->error || ctrl->done) return;
    __shared__ double red[4][64][NPART];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int kg = a.kg, rows_per_pass = 64 / kg, sub = lane / kg, cl = lane % kg;
    const int64_t r0 = (int64_t)blockIdx.x * ZSP_ROWS;
    int64_t r1 = r0 + ZSP_ROWS;
    if (r1 > a.n) r1 = a.n;
    for (int64_t c0 = 0; c0 < a.k; c0 += 64) {
        const int64_t c = c0 + cl;
        const bool colok = c < a.k && a.cs.state[c] == COL_ACTIVE;
        const int32_t i = colok ? a.cs.idx[c] : 0;
        const double2 thi{a.th_re[i], a.th_im[i]};
        const double2 d = colok ? double2{a.d_re[c], a.d_im[c]} : double2{0.0, 0.0};
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int64_t jb = r0 + (int64_t)wv * rows_per_pass; jb < r1; jb += 4 * rows_per_pass) {
            const int64_t j = jb + sub;
            if (j >= r1 || !colok) continue;
            const int32_t pb = a.row_ptr[j], pe = a.row_ptr[j + 1];
            const double2 z = a.zin[j * a.ldz + c];
            const double2 thj{a.th_re[j], a.th_im[j]};
            double2 y{0.0, 0.0};
            for (int32_t p = pb; p < pe; p += ZSP_GATHER) {
                int32_t cq[ZSP_GATHER];
                double2 vq[ZSP_GATHER], zq[ZSP_GATHER];
#pragma unroll
                for (int u = 0; u < ZSP_GATHER; ++u) {
                    const bool in = p + u < pe;
                    cq[u] = in ? a.col[p + u] : (int32_t)j;  // past the row's end: row j again, term skipped
                    vq[u] = in ? a.val[p + u] : double2{0.0, 0.0};
                }
#pragma unroll
                for (int u = 0; u < ZSP_GATHER; ++u) zq[u] = a.zin[(int64_t)cq[u] * a.ldz + c];
#pragma unroll
                for (int u = 0; u < ZSP_GATHER; ++u)
                    if (p + u < pe) {
                        const double2 t = zc_mul(vq[u], zq[u]);
                        y.x += t.x;
                        y.y += t.y;
                    }
            }
            double2 w, st, gs, we;
            if (j == i) {
                w = double2{1.0, 0.0};
                st = double2{w.x - z.x, w.y - z.y};
                gs = double2{0.0, 0.0};
                we = double2{0.0, 0.0};
            } else {
                const double2 gap{thj.x - thi.x, thj.y - thi.y};
                const double2 zd = zc_mul(z, d);
                w = zc_mul(zc_inv(gap), double2{zd.x - y.x, zd.y - y.y});
                st = double2{w.x - z.x, w.y - z.y};
                gs = zc_mul(gap, st);
                we = w;
            }
            a.zout[j * a.ldz + c] = w;
            s0 += zc_abs2(st);
            s1 += zc_abs2(z);
            s2 += zc_abs2(gs);
            s3 += zc_abs2(we);
        }
        zsp_store_sums(a, red, s0, s1, s2, s3, c0);
    }
}

// The product-free first sweep of a cold start (Z = E): Y_jc is the sum of the entries
// (j, i = idx[c]) in storage order (no gathers); d_c = Delta_ii from row i itself.
__global__ __launch_bounds__(256) void k_zspmm_unit(const Ctrl *ctrl, ZSpArgs a) {
    if (ctrl->error || ctrl->done) return;
    __shared__ double red[4][64][NPART];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int kg = a.kg, rows_per_pass = 64 / kg, sub = lane / kg, cl = lane % kg;
    const int64_t r0 = (int64_t)blockIdx.x * ZSP_ROWS;
    int64_t r1 = r0 + ZSP_ROWS;
    if (r1 > a.n) r1 = a.n;
    for (int64_t c0 = 0; c0 < a.k; c0 += 64) {
        const int64_t c = c0 + cl;
        const bool colok = c < a.k && a.cs.state[c] == COL_ACTIVE;
        const int32_t i = colok ? a.cs.idx[c] : 0;
        const double2 thi{a.th_re[i], a.th_im[i]};
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int64_t jb = r0 + (int64_t)wv * rows_per_pass; jb < r1; jb += 4 * rows_per_pass) {
            const int64_t j = jb + sub;
            if (j >= r1 || !colok) continue;
            const int32_t pb = a.row_ptr[j], pe = a.row_ptr[j + 1];
            double2 y{0.0, 0.0};
            for (int32_t p = pb; p < pe; p += 8) {
                int32_t cq[8];
                double2 vq[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const bool in = p + u < pe;
                    cq[u] = in ? a.col[p + u] : -1;
                    vq[u] = in ? a.val[p + u] : double2{0.0, 0.0};
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (cq[u] == i) {
                        y.x += vq[u].x;
                        y.y += vq[u].y;
                    }
            }
            if (j == i) {
                a.d_re[c] = y.x;  // d_c = Delta_ii for this sweep's finalize
                a.d_im[c] = y.y;
                a.zout[j * a.ldz + c] = double2{1.0, 0.0};
                s1 += 1.0;  // |Z|^2 of e_i; W - Z and W - e vanish in row i
            } else {
                const double2 gap{a.th_re[j] - thi.x, a.th_im[j] - thi.y};
                const double2 w = zc_mul(zc_inv(gap), double2{-y.x, -y.y});  // (z d - y) / gap with z = 0
                const double2 gs = zc_mul(gap, w);
                a.zout[j * a.ldz + c] = w;
                s0 += zc_abs2(w);
                s2 += zc_abs2(gs);
                s3 += zc_abs2(w);
            }
        }
        zsp_store_sums(a, red, s0, s1, s2, s3, c0);
    }
}

// d_c = (Delta Z)_{i,c} = sum over row i of val[p] Z[col[p], c], one wave per column:
// lane-strided partial sums, then a fixed xor tree.
__global__ void k_zdiag_csr(const Ctrl *ctrl, const int32_t *row_ptr, const int32_t *col, const double2 *val,
                            const double2 *zin, int64_t ldz, ColState cs, double *d_re, double *d_im, int64_t k) {
    if (ctrl->error || ctrl->done) return;
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= k || cs.state[c] != COL_ACTIVE) return;
    const int32_t i = cs.idx[c];
    double re = 0.0, im = 0.0;
    for (int32_t p = row_ptr[i] + lane; p < row_ptr[i + 1]; p += 64) {
        const double2 t = zc_mul(val[p], zin[(int64_t)col[p] * ldz + c]);
        re += t.x;
        im += t.y;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_xor(re, off);
        im += __shfl_xor(im, off);
    }
    if (lane == 0) {
        d_re[c] = re;
        d_im[c] = im;
    }
}

inline unsigned zsp_blocks(int64_t count, int per) { return (unsigned)((count + per - 1) / per); }

}  // namespace

int64_t zspmm_row_blocks(int64_t n) { return (n + ZSP_ROWS - 1) / ZSP_ROWS; }

hipError_t launch_zspmm_sweep(hipStream_t s, const Ctrl *ctrl, const int32_t *row_ptr, const int32_t *col,
                              const double *val, const double *th_re, const double *th_im, const double *zin,
                              double *zout, ColState cs, double *d_re, double *d_im, double *part, int64_t n,
                              int64_t k, int64_t ldz, int32_t unit_in) {
    int kg = 1;
    while (kg < k && kg < 64) kg <<= 1;
    ZSpArgs a{row_ptr, col, (const double2 *)val, th_re, th_im, (const double2 *)zin, (double2 *)zout, cs, d_re,
              d_im, part, n, k, ldz, kg};
    if (unit_in)
        k_zspmm_unit<<<zsp_blocks(n, ZSP_ROWS), 256, 0, s>>>(ctrl, a);
    else
        k_zspmm_sweep<<<zsp_blocks(n, ZSP_ROWS), 256, 0, s>>>(ctrl, a);
    return hipGetLastError();
}

hipError_t launch_zdiag_csr(hipStream_t s, const Ctrl *ctrl, const int32_t *row_ptr, const int32_t *col,
                            const double *val, const double *zin, int64_t ldz, ColState cs, double *d_re,
                            double *d_im, int64_t k) {
    k_zdiag_csr<<<zsp_blocks(k, 4), 256, 0, s>>>(ctrl, row_ptr, col, (const double2 *)val, (const double2 *)zin,
                                                  ldz, cs, d_re, d_im, k);
    return hipGetLastError();
}

}  // namespace ipt
