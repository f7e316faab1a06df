// Dense IPT over C^n (the paper states the method for complex M, Sec. 2): theta,
// Delta and Z complex, the same map
//   W_jc = (Z_jc d_c - Y_jc) / (theta_j - theta_i)  (j != i),  W_ic = 1,  Y = Delta Z,
//   d_c = Y_ic                                                      (eq. dyn)
// the same per-column stopping test on the Euclidean norm of C^n and lambda_c =
// theta_i + d_c.  Complex numbers are (re, im) pairs of doubles (double2).
//
// The product is four real FP64 matrix-core products per tile, Re Y = Ar Br - Ai Bi
// and Im Y = Ar Bi + Ai Br (the minus folded into the Ai operand), with the update
// fused into the epilogue like the real sweep: the complex gap is inverted by
// Smith's method, and the per-column partial sums |W - Z|^2, |Z|^2, |gap (W - Z)|^2,
// |W - e|^2 of each 64-row tile go to the same finalize as the real path.  d comes
// from a separate pass over the rows idx[c] of Delta.  A cold start's first sweep
// needs no product (k_zsweep1).
#include <math.h>

#include "ipt_internal.h"

namespace ipt {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int ZT = 64;  // rows and columns of a complex sweep tile (4 waves of 32 x 32)
constexpr int ZK = 16;  // complex elements of K per LDS stage
constexpr int ZCH = 32; // row chunks of the |M|_1 column sums

__device__ inline double2 cmul(double2 a, double2 b) {
    return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// 1/x by Smith's method (the larger component divides first)
__device__ inline double2 cinv(double2 x) {
    if (fabs(x.x) >= fabs(x.y)) {
        const double q = x.y / x.x, den = x.x + x.y * q;
        return double2{1.0 / den, -q / den};
    }
    const double q = x.x / x.y, den = x.y + x.x * q;
    return double2{q / den, -1.0 / den};
}

__device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

__device__ inline uint64_t zbits(double v) { return (uint64_t)__double_as_longlong(v); }

__device__ inline void zblock_max(uint64_t *p, uint64_t v) {
    __shared__ uint64_t wm[4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = (uint64_t)__shfl_xor((unsigned long long)v, off);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t m = 0;
        for (int w = 0; w < 4; ++w) m = wm[w] > m ? wm[w] : m;
        if (m) atomicMax((unsigned long long *)p, (unsigned long long)m);
    }
}

struct ZArgs {
    const double2 *delta;  // n x n row-major, leading dimension lda
    int64_t lda;
    const double *th_re, *th_im;
    const double2 *zin;  // np x kp row-major
    double2 *zout;
    ColState cs;
    const double *d_re, *d_im;
    double *part;  // [row tile of ZT][kp][NPART]
    int64_t n, np, kp;
};

// Block: a 64-row tile of Delta x a tile of 64 packed active columns; wave (wm, wn)
// owns 32 x 32 outputs as 2 x 2 blocks of 16 x 16.  Tiles past the packed columns
// return at once (the grid covers every column tile).
__global__ __launch_bounds__(256, 2) void k_zsweep(const Ctrl *ctrl, ZArgs g) {
    if (ctrl->error || ctrl->done) return;
    const int ntm = (int)(g.np / ZT);
    const int tm = (int)(blockIdx.x % ntm), tn = (int)(blockIdx.x / ntm);
    const int32_t kact = ctrl->kact;
    if ((int64_t)tn * ZT >= kact) return;
    const int32_t lim = kact - tn * ZT;  // packed columns of this tile
    __shared__ double Ar[2][ZT][ZK + 1], Ai[2][ZT][ZK + 1];
    __shared__ double Br[2][ZK][ZT + 1], Bi[2][ZK][ZT + 1];
    __shared__ double red[2][ZT][NPART];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, wm = wv >> 1, wn = wv & 1;
    // loaders: A row t/4 and K elements 4 (t % 4) .. +3; B column t % 64 and K rows
    // 4 (t / 64) .. +3 (one 16-byte complex per element)
    const int a_r = t >> 2, a_k = (t & 3) * 4;
    const int b_c = t & 63, b_k = (t >> 6) * 4;
    const int64_t arow = (int64_t)tm * ZT + a_r;
    const int32_t bcol = b_c < lim ? g.cs.alist[(int64_t)tn * ZT + b_c] : -1;
    const double2 zero2{0.0, 0.0};
    double2 ra[4], rb[4];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t ka = k0 + a_k + u, kb = k0 + b_k + u;
            ra[u] = (arow < g.n && ka < g.n) ? g.delta[arow * g.lda + ka] : zero2;
            rb[u] = (bcol >= 0 && kb < g.n) ? g.zin[kb * g.kp + bcol] : zero2;
        }
    };
    auto put = [&](int s) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            Ar[s][a_r][a_k + u] = ra[u].x;
            Ai[s][a_r][a_k + u] = ra[u].y;
            Br[s][b_k + u][b_c] = rb[u].x;
            Bi[s][b_k + u][b_c] = rb[u].y;
        }
    };
    d4_t are[2][2], aim[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            are[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
            aim[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
        }
    const int nk = (int)(g.np / ZK);
    load(0);
    put(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        // the last iteration re-reads its own slice into the idle stage (no branch)
        load((int64_t)(kt + 1 < nk ? kt + 1 : kt) * ZK);
#pragma unroll
        for (int s4 = 0; s4 < ZK / 4; ++s4) {
            const int kk = 4 * s4 + (lane >> 4);
            double far[2], fai[2], fbr[2], fbi[2];
#pragma unroll
            for (int ib = 0; ib < 2; ++ib) {
                const int r = wm * 32 + 16 * ib + (lane & 15);
                far[ib] = Ar[cur][r][kk];
                fai[ib] = Ai[cur][r][kk];
            }
#pragma unroll
            for (int jb = 0; jb < 2; ++jb) {
                const int cc = wn * 32 + 16 * jb + (lane & 15);
                fbr[jb] = Br[cur][kk][cc];
                fbi[jb] = Bi[cur][kk][cc];
            }
#pragma unroll
            for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                for (int jb = 0; jb < 2; ++jb) {
                    are[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(far[ib], fbr[jb], are[ib][jb], 0, 0, 0);
                    are[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-fai[ib], fbi[jb], are[ib][jb], 0, 0, 0);
                    aim[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(far[ib], fbi[jb], aim[ib][jb], 0, 0, 0);
                    aim[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(fai[ib], fbr[jb], aim[ib][jb], 0, 0, 0);
                }
        }
        put(cur ^ 1);
        __syncthreads();
    }

    // Epilogue.  v_mfma_f64_16x16x4f64: lane l, register r holds row 4r + l/16 and
    // column l%16 of a 16 x 16 block.
    double sum[2][NPART];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int q = 0; q < NPART; ++q) sum[jb][q] = 0.0;
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
        const int x = wn * 32 + 16 * jb + (lane & 15);  // packed position in the tile
        if (x >= lim) continue;
        const int32_t c = g.cs.alist[(int64_t)tn * ZT + x];
        const int32_t i = g.cs.idx[c];
        const double2 d{g.d_re[c], g.d_im[c]};
        const double2 thi{g.th_re[i], g.th_im[i]};
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t j = (int64_t)tm * ZT + wm * 32 + 16 * ib + 4 * r + (lane >> 4);
                if (j >= g.n) continue;
                const double2 y{are[ib][jb][r], aim[ib][jb][r]};
                const double2 z = g.zin[j * g.kp + c];
                double2 w, st, gs, we;
                if (j == i) {
                    w = double2{1.0, 0.0};
                    st = double2{w.x - z.x, w.y - z.y};
                    gs = zero2;
                    we = zero2;
                } else {
                    const double2 gap{g.th_re[j] - thi.x, g.th_im[j] - thi.y};
                    const double2 zd = cmul(z, d);
                    w = cmul(cinv(gap), double2{zd.x - y.x, zd.y - y.y});
                    st = double2{w.x - z.x, w.y - z.y};
                    gs = cmul(gap, st);
                    we = w;
                }
                g.zout[j * g.kp + c] = w;
                sum[jb][0] += cabs2(st);
                sum[jb][1] += cabs2(z);
                sum[jb][2] += cabs2(gs);
                sum[jb][3] += cabs2(we);
            }
    }
    // the four lane groups that share a column, in a fixed pattern, then the two
    // row halves of the tile in order
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int q = 0; q < NPART; ++q) {
            sum[jb][q] += __shfl_xor(sum[jb][q], 16);
            sum[jb][q] += __shfl_xor(sum[jb][q], 32);
        }
    if (lane < 16) {
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int q = 0; q < NPART; ++q) red[wm][wn * 32 + 16 * jb + lane][q] = sum[jb][q];
    }
    __syncthreads();
    if (t < ZT && t < lim) {
        const int32_t c = g.cs.alist[(int64_t)tn * ZT + t];
#pragma unroll
        for (int q = 0; q < NPART; ++q) g.part[((int64_t)tm * g.kp + c) * NPART + q] = red[0][t][q] + red[1][t][q];
    }
}

// Product-free first sweep of a cold start: from Z = E, Delta Z is the gather of
// the columns idx[c] of Delta (exact), so W = E - G o Delta on the requested columns
// and d_c = Delta_ii.  Block: 64 columns x 4 row lanes over one 64-row tile; the
// per-column partial sums of the tile, lanes added in order.
__global__ __launch_bounds__(256) void k_zsweep1(const Ctrl *ctrl, const double2 *delta, int64_t lda,
                                                 const double *th_re, const double *th_im, ColState cs, double *d_re,
                                                 double *d_im, double2 *zout, int64_t kp, double *part, int64_t n) {
    if (ctrl->error || ctrl->done) return;
    __shared__ double red[4][64][NPART];
    const int cx = threadIdx.x & 63, gr = threadIdx.x >> 6;
    const int64_t c = (int64_t)blockIdx.x * 64 + cx;
    const int64_t tm = blockIdx.y;
    const bool act = c < kp && cs.state[c] == COL_ACTIVE;
    double sm[NPART] = {0.0, 0.0, 0.0, 0.0};
    if (act) {
        const int32_t i = cs.idx[c];
        const double2 thi{th_re[i], th_im[i]};
        int64_t j1 = (tm + 1) * ZT;
        if (j1 > n) j1 = n;
        for (int64_t j = tm * ZT + gr; j < j1; j += 4) {
            const double2 dji = delta[j * lda + i];
            if (j == i) {
                zout[j * kp + c] = double2{1.0, 0.0};
                sm[1] += 1.0;  // |Z|^2 of e_i; W - Z and W - e vanish in row i
                d_re[c] = dji.x;
                d_im[c] = dji.y;
            } else {
                const double2 gap{th_re[j] - thi.x, th_im[j] - thi.y};
                const double2 w = cmul(cinv(gap), double2{-dji.x, -dji.y});
                const double2 gs = cmul(gap, w);
                zout[j * kp + c] = w;
                sm[0] += cabs2(w);  // W - Z with Z_jc = 0
                sm[2] += cabs2(gs);
                sm[3] += cabs2(w);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NPART; ++q) red[gr][cx][q] = sm[q];
    __syncthreads();
    if (gr == 0 && act) {
#pragma unroll
        for (int q = 0; q < NPART; ++q)
            part[(tm * kp + c) * NPART + q] = ((red[0][cx][q] + red[1][cx][q]) + red[2][cx][q]) + red[3][cx][q];
    }
}

// d_c = (Delta Z)_{i,c} for the active columns, in two passes: per chunk of rows,
// block = 64 columns x 4 row lanes (lane g sums rows g, g + 4, ... of the chunk, the
// lanes added in order) into dpart[chunk][c]; then the chunks in order.
constexpr int ZDCH = 16;

__global__ __launch_bounds__(256) void k_zdiag_part(const Ctrl *ctrl, const double2 *delta, int64_t lda,
                                                    const double2 *zin, int64_t kp, ColState cs, double2 *dpart,
                                                    int64_t n) {
    if (ctrl->error || ctrl->done) return;
    __shared__ double2 sh[4][64];
    const int cx = threadIdx.x & 63, gr = threadIdx.x >> 6;
    const int64_t c = (int64_t)blockIdx.x * 64 + cx;
    const bool act = c < kp && cs.state[c] == COL_ACTIVE;
    const int64_t per = (n + ZDCH - 1) / ZDCH;
    const int64_t j0 = (int64_t)blockIdx.y * per;
    int64_t j1 = j0 + per;
    if (j1 > n) j1 = n;
    double2 acc{0.0, 0.0};
    if (act) {
        const double2 *row = delta + (int64_t)cs.idx[c] * lda;
        for (int64_t j = j0 + gr; j < j1; j += 4) {
            const double2 p = cmul(row[j], zin[j * kp + c]);
            acc.x += p.x;
            acc.y += p.y;
        }
    }
    sh[gr][cx] = acc;
    __syncthreads();
    if (gr == 0 && act)
        dpart[blockIdx.y * kp + c] = double2{((sh[0][cx].x + sh[1][cx].x) + sh[2][cx].x) + sh[3][cx].x,
                                             ((sh[0][cx].y + sh[1][cx].y) + sh[2][cx].y) + sh[3][cx].y};
}

__global__ void k_zdiag_reduce(const Ctrl *ctrl, ColState cs, const double2 *dpart, double *d_re, double *d_im,
                               int64_t kp) {
    if (ctrl->error || ctrl->done) return;
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= kp || cs.state[c] != COL_ACTIVE) return;
    double re = 0.0, im = 0.0;
    for (int q = 0; q < ZDCH; ++q) {
        re += dpart[q * kp + c].x;
        im += dpart[q * kp + c].y;
    }
    d_re[c] = re;
    d_im[c] = im;
}

// theta split into planes; a non-finite theta is IPT_EINVAL.
__global__ void k_zprep_theta(Ctrl *ctrl, const double2 *theta, double *th_re, double *th_im, int64_t n) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double2 v = theta[j];
    th_re[j] = v.x;
    th_im[j] = v.y;
    if (!isfinite(v.x) || !isfinite(v.y)) atomicMax(&ctrl->error, (int32_t)IPT_EINVAL);
}

// theta_j == theta_i (both parts) for a requested i and j != i: the inverse gap is
// undefined (IPT_EDEGENERATE).  Block per (requested column, chunk of rows), so that a
// few requested columns of a long theta still spread over the chip.
__global__ void k_zcheck_gaps(Ctrl *ctrl, const double *th_re, const double *th_im, const int32_t *idx, int64_t n,
                              int64_t k, int64_t chunk) {
    if (ctrl->error) return;
    const int64_t c = blockIdx.x;
    if (c >= k) return;
    const int32_t i = idx[c];
    const double a = th_re[i], b = th_im[i];
    const int64_t j0 = (int64_t)blockIdx.y * chunk;
    const int64_t j1 = j0 + chunk < n ? j0 + chunk : n;
    bool bad = false;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) bad |= (j != i) && th_re[j] == a && th_im[j] == b;
    if (bad) atomicMax(&ctrl->error, (int32_t)IPT_EDEGENERATE);
}

// |M|_1 = max_c sum_j |M_jc|, M = diag(theta) + Delta: per row chunk, block = 64
// columns x 4 row lanes (coalesced rows), partial sums part2[chunk][c]; then the
// chunks in order and the maximum.
__global__ __launch_bounds__(256) void k_znorm_part(const Ctrl *ctrl, const double2 *delta, int64_t lda,
                                                    const double *th_re, const double *th_im, int64_t n,
                                                    double *part2) {
    if (ctrl->error) return;
    __shared__ double sh[4][64];
    const int cx = threadIdx.x & 63, gr = threadIdx.x >> 6;
    const int64_t c = (int64_t)blockIdx.x * 64 + cx;
    const int64_t per = (n + ZCH - 1) / ZCH;
    const int64_t j0 = (int64_t)blockIdx.y * per;
    int64_t j1 = j0 + per;
    if (j1 > n) j1 = n;
    double acc = 0.0;
    if (c < n)
        for (int64_t j = j0 + gr; j < j1; j += 4) {
            double2 v = delta[j * lda + c];
            if (j == c) {
                v.x += th_re[c];
                v.y += th_im[c];
            }
            acc += sqrt(cabs2(v));
        }
    sh[gr][cx] = acc;
    __syncthreads();
    if (gr == 0 && c < n) part2[blockIdx.y * n + c] = ((sh[0][cx] + sh[1][cx]) + sh[2][cx]) + sh[3][cx];
}

__global__ __launch_bounds__(256) void k_znorm_max(Ctrl *ctrl, const double *part2, int64_t n) {
    if (ctrl->error) return;
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double s = 0.0;
    if (c < n)
        for (int q = 0; q < ZCH; ++q) s += part2[q * n + c];
    zblock_max(&ctrl->norm1_bits, zbits(s));
}

// Z <- z0 with Z[idx[c], c] = 1 (chart z_i = 1), or Z <- E; padding zero.
__global__ void k_zload(const Ctrl *ctrl, const double2 *z0, int64_t ldz0, double2 *zb, int64_t kp,
                        const int32_t *idx, int64_t n, int64_t np, int64_t k) {
    if (ctrl->error) return;
    const int64_t total = np * kp;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / kp, c = e - j * kp;
        double2 v{0.0, 0.0};
        if (j < n && c < k) {
            if (j == idx[c]) v = double2{1.0, 0.0};
            else if (z0) v = z0[j * ldz0 + c];
        }
        zb[e] = v;
    }
}

// Certified (or last) iterates, eigenvalues and statuses to the caller's arrays.
// Block: cw columns x 256 / cw row lanes over 64-row chunks.
__global__ __launch_bounds__(256) void k_zcopyout(const Ctrl *ctrl, ColState cs, const double2 *buf0,
                                                  const double2 *buf1, int64_t kp, double2 *z_out, int64_t ldz,
                                                  const double *lam_im, double2 *lambda_out, int32_t *status_out,
                                                  int64_t n, int64_t k, int32_t cw, int32_t *ci_sweeps,
                                                  double *ci_step, double *ci_resid) {
    if (ctrl->error) return;
    const int rl = threadIdx.x / cw, rstep = 256 / cw;
    const int64_t c = blockIdx.x * (int64_t)cw + (threadIdx.x % cw);
    if (c >= k) return;
    const int32_t par = cs.par[c];
    const int32_t i = cs.idx[c];
    const double2 *src = (par == PAR_BUF1) ? buf1 : buf0;
    for (int64_t jb = (int64_t)blockIdx.y * 64; jb < n; jb += (int64_t)gridDim.y * 64) {
        int64_t j1 = jb + 64;
        if (j1 > n) j1 = n;
        for (int64_t j = jb + rl; j < j1; j += rstep)
            z_out[j * ldz + c] = (par == PAR_UNIT) ? double2{j == i ? 1.0 : 0.0, 0.0} : src[j * kp + c];
    }
    if (blockIdx.y == 0 && rl == 0) {
        lambda_out[c] = double2{cs.lam[c], lam_im[c]};
        const int32_t st = cs.state[c];
        status_out[c] = (st == COL_ACTIVE) ? IPT_NOT_CONVERGED : st;
        if (ci_sweeps) ci_sweeps[c] = cs.sweeps[c];
        if (ci_step) ci_step[c] = cs.step[c];
        if (ci_resid) ci_resid[c] = cs.resid[c];
    }
}

inline unsigned zblocks(int64_t count, int per) { return (unsigned)((count + per - 1) / per); }

}  // namespace

hipError_t launch_zsetup(hipStream_t s, Ctrl *ctrl, const double *theta, const double *delta, int64_t lda,
                         double *th_re, double *th_im, double *part2, int64_t n) {
    k_zprep_theta<<<zblocks(n, 256), 256, 0, s>>>(ctrl, (const double2 *)theta, th_re, th_im, n);
    if (part2) {
        k_znorm_part<<<dim3(zblocks(n, 64), ZCH), 256, 0, s>>>(ctrl, (const double2 *)delta, lda, th_re, th_im, n,
                                                                 part2);
        k_znorm_max<<<zblocks(n, 256), 256, 0, s>>>(ctrl, part2, n);
    }
    return hipGetLastError();
}

int64_t zsetup_part2_doubles(int64_t n) { return (int64_t)ZCH * n; }

hipError_t launch_zcheck_gaps(hipStream_t s, Ctrl *ctrl, const double *th_re, const double *th_im, const int32_t *idx,
                              int64_t n, int64_t k) {
    int64_t chunk = 4096;  // 16 rows per thread
    if ((n + chunk - 1) / chunk > 65535) chunk = (n + 65534) / 65535;
    const dim3 g((unsigned)k, (unsigned)((n + chunk - 1) / chunk));
    k_zcheck_gaps<<<g, 256, 0, s>>>(ctrl, th_re, th_im, idx, n, k, chunk);
    return hipGetLastError();
}

hipError_t launch_zload(hipStream_t s, const Ctrl *ctrl, const double *z0, int64_t ldz0, double *zb, int64_t kp,
                        const int32_t *idx, int64_t n, int64_t np, int64_t k) {
    unsigned b = zblocks(np * kp, 256);
    if (b > 8192) b = 8192;
    k_zload<<<b, 256, 0, s>>>(ctrl, (const double2 *)z0, ldz0, (double2 *)zb, kp, idx, n, np, k);
    return hipGetLastError();
}

int64_t zdiag_part_doubles(int64_t kp) { return 2 * (int64_t)ZDCH * kp; }

hipError_t launch_zdiag(hipStream_t s, const Ctrl *ctrl, const double *delta, int64_t lda, const double *zin,
                        int64_t kp, ColState cs, double *dpart, double *d_re, double *d_im, int64_t n) {
    k_zdiag_part<<<dim3(zblocks(kp, 64), ZDCH), 256, 0, s>>>(ctrl, (const double2 *)delta, lda,
                                                              (const double2 *)zin, kp, cs, (double2 *)dpart, n);
    k_zdiag_reduce<<<zblocks(kp, 256), 256, 0, s>>>(ctrl, cs, (const double2 *)dpart, d_re, d_im, kp);
    return hipGetLastError();
}

int64_t zsweep_tile() { return ZT; }

hipError_t launch_zsweep1(hipStream_t s, const Ctrl *ctrl, const double *delta, int64_t lda, const double *th_re,
                          const double *th_im, ColState cs, double *d_re, double *d_im, double *zout, int64_t kp,
                          double *part, int64_t n, int64_t np) {
    k_zsweep1<<<dim3(zblocks(kp, 64), (unsigned)(np / ZT)), 256, 0, s>>>(
        ctrl, (const double2 *)delta, lda, th_re, th_im, cs, d_re, d_im, (double2 *)zout, kp, part, n);
    return hipGetLastError();
}

hipError_t launch_zsweep(hipStream_t s, const Ctrl *ctrl, const double *delta, int64_t lda, const double *th_re,
                         const double *th_im, const double *zin, double *zout, ColState cs, const double *d_re,
                         const double *d_im, double *part, int64_t n, int64_t np, int64_t kp) {
    ZArgs a{(const double2 *)delta, lda, th_re, th_im, (const double2 *)zin, (double2 *)zout, cs, d_re, d_im,
            part, n, np, kp};
    k_zsweep<<<(unsigned)((np / ZT) * (kp / ZT)), 256, 0, s>>>(ctrl, a);
    return hipGetLastError();
}

hipError_t launch_zcopyout(hipStream_t s, const Ctrl *ctrl, ColState cs, const double *buf0, const double *buf1,
                           int64_t kp, double *z_out, int64_t ldz, const double *lam_im, double *lambda_out,
                           int32_t *status_out, int64_t n, int64_t k, const ipt_colinfo *ci) {
    const unsigned gy = zblocks(n, 64) < 65535 ? zblocks(n, 64) : 65535;
    int32_t cw = 1;
    while (cw < 256 && cw < k) cw <<= 1;
    k_zcopyout<<<dim3(zblocks(k, cw), gy), 256, 0, s>>>(
        ctrl, cs, (const double2 *)buf0, (const double2 *)buf1, kp, (double2 *)z_out, ldz, lam_im,
        (double2 *)lambda_out, status_out, n, k, cw, ci ? ci->sweeps : nullptr, ci ? ci->step : nullptr,
        ci ? ci->resid : nullptr);
    return hipGetLastError();
}

}  // namespace ipt
