// The choice of D per near-degenerate pair (the concluding section's suggestion of
// using the freedom in D to widen the domain of convergence), as a similarity of M.
//
// Pairing: r_ik = |Delta_ik| / |theta_i - theta_k| (k != i) is the coupling of i and k
// relative to their gap.  i and j = argmax_k r_ik (the first index on ties) form a pair
// when i is also the argmax for j, r_ij > tau and Delta_ij == Delta_ji (a symmetric
// 2x2 block).  Each pair's block of M = diag(theta) + Delta is diagonalized by the
// rotation J = [[c, s], [-s, c]] (symmetric Schur decomposition, |angle| <= pi/4); R
// is the product of the pairs' rotations and M' = R^T M R.  The new partition keeps
// every unpaired theta_k and Delta_kk; a pair takes the diagonal of its rotated block
// as theta', and its coupling leaves Delta'.  IPT then runs on (theta', Delta'), whose
// near-degenerate pairs are gone, and its eigenvectors map back as z = R z'.  The
// level shifts then move into D as well: first order (diag Delta) and second order
// (the RS energy shift), so that two levels whose shifts differ by more than their gap
// no longer make the fixed point repelling; the matrix is unchanged (theta' + Delta'
// on the diagonal is the rotated M's, to the rounding of theta').
#include <math.h>

#include "ipt_internal.h"

namespace ipt {

namespace {

// Per problem b: rows of Delta_b (n_b x n_b row-major at doff[b]), theta_b at toff[b].
struct PairMeta {
    const int32_t *n;
    const int64_t *toff, *doff;
};

// One wave per row r of problem blockIdx.y: best[toff + r] = argmax_k r_rk (first on
// ties), rmax[toff + r] = its ratio (-1 when n = 1); the row is also copied to dp (the
// copy that k_pair_rotate re-partitions), at the same offset.
__global__ __launch_bounds__(256) void k_pair_best(PairMeta m, const double *theta, const double *delta,
                                                   int32_t *best, double *rmax, double *dp) {
    const int b = blockIdx.y;
    const int n = m.n[b];
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n) return;
    const double *th = theta + m.toff[b];
    const double *row = delta + m.doff[b] + (int64_t)r * n;
    double *out = dp + m.doff[b] + (int64_t)r * n;
    const double tr = th[r];
    double bv = -1.0;
    int bk = r;
    for (int k = lane; k < n; k += 64) {
        const double x = row[k];
        out[k] = x;
        if (k == r) continue;
        const double v = fabs(x) / fabs(tr - th[k]);
        if (v > bv) {  // k rises: the first index among equal values stays
            bv = v;
            bk = k;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off);
        const int ok = __shfl_xor(bk, off);
        if (ov > bv || (ov == bv && ok < bk)) {
            bv = ov;
            bk = ok;
        }
    }
    if (lane == 0) {
        best[m.toff[b] + r] = bk;
        rmax[m.toff[b] + r] = bv;
    }
}

__device__ inline void jacobi_cs(double a, double b, double d, double &c, double &s) {
    if (b == 0.0) {
        c = 1.0;
        s = 0.0;
        return;
    }
    const double zeta = (d - a) / (2.0 * b);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    c = 1.0 / sqrt(1.0 + t * t);
    s = t * c;
}

// One block per problem: pairs, rotation coefficients, then M' = R^T M R on the copy
// (dp = Delta' at doff[b], tp = theta' at toff[b]; both hold the input on entry):
// columns first, then rows; pairs are disjoint, so their rotations commute within
// each pass; then the level shifts.  partner[toff + r] = j or -1;
// cs[2 (toff + r) + 0/1] = c, s.
__global__ __launch_bounds__(256) void k_pair_rotate(PairMeta m, double *tp, double *dp, const int32_t *best,
                                                     const double *rmax, int32_t *partner, double *cs, double tau,
                                                     double *th2) {
    __shared__ int32_t list[2048];
    __shared__ int32_t count;
    const int b = blockIdx.x;
    const int n = m.n[b];
    const int64_t to = m.toff[b];
    double *D = dp + m.doff[b];
    double *th = tp + to;
    if (threadIdx.x == 0) count = 0;
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        const int j = best[to + r];
        const bool pair = n > 1 && j != r && best[to + j] == r && rmax[to + r] > tau &&
                          D[(int64_t)r * n + j] == D[(int64_t)j * n + r];
        partner[to + r] = pair ? j : -1;
        double c = 1.0, s = 0.0;
        if (pair) {
            const int i = r < j ? r : j, k = r < j ? j : r;
            jacobi_cs(th[i] + D[(int64_t)i * n + i], D[(int64_t)i * n + k], th[k] + D[(int64_t)k * n + k], c, s);
            if (r < j) list[atomicAdd(&count, 1)] = r;
        }
        cs[2 * (to + r)] = c;
        cs[2 * (to + r) + 1] = s;
    }
    __syncthreads();
    const int np_ = count;
    // a pair's diagonal entries of Delta' carry M's (theta added) while it rotates
    for (int q = threadIdx.x; q < np_; q += blockDim.x) {
        const int i = list[q], j = partner[to + i];
        D[(int64_t)i * n + i] += th[i];
        D[(int64_t)j * n + j] += th[j];
    }
    __syncthreads();
    for (int q = 0; q < np_; ++q) {  // columns: X <- X R
        const int i = list[q], j = partner[to + i];
        const double c = cs[2 * (to + i)], s = cs[2 * (to + i) + 1];
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            const double xi = D[(int64_t)k * n + i], xj = D[(int64_t)k * n + j];
            D[(int64_t)k * n + i] = c * xi - s * xj;
            D[(int64_t)k * n + j] = s * xi + c * xj;
        }
    }
    __syncthreads();
    for (int q = 0; q < np_; ++q) {  // rows: X <- R^T X
        const int i = list[q], j = partner[to + i];
        const double c = cs[2 * (to + i)], s = cs[2 * (to + i) + 1];
        for (int l = threadIdx.x; l < n; l += blockDim.x) {
            const double xi = D[(int64_t)i * n + l], xj = D[(int64_t)j * n + l];
            D[(int64_t)i * n + l] = c * xi - s * xj;
            D[(int64_t)j * n + l] = s * xi + c * xj;
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < np_; q += blockDim.x) {  // the pair's block leaves Delta'
        const int i = list[q], j = partner[to + i];
        th[i] = D[(int64_t)i * n + i];
        th[j] = D[(int64_t)j * n + j];
        D[(int64_t)i * n + i] = 0.0;
        D[(int64_t)j * n + j] = 0.0;
        D[(int64_t)i * n + j] = 0.0;
        D[(int64_t)j * n + i] = 0.0;
    }
    __syncthreads();
    // first-order level shift into D: theta2 = theta + diag(Delta) (k_level_shift adds
    // the second order)
    for (int k = threadIdx.x; k < n; k += blockDim.x) th2[to + k] = th[k] + D[(int64_t)k * n + k];
}

// Second-order level shift into D, one block per 32-row tile I of problem blockIdx.y:
// s_i = sum_{k != i} Delta_ik Delta_ki / (theta2_i - theta2_k) over the rotated Delta
// (terms with a zero product are 0), then theta'_i = theta2_i + s_i, Delta'_ii = -s_i.
// The products pair D[I, K] with D[K, I]: both 32 x 32 tiles come in row by row
// through LDS.  Only this block touches its rows' theta' and diagonal entries; every
// block reads theta2, and the diagonal entries only for terms it skips.
__global__ __launch_bounds__(256) void k_level_shift(PairMeta m, double *tp, double *dp, const double *th2) {
    __shared__ double ta[32][33], tb[32][33];
    const int b = blockIdx.y;
    const int n = m.n[b];
    const int i0 = blockIdx.x * 32;
    if (i0 >= n) return;
    const int64_t to = m.toff[b];
    double *D = dp + m.doff[b];
    const double *t2 = th2 + to;
    const int tr = threadIdx.x >> 3, tk = (threadIdx.x & 7) * 4;  // row of the tile, 4 columns
    const int i = i0 + tr;
    const double ti = i < n ? t2[i] : 0.0;
    double acc = 0.0;
    for (int k0 = 0; k0 < n; k0 += 32) {
        for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) {
            const int a = e >> 5, c = e & 31;
            ta[a][c] = (i0 + a < n && k0 + c < n) ? D[(int64_t)(i0 + a) * n + k0 + c] : 0.0;  // D[I, K]
            tb[a][c] = (k0 + a < n && i0 + c < n) ? D[(int64_t)(k0 + a) * n + i0 + c] : 0.0;  // D[K, I]
        }
        __syncthreads();
        if (i < n) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = k0 + tk + u;
                const double p = ta[tr][tk + u] * tb[tk + u][tr];
                if (k < n && k != i && p != 0.0) acc += p / (ti - t2[k]);
            }
        }
        __syncthreads();
    }
    // the 8 threads of a row are consecutive lanes
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    acc += __shfl_xor(acc, 4);
    if ((threadIdx.x & 7) == 0 && i < n) {
        tp[to + i] = ti + acc;
        D[(int64_t)i * n + i] = -acc;
    }
}

// Rows i < j of each pair of problem blockIdx.x in z (ncols[b] columns, leading
// dimension ldz[b], at zoff[b]): z = R z' (forward = 0) or z' = R^T z (forward = 1).
__global__ __launch_bounds__(256) void k_pair_rows(PairMeta m, const int64_t *zoff, const int64_t *ldz,
                                                   const int32_t *ncols, double *z, const int32_t *partner,
                                                   const double *cs, int32_t forward) {
    const int b = blockIdx.x;
    const int n = m.n[b];
    const int64_t to = m.toff[b];
    double *Z = z + zoff[b];
    const int64_t ld = ldz[b];
    const int kc = ncols[b];
    for (int i = 0; i < n; ++i) {
        const int j = partner[to + i];
        if (j <= i) continue;  // uniform across the block
        const double c = cs[2 * (to + i)], s = forward ? -cs[2 * (to + i) + 1] : cs[2 * (to + i) + 1];
        for (int l = threadIdx.x; l < kc; l += blockDim.x) {
            const double zi = Z[(int64_t)i * ld + l], zj = Z[(int64_t)j * ld + l];
            Z[(int64_t)i * ld + l] = c * zi + s * zj;
            Z[(int64_t)j * ld + l] = -s * zi + c * zj;
        }
    }
}

}  // namespace

hipError_t launch_pair_rotate(hipStream_t s, int32_t count, int32_t max_n, const int32_t *n, const int64_t *toff,
                              const int64_t *doff, const double *theta, const double *delta, double *tp, double *dp,
                              int32_t *best, double *rmax, int32_t *partner, double *cs, double tau, double *th2) {
    const PairMeta m{n, toff, doff};
    dim3 g((unsigned)((max_n + 3) / 4), (unsigned)count);
    k_pair_best<<<g, 256, 0, s>>>(m, theta, delta, best, rmax, dp);
    k_pair_rotate<<<(unsigned)count, 256, 0, s>>>(m, tp, dp, best, rmax, partner, cs, tau, th2);
    k_level_shift<<<dim3((unsigned)((max_n + 31) / 32), (unsigned)count), 256, 0, s>>>(m, tp, dp, th2);
    return hipGetLastError();
}

hipError_t launch_pair_rows(hipStream_t s, int32_t count, const int32_t *n, const int64_t *toff, const int64_t *zoff,
                            const int64_t *ldz, const int32_t *ncols, double *z, const int32_t *partner,
                            const double *cs, int32_t forward) {
    const PairMeta m{n, toff, nullptr};
    k_pair_rows<<<(unsigned)count, 256, 0, s>>>(m, zoff, ldz, ncols, z, partner, cs, forward);
    return hipGetLastError();
}

}  // namespace ipt
