// Batched full-spectrum IPT: many independent dense problems M_b = D_b + Delta_b of
// uneven size n_b, all advanced by the same few launches per sweep.
//
// Every matrix is cut into T x T tiles (T = 64 or 128, chosen per size bucket); the
// work list holds one item (b, row tile, column tile) per tile, largest matrices
// first.  The sweep GEMM is persistent: a fixed grid of workgroups takes items from
// an atomic ticket until the list is drained, and skips column tiles with no active
// column.  Each column tile carries its own precision for the sweep (a stamped
// word: sweep << 2 | precision), chosen by the finalize kernel from the columns'
// steps: FP32 split-form sweeps (only Z - E in FP32, Delta E exact in FP64) until a
// column's step reaches tau_32 or stalls, then FP64 sweeps, which alone may certify.
//
// Layouts (all row-major, leading dimension n_b): Delta_b in the caller's pool, the
// two iterate buffers in a packed pool, columns of all problems concatenated.
#include <math.h>

#include <type_traits>

#include "ipt_internal.h"

namespace ipt {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ inline uint64_t dbits(double x) {
    if (!(x >= 0.0)) x = INFINITY;
    return (uint64_t)__double_as_longlong(x);
}
__device__ inline double bitsd(uint64_t b) { return __longlong_as_double((long long)b); }

typedef BatchLaunch BArgs;

__device__ inline uint32_t flag_word(uint32_t *tflag, int64_t total, int32_t parity, int64_t tile) {
    return tflag[(int64_t)parity * total + tile];
}

// ----------------------------------------------------------------- setup
// Column init, theta checks (finite, distinct within each problem; brute force in
// LDS, n_b <= 4096) and the initial tile flags.  One block per problem.
__global__ __launch_bounds__(256) void k_binit(Ctrl *ctrl, BArgs a, int32_t start_prec) {
    const int b = blockIdx.x;
    const BatchMeta m = a.meta[b];
    __shared__ double th[4096];
    const double *tb = a.theta + m.offt;
    bool bad_nan = false, degen = false;
    for (int j = threadIdx.x; j < m.n; j += blockDim.x) {
        th[j] = tb[j];
        bad_nan |= !isfinite(tb[j]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m.n; i += blockDim.x) {
        const double ti = th[i];
        for (int j = 0; j < m.n; ++j) degen |= (j != i) && (th[j] == ti);
        const int64_t c = m.offc + i;
        a.col.prob[c] = b;
        a.col.state[c] = COL_ACTIVE;
        a.col.sweeps[c] = 0;
        a.col.grow[c] = 0;
        a.col.par[c] = PAR_BUF0;
        a.col.prev[c] = INFINITY;
        a.col.step[c] = INFINITY;
        a.col.lam[c] = 0.0;
        a.col.resid[c] = 0.0;
    }
    if (bad_nan) atomicMax(&ctrl->error, (int32_t)IPT_EINVAL);
    if (degen) atomicMax(&ctrl->error, (int32_t)IPT_EDEGENERATE);
    const int ntn = (m.n + m.T - 1) / m.T;
    for (int q = threadIdx.x; q < ntn; q += blockDim.x) {
        a.tflag[m.offf + q] = (0u << 2) | (uint32_t)start_prec;                   // sweep 1 (stamp 0)
        a.tflag[a.total_tiles + m.offf + q] = (0u << 2) | (uint32_t)start_prec;
    }
    if (threadIdx.x == 0) a.col.norm_bits[b] = 0;
}

// |M_b|_1 per problem (max column sum of |D_b + Delta_b|), block per problem.
__global__ __launch_bounds__(256) void k_bnorm(const Ctrl *ctrl, BArgs a) {
    if (ctrl->error) return;
    const int b = blockIdx.x;
    const BatchMeta m = a.meta[b];
    const double *db = a.delta + m.offd;
    const double *tb = a.theta + m.offt;
    double best = 0.0;
    for (int c = threadIdx.x; c < m.n; c += blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < m.n; ++j) {
            const double v = db[(int64_t)j * m.n + c] + (j == c ? tb[c] : 0.0);
            s += fabs(v);
        }
        best = fmax(best, s);
    }
    atomicMax((unsigned long long *)&a.col.norm_bits[b], (unsigned long long)dbits(best));
}

// Product-free first sweep of a cold start: W = I - G o Delta (eq. dyn at Z = I),
// d_c = Delta_cc.  Item = (problem, row tile, 64 columns); same partial layout as the
// GEMM epilogue.
__global__ __launch_bounds__(256) void k_bsweep1(const Ctrl *ctrl, BArgs a, const int4 *items, int64_t nitems) {
    if (ctrl->error || ctrl->done) return;
    __shared__ double sh[4][NPART][64];
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int4 w = items[it];
        const BatchMeta m = a.meta[w.x];
        const int tm = w.y, cb = w.z;
        const int cx = threadIdx.x & 63, ry = threadIdx.x >> 6;
        const int c = cb * 64 + cx;
        const bool colok = c < m.n;
        const double *db = a.delta + m.offd;
        const double *tb = a.theta + m.offt;
        double *zout = a.z1 + m.offz;
        double v[NPART] = {0.0, 0.0, 0.0, 0.0};
        const double ti = colok ? tb[c] : 0.0;
        for (int r = ry; r < m.T; r += 4) {
            const int j = tm * m.T + r;
            if (!colok || j >= m.n) continue;
            double wv;
            if (j == c) {
                wv = 1.0;
                v[1] += 1.0;
            } else {
                const double gap = tb[j] - ti;
                wv = -db[(int64_t)j * m.n + c] / gap;
                v[0] += wv * wv;
                v[2] += (gap * wv) * (gap * wv);
                v[3] += wv * wv;
            }
            zout[(int64_t)j * m.n + c] = wv;
        }
        if (colok && tm == c / m.T && ry == 0) a.col.d[m.offc + c] = db[(int64_t)c * m.n + c];
#pragma unroll
        for (int q = 0; q < NPART; ++q) sh[ry][q][cx] = v[q];
        __syncthreads();
        if (ry == 0 && colok) {
#pragma unroll
            for (int q = 0; q < NPART; ++q)
                a.part[m.offp + ((int64_t)tm * m.n + c) * NPART + q] =
                    ((sh[0][q][cx] + sh[1][q][cx]) + sh[2][q][cx]) + sh[3][q][cx];
        }
        __syncthreads();
    }
}

// d_c = sum_l Delta_cl Z_lc (FP64) for the active columns.  Item = (problem, 64
// columns); 4 lane groups split l and are added in order.
__global__ __launch_bounds__(256) void k_bdiag(const Ctrl *ctrl, BArgs a, const int4 *items, int64_t nitems,
                                               int32_t in_buf) {
    if (ctrl->error || ctrl->done) return;
    __shared__ double red[4][64];
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int4 w = items[it];
        const BatchMeta m = a.meta[w.x];
        const int cx = threadIdx.x & 63, g = threadIdx.x >> 6;
        const int c = w.z * 64 + cx;
        const bool act = c < m.n && a.col.state[m.offc + c] == COL_ACTIVE;
        const double *db = a.delta + m.offd + (int64_t)(act ? c : 0) * m.n;
        const double *zb = (in_buf ? a.z1 : a.z0) + m.offz;
        const int span = (m.n + 3) / 4;
        double acc = 0.0;
        if (act) {
            const int l1 = min(m.n, (g + 1) * span);
            for (int l = g * span; l < l1; ++l) acc += db[l] * zb[(int64_t)l * m.n + c];
        }
        red[g][cx] = acc;
        __syncthreads();
        if (g == 0 && act) a.col.d[m.offc + c] = ((red[0][cx] + red[1][cx]) + red[2][cx]) + red[3][cx];
        __syncthreads();
    }
}

// ------------------------------------------------------------------ GEMM
// One T x T tile of W = F(Z) for problem b: Y = Delta_b Z_b on the matrix cores
// (FP64, or FP32 on the split iterate), bounds-checked loads (n_b need not be a
// multiple of T), fused IPT epilogue and per-column partial sums.
template <int T>
struct BCfg {
    static constexpr int MI = T / 32;  // 16x16 MFMA blocks per wave and dimension (waves are 2 x 2)
    static constexpr int BK = 16;
    static constexpr int PA = T * BK / 256;  // A elements staged per thread per K slice
};

template <int T, bool F64>
__device__ __forceinline__ void btile(char *smem, double (*red)[T][NPART], const BArgs &a, const BatchMeta &m, int tm,
                                      int tn, int32_t in_buf) {
    using C = BCfg<T>;
    constexpr int MI = C::MI, BK = C::BK, PA = C::PA;
    typedef typename std::conditional<F64, double, float>::type E;
    typedef E ATile[T][BK + 1];
    typedef E BTile[BK][T];
    ATile *As = (ATile *)smem;
    BTile *Bs = (BTile *)(smem + 2 * sizeof(ATile));
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, wm = wv >> 1, wn = wv & 1;
    const int n = m.n;
    const double *Ab = a.delta + m.offd;
    const double *zin = (in_buf ? a.z1 : a.z0) + m.offz;
    double *zout = (in_buf ? a.z0 : a.z1) + m.offz;
    const int r0 = tm * T, c0 = tn * T;
    // loader mapping: A slice T x BK, thread t loads rows (t / BK) + (256 / BK) q, column t % BK;
    //                 B slice BK x T, thread t loads row t / T + (256 / T) q, column t % T
    const int a_r = t / BK, a_k = t % BK;
    const int b_r = t / T, b_c = t % T;
    constexpr int AR = 256 / BK, BR = 256 / T;
    E ra[PA], rb[PA];
#define IPT_BLOAD(K0)                                                                          \
    do {                                                                                       \
        _Pragma("unroll") for (int q = 0; q < PA; ++q) {                                       \
            const int row = r0 + a_r + AR * q, kk = (K0) + a_k;                                \
            ra[q] = (E)((row < n && kk < n) ? Ab[(int64_t)row * n + kk] : 0.0);                \
        }                                                                                      \
        _Pragma("unroll") for (int q = 0; q < PA; ++q) {                                       \
            const int kk = (K0) + b_r + BR * q, cc = c0 + b_c;                                 \
            double v = (kk < n && cc < n) ? zin[(int64_t)kk * n + cc] : 0.0;                   \
            if (!F64 && kk == cc && kk < n) v -= 1.0; /* split iterate Z - E */                \
            rb[q] = (E)v;                                                                      \
        }                                                                                      \
    } while (0)
#define IPT_BSTORE(S)                                                                          \
    do {                                                                                       \
        _Pragma("unroll") for (int q = 0; q < PA; ++q) As[S][a_r + AR * q][a_k] = ra[q];       \
        _Pragma("unroll") for (int q = 0; q < PA; ++q) Bs[S][b_r + BR * q][b_c] = rb[q];       \
    } while (0)
    typedef typename std::conditional<F64, d4_t, f4_t>::type ACC;
    ACC acc[MI][MI];
#pragma unroll
    for (int x = 0; x < MI; ++x)
#pragma unroll
        for (int y = 0; y < MI; ++y) acc[x][y] = ACC{0, 0, 0, 0};
    const int nk = (n + BK - 1) / BK;
    IPT_BLOAD(0);
    IPT_BSTORE(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        IPT_BLOAD((kt + 1 < nk ? kt + 1 : kt) * BK);
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            E fa[MI], fb[MI];
#pragma unroll
            for (int x = 0; x < MI; ++x) fa[x] = As[cur][wm * (T / 2) + 16 * x + (lane & 15)][4 * kk + (lane >> 4)];
#pragma unroll
            for (int y = 0; y < MI; ++y) fb[y] = Bs[cur][4 * kk + (lane >> 4)][wn * (T / 2) + 16 * y + (lane & 15)];
#pragma unroll
            for (int x = 0; x < MI; ++x)
#pragma unroll
                for (int y = 0; y < MI; ++y) {
                    if constexpr (F64)
                        acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[x], fb[y], acc[x][y], 0, 0, 0);
                    else
                        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[x], fb[y], acc[x][y], 0, 0, 0);
                }
        }
        IPT_BSTORE(cur ^ 1);
        __syncthreads();
    }
#undef IPT_BLOAD
#undef IPT_BSTORE
    // epilogue (idx = identity: column c continues e_c)
    const double *tb = a.theta + m.offt;
    int cols[MI];
    bool act[MI];
    double ti[MI], dd[MI];
#pragma unroll
    for (int y = 0; y < MI; ++y) {
        const int c = c0 + wn * (T / 2) + 16 * y + (lane & 15);
        cols[y] = c;
        act[y] = c < n && a.col.state[m.offc + c] == COL_ACTIVE;
        ti[y] = c < n ? tb[c] : 0.0;
        dd[y] = c < n ? a.col.d[m.offc + c] : 0.0;
    }
    double sums[MI][NPART];
#pragma unroll
    for (int y = 0; y < MI; ++y)
#pragma unroll
        for (int q = 0; q < NPART; ++q) sums[y][q] = 0.0;
#pragma unroll
    for (int x = 0; x < MI; ++x)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            // f64 MFMA: row 4r + l/16; f32 MFMA: row 4(l/16) + r
            const int lr = F64 ? (16 * x + 4 * r + (lane >> 4)) : (16 * x + 4 * (lane >> 4) + r);
            const int j = r0 + wm * (T / 2) + lr;
            if (j >= n) continue;
            const double tj = tb[j];
#pragma unroll
            for (int y = 0; y < MI; ++y) {
                if (!act[y]) continue;
                const int c = cols[y];
                const double z = zin[(int64_t)j * n + c];
                double wv, st, gs, de;
                if (j == c) {
                    wv = 1.0;
                    st = wv - z;
                    gs = 0.0;
                    de = 0.0;
                } else {
                    const double yv = F64 ? (double)acc[x][y][r] : Ab[(int64_t)j * n + c] + (double)acc[x][y][r];
                    const double gap = tj - ti[y];
                    wv = (z * dd[y] - yv) / gap;
                    st = wv - z;
                    gs = gap * st;
                    de = wv;
                }
                zout[(int64_t)j * n + c] = wv;
                sums[y][0] += st * st;
                sums[y][1] += z * z;
                sums[y][2] += gs * gs;
                sums[y][3] += de * de;
            }
        }
#pragma unroll
    for (int y = 0; y < MI; ++y)
#pragma unroll
        for (int q = 0; q < NPART; ++q) {
            double v = sums[y][q];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            sums[y][q] = v;
        }
    if (lane < 16) {
#pragma unroll
        for (int y = 0; y < MI; ++y)
#pragma unroll
            for (int q = 0; q < NPART; ++q) red[wm][wn * (T / 2) + 16 * y + lane][q] = sums[y][q];
    }
    __syncthreads();
    if (t < T) {
        const int c = c0 + t;
        if (c < n) {
#pragma unroll
            for (int q = 0; q < NPART; ++q)
                a.part[m.offp + ((int64_t)tm * n + c) * NPART + q] = red[0][t][q] + red[1][t][q];
        }
    }
    __syncthreads();
}

template <int T>
__global__ __launch_bounds__(256, (T == 64 ? 3 : 2)) void k_bgemm(const Ctrl *ctrl, BArgs a, const int4 *items, int64_t nitems,
                                               int32_t sweep, int32_t in_buf, int32_t *ticket) {
    if (ctrl->error || ctrl->done) return;
    constexpr int SM = 2 * T * (16 + 1) * 8 + 2 * 16 * T * 8;
    __shared__ __attribute__((aligned(16))) char smem[SM];
    __shared__ double red[2][T][NPART];
    __shared__ int64_t cur_item;
    const int32_t par = (sweep - 1) & 1;  // tile flags of this sweep were written by the previous finalize
    for (;;) {
        if (threadIdx.x == 0) cur_item = atomicAdd(ticket, 1);
        __syncthreads();
        const int64_t it = cur_item;
        __syncthreads();
        if (it >= nitems) break;
        const int4 w = items[it];
        const BatchMeta m = a.meta[w.x];
        const uint32_t f = flag_word(a.tflag, a.total_tiles, par, m.offf + w.z);
        if ((int32_t)(f >> 2) != sweep - 1) continue;  // no active column in this column tile
        if ((f & 3u) == (uint32_t)PREC_F64) btile<T, true>(smem, red, a, m, w.y, w.z, in_buf);
        else btile<T, false>(smem, red, a, m, w.y, w.z, in_buf);
    }
}

// --------------------------------------------------------------- finalize
// Per column of every problem: reduce the partials of its problem's row tiles in
// order, form s_c, decide (only an FP64 or product-free sweep certifies), and stamp
// the column tile's flag for the next sweep with the precision it needs.
__global__ __launch_bounds__(256) void k_bfinalize(Ctrl *ctrl, DevOpts o, BArgs a, int64_t total_cols,
                                                   int32_t sweep, int32_t in_par, int32_t out_par) {
    if (ctrl->error || ctrl->done) return;
    const int64_t gc = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int32_t decided = -1;
    double s = 0.0;
    bool act = false, still = false;
    uint64_t res_bits = 0;
    double dist = 0.0;
    if (gc < total_cols && a.col.state[gc] == COL_ACTIVE) {
        act = true;
        const int b = a.col.prob[gc];
        const BatchMeta m = a.meta[b];
        const int c = (int)(gc - m.offc);
        const int nrt = (m.n + m.T - 1) / m.T;
        double p[NPART] = {0.0, 0.0, 0.0, 0.0};
        for (int rt = 0; rt < nrt; ++rt) {
            const double4 v = *(const double4 *)&a.part[m.offp + ((int64_t)rt * m.n + c) * NPART];
            p[0] += v.x;
            p[1] += v.y;
            p[2] += v.z;
            p[3] += v.w;
        }
        s = sqrt(p[0]) / sqrt(p[1]);
        dist = sqrt(p[3]);
        const uint32_t f = flag_word(a.tflag, a.total_tiles, (sweep - 1) & 1, m.offf + c / m.T);
        const int32_t prec = (sweep == 1 && in_par == PAR_UNIT) ? PREC_EXACT_FIRST : (int32_t)(f & 3u);
        const bool exact = prec == PREC_F64 || prec == PREC_EXACT_FIRST;
        const double resid = sqrt(p[2]) / sqrt(p[1]);  // normalised by |M_b|_1 at copy-out
        if (exact && s <= o.tol) {
            decided = COL_CONVERGED;
            a.col.par[gc] = in_par;
            res_bits = 1;
        } else {
            const bool bad = !isfinite(s) || !(dist <= o.div_norm);
            int32_t grow = a.col.grow[gc];
            if (exact) {
                grow = (s > a.col.prev[gc]) ? grow + 1 : 0;
                a.col.grow[gc] = grow;
            }
            if (bad || grow >= o.div_growth) {
                decided = COL_DIVERGED;
                a.col.par[gc] = out_par;
            } else if (sweep >= o.max_iter) {
                decided = COL_NOT_CONVERGED;
                a.col.par[gc] = out_par;
            }
        }
        const double prev = a.col.prev[gc];
        a.col.prev[gc] = s;
        if (decided >= 0) {
            a.col.state[gc] = decided;
            a.col.sweeps[gc] = sweep;
            a.col.step[gc] = s;
            a.col.lam[gc] = a.theta[m.offt + c] + a.col.d[gc];
            a.col.resid[gc] = resid;
        } else {
            still = true;
            // precision this column asks of its tile next sweep
            int32_t want = PREC_F64;
            if (o.ladder && prec != PREC_F64) want = (s <= o.tau_32 || !(s < prev)) ? PREC_F64 : PREC_F32;
            atomicMax(&a.tflag[(int64_t)(sweep & 1) * a.total_tiles + m.offf + c / m.T],
                      ((uint32_t)sweep << 2) | (uint32_t)want);
        }
    }
    // wave-aggregated bookkeeping
    uint64_t v = act ? dbits(s) : 0;
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t q = (uint64_t)__shfl_xor((unsigned long long)v, off);
        v = q > v ? q : v;
    }
    uint64_t dv = decided >= 0 ? dbits(s) : 0;
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t q = (uint64_t)__shfl_xor((unsigned long long)dv, off);
        dv = q > dv ? q : dv;
    }
    const uint64_t m_still = __ballot(still), m_conv = __ballot(decided == COL_CONVERGED),
                   m_div = __ballot(decided == COL_DIVERGED), m_nc = __ballot(decided == COL_NOT_CONVERGED);
    (void)res_bits;
    (void)dist;
    if ((threadIdx.x & 63) == 0) {
        if (v) atomicMax((unsigned long long *)&ctrl->acc_maxstep, (unsigned long long)v);
        if (dv) atomicMax((unsigned long long *)&ctrl->dec_maxstep, (unsigned long long)dv);
        if (m_still) atomicAdd(&ctrl->acc_active, (int32_t)__popcll(m_still));
        if (m_conv) atomicAdd(&ctrl->n_conv, (int32_t)__popcll(m_conv));
        if (m_div) atomicAdd(&ctrl->n_div, (int32_t)__popcll(m_div));
        if (m_nc) atomicAdd(&ctrl->n_notconv, (int32_t)__popcll(m_nc));
    }
}

// Sweep bookkeeping of the batch (history, done flag) and ticket reset.
__global__ void k_bcontrol(Ctrl *ctrl, DevOpts o, int32_t sweep, int32_t *tickets) {
    if (ctrl->error || ctrl->done) return;
    const double ms = bitsd(ctrl->acc_maxstep);
    if (sweep - 1 < IPT_HIST) {
        ctrl->hist_prec[sweep - 1] = ctrl->prec;
        ctrl->hist_active[sweep - 1] = ctrl->active;
        ctrl->hist_step[sweep - 1] = ms;
    }
    ctrl->matvecs += (sweep == 1 && ctrl->prec == PREC_EXACT_FIRST) ? 0 : ctrl->active;
    ctrl->active = ctrl->acc_active;
    ctrl->acc_active = 0;
    ctrl->acc_maxstep = 0;
    ctrl->sweeps = sweep;
    if (ctrl->active == 0 || sweep >= o.max_iter) ctrl->done = 1;
    // the batch records FP64 once any tile runs in FP64, else FP32 (tile precisions vary)
    ctrl->prec = o.ladder ? PREC_F32 : PREC_F64;
    tickets[0] = 0;
    tickets[1] = 0;
}

// Outputs: z_pool[b] <- final iterate of each column, lambda, status; the
// eigen-residual is normalised by |M_b|_1 here.
__global__ void k_bcopyout(const Ctrl *ctrl, BArgs a, const int64_t *z_off, double *z_pool, double *lambda_pool,
                           int32_t *status_pool, int64_t total_cols, double *max_resid_out) {
    if (ctrl->error) return;
    const int64_t gc = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gc >= total_cols) return;
    const int b = a.col.prob[gc];
    const BatchMeta m = a.meta[b];
    const int c = (int)(gc - m.offc);
    const int32_t par = a.col.par[gc];
    const double *src = (par == PAR_BUF1 ? a.z1 : a.z0) + m.offz;
    double *dst = z_pool + z_off[b];
    for (int j = 0; j < m.n; ++j) dst[(int64_t)j * m.n + c] = (par == PAR_UNIT) ? (j == c ? 1.0 : 0.0) : src[(int64_t)j * m.n + c];
    lambda_pool[m.offt + c] = a.col.lam[gc];
    const int32_t st = a.col.state[gc];
    status_pool[m.offt + c] = st == COL_ACTIVE ? IPT_NOT_CONVERGED : st;
    const double nrm = bitsd(a.col.norm_bits[b]);
    const double r = a.col.resid[gc] / (nrm > 0.0 ? nrm : 1.0);
    a.col.resid[gc] = r;
    if (st == COL_CONVERGED)
        atomicMax((unsigned long long *)max_resid_out, (unsigned long long)dbits(r));
}

}  // namespace

// ------------------------------------------------------------- launchers
BatchLaunch make_batch_launch(const BatchMeta *meta, const double *theta, const double *delta, double *z0, double *z1,
                              BatchCols col, double *part, uint32_t *tflag, int64_t total_tiles) {
    BatchLaunch L;
    L.meta = meta;
    L.theta = theta;
    L.delta = delta;
    L.z0 = z0;
    L.z1 = z1;
    L.col = col;
    L.part = part;
    L.tflag = tflag;
    L.total_tiles = total_tiles;
    return L;
}

static const BArgs &to_args(const BatchLaunch &L) { return L; }

int bgemm_grid(int tile) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 512;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    hipError_t e = tile == 64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_bgemm<64>, 256, 0)
                              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_bgemm<128>, 256, 0);
    if (e != hipSuccess || per <= 0) per = 1;
    return cus * per;
}

hipError_t launch_binit(hipStream_t s, Ctrl *ctrl, const BatchLaunch &L, int32_t count, int32_t start_prec) {
    k_binit<<<count, 256, 0, s>>>(ctrl, to_args(L), start_prec);
    return hipGetLastError();
}

hipError_t launch_bnorm(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, int32_t count) {
    k_bnorm<<<count, 256, 0, s>>>(ctrl, to_args(L));
    return hipGetLastError();
}

hipError_t launch_bsweep1(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, const int4 *items, int64_t nitems) {
    const int g = nitems < 8192 ? (int)nitems : 8192;
    k_bsweep1<<<g > 0 ? g : 1, 256, 0, s>>>(ctrl, to_args(L), items, nitems);
    return hipGetLastError();
}

hipError_t launch_bdiag(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, const int4 *items, int64_t nitems,
                        int32_t in_buf) {
    const int g = nitems < 8192 ? (int)nitems : 8192;
    k_bdiag<<<g > 0 ? g : 1, 256, 0, s>>>(ctrl, to_args(L), items, nitems, in_buf);
    return hipGetLastError();
}

hipError_t launch_bgemm(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, int tile, const int4 *items,
                        int64_t nitems, int32_t sweep, int32_t in_buf, int32_t *ticket, int grid) {
    if (nitems == 0) return hipSuccess;
    if (tile == 64) k_bgemm<64><<<grid, 256, 0, s>>>(ctrl, to_args(L), items, nitems, sweep, in_buf, ticket);
    else k_bgemm<128><<<grid, 256, 0, s>>>(ctrl, to_args(L), items, nitems, sweep, in_buf, ticket);
    return hipGetLastError();
}

hipError_t launch_bfinalize(hipStream_t s, Ctrl *ctrl, const DevOpts &o, const BatchLaunch &L, int64_t total_cols,
                            int32_t sweep, int32_t in_par, int32_t out_par) {
    k_bfinalize<<<(unsigned)((total_cols + 255) / 256), 256, 0, s>>>(ctrl, o, to_args(L), total_cols, sweep, in_par,
                                                                      out_par);
    return hipGetLastError();
}

hipError_t launch_bcontrol(hipStream_t s, Ctrl *ctrl, const DevOpts &o, int32_t sweep, int32_t *tickets) {
    k_bcontrol<<<1, 1, 0, s>>>(ctrl, o, sweep, tickets);
    return hipGetLastError();
}

hipError_t launch_bcopyout(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, const int64_t *z_off,
                           double *z_pool, double *lambda_pool, int32_t *status_pool, int64_t total_cols,
                           double *max_resid_out) {
    k_bcopyout<<<(unsigned)((total_cols + 255) / 256), 256, 0, s>>>(ctrl, to_args(L), z_off, z_pool, lambda_pool,
                                                                     status_pool, total_cols, max_resid_out);
    return hipGetLastError();
}

}  // namespace ipt
