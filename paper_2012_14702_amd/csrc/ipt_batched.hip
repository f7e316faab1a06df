// Batched full-spectrum IPT: many independent dense problems M_b = D_b + Delta_b of
// uneven size n_b, all advanced by the same few launches per sweep.
//
// Every problem is cut into T x T tiles, T in {32, 64, 128} chosen per size bucket
// (by the autotuner in ipt_api.hip), and padded to np_b = round_up(n_b, T) so that
// the Delta operand is read in aligned 16-byte chunks with no bounds checks.  The
// active columns of each problem are packed: after every sweep a plan kernel lists
// them in ascending order, and the GEMM tiles run over packed column positions,
// gathering their iterate columns, so frozen columns cost nothing (the iterates
// keep their natural layout).  A sweep is one persistent GEMM launch per tile size
// over the work list of (problem, row tile, packed column tile) items, a finalize
// over all columns, the plan kernel (one block per problem: packed columns, tile
// precisions, work items of the next sweep) and a control kernel.  The sweep number
// lives in the device control block, so every sweep's launches are the same and a
// chunk of sweeps is captured once in a hipGraph and replayed.
//
// Each packed column tile carries its own precision, the highest its columns ask
// for (from their steps, in the finalize): FP32 split-form sweeps (Delta_32 (Z - E)_32 on the matrix cores, Delta E added
// exactly in FP64) until a column's step reaches tau_32 or stalls, then FP64 sweeps,
// which alone may certify.  FP32 tiles also write the FP32 shadow of W - E that the
// next FP32 sweep multiplies.
//
// d_c = (Delta Z)_{cc} of sweep t + 1 is summed by the epilogues of sweep t from the W
// they produce (per row tile, the sum over its rows l of Delta_cl W_lc) and reduced
// in row-tile order by the finalize, so no separate pass over Delta and Z is needed.
//
// Workspace layouts (row-major, leading dimension np_b, problems packed largest
// first): padded Delta (FP64, and its FP32 shadow for the ladder), two FP64 iterate
// buffers and their two FP32 (Z - E) shadows.  The caller's Delta is read only by
// the first sweep, which also builds the padded copies.
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

__device__ inline int32_t cur_sweep(const Ctrl *ctrl) { return ctrl->sweeps + 1; }

template <int T>
constexpr int tile_class() {
    return T == 32 ? 0 : (T == 64 ? 1 : 2);
}
__device__ inline int tile_class_of(int T) { return T == 32 ? 0 : (T == 64 ? 1 : 2); }

// Segmented inclusive max over a wave.  Lanes with equal keys must be contiguous;
// the segment maximum ends up in the segment's last lane, which gets leader = true.
__device__ inline uint64_t seg_max(int64_t key, uint64_t v, bool &leader) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t ov = (uint64_t)__shfl_up((unsigned long long)v, off);
        const int64_t ok = (int64_t)__shfl_up((long long)key, off);
        if (lane >= off && ok == key) v = ov > v ? ov : v;
    }
    const int64_t nk = (int64_t)__shfl_down((long long)key, 1);
    leader = (lane == 63) || (nk != key);
    return v;
}

__device__ inline int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(v, off);
        if (lane >= off) v += o;
    }
    return v;
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
        a.col.d[c] = 0.0;
    }
    if (bad_nan) atomicMax(&ctrl->error, (int32_t)IPT_EINVAL);
    if (degen) atomicMax(&ctrl->error, (int32_t)IPT_EDEGENERATE);
    (void)start_prec;
    if (threadIdx.x == 0) {
        a.col.norm_bits[b] = 0;
        a.col.kact[b] = 0;
        a.col.asym[b] = 0;
    }
}

// Product-free first sweep of a cold start, W = I - G o Delta (eq. 2 at Z = I), with
// d_c = Delta_cc for this sweep.  It also writes the padded copies of Delta (FP64 and,
// for the ladder, FP32), zeroes the padding of both iterate buffers and shadows, and
// stores the row-tile partials of the next sweep's d (sum_l Delta_cl W_lc, the
// transposed Delta block staged through LDS) and of the column sums of |M_b| (for
// |M_b|_1).  Item = (problem, row tile, 64 columns of the padded width).
__global__ __launch_bounds__(256) void k_bsweep1(const Ctrl *ctrl, BArgs a, const int4 *items, int64_t nitems,
                                                 int32_t ladder, int32_t acx) {
    if (ctrl->error || ctrl->done) return;
    __shared__ double tt[32][64 + 1];            // Delta[c0 + ci][j0 + jj] at tt[jj][ci]
    __shared__ double sh[4][NPART + 2][64];
    const int cx = threadIdx.x & 63, ry = threadIdx.x >> 6;
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int4 w = items[it];
        const BatchMeta m = a.meta[w.x];
        const int n = m.n, np = m.np, tm = w.y;
        const int c0 = w.z * 64, c = c0 + cx;
        const bool colok = c < n;
        const double *db = a.delta + m.offd;
        const double *tb = a.theta + m.offt;
        const double ti = colok ? tb[c] : 0.0;
        // partials: step^2, |z|^2, gap^2 step^2, |w - e|^2 (as the GEMM epilogue), next d,
        // |M| column sum
        double v[NPART + 2] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int j0 = tm * m.T; j0 < tm * m.T + m.T; j0 += 32) {
            {   // transposed block: thread loads 8 consecutive j of row c0 + t / 4
                const int ci = threadIdx.x >> 2, jb = (threadIdx.x & 3) * 8;
                const int cc = c0 + ci;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int jj = j0 + jb + e;
                    tt[jb + e][ci] = (cc < n && jj < n) ? db[(int64_t)cc * n + jj] : 0.0;
                }
            }
            __syncthreads();
            // the eight rows' loads go out together (clamped to valid addresses), then the
            // writes of each row
            double dv[8], tv[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int j = j0 + ry + 4 * i;
                const int jc = j < n ? j : n - 1, cc = colok ? c : 0;
                dv[i] = db[(int64_t)jc * n + cc];
                tv[i] = tb[jc];
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int jj = ry + 4 * i, j = j0 + jj;
                if (c >= np) continue;
                const bool in = colok && j < n;
                const double djc = in ? dv[i] : 0.0;
                const int64_t e = m.offz + (int64_t)j * np + c;
                a.dpad[e] = djc;
                double wv = 0.0;
                if (in) {
                    if (j == c) {
                        wv = 1.0;
                        v[1] += 1.0;
                        v[5] += fabs(djc + ti);
                    } else {
                        const double gap = tv[i] - ti;
                        wv = -djc / gap;
                        v[0] += wv * wv;
                        v[2] += (gap * wv) * (gap * wv);
                        v[3] += wv * wv;
                        v[5] += fabs(djc);
                    }
                    v[4] += tt[jj][cx] * wv;
                }
                if (in && djc != tt[jj][cx]) a.col.asym[w.x] = 1;  // Delta_jc vs Delta_cj
                a.zs[1][e] = wv;
                // slot 0: padding zeroed; with ACX it holds E, the base iterate of the first cycle
                if (acx) a.zs[0][e] = (in && j == c) ? 1.0 : 0.0;
                else if (!in) a.zs[0][e] = 0.0;
                if (acx && !in) {
                    a.zs[2][e] = 0.0;
                    a.zs[3][e] = 0.0;
                }
                if (ladder) {
                    a.d32[e] = (float)djc;
                    a.zlo1[e] = (float)(wv - (in && j == c ? 1.0 : 0.0));
                    if (!in) a.zlo0[e] = 0.f;
                }
            }
            __syncthreads();
        }
        if (colok && tm == c / m.T && ry == 0) a.col.d[m.offc + c] = db[(int64_t)c * n + c];
#pragma unroll
        for (int q = 0; q < NPART + 2; ++q) sh[ry][q][cx] = v[q];
        __syncthreads();
        if (ry == 0 && colok) {
            double r6[NPART + 2];
#pragma unroll
            for (int q = 0; q < NPART + 2; ++q) r6[q] = ((sh[0][q][cx] + sh[1][q][cx]) + sh[2][q][cx]) + sh[3][q][cx];
#pragma unroll
            for (int q = 0; q < NPART; ++q) a.part[m.offp + ((int64_t)tm * n + c) * NPART + q] = r6[q];
            a.dpart[m.offq + (int64_t)tm * n + c] = r6[4];
            a.normpart[m.offq + (int64_t)tm * n + c] = r6[5];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ GEMM
// One T x T tile of W = F(Z) for problem b: Y = Delta_b Z_b on the matrix cores
// (FP64, or FP32 on the shadows), fused IPT epilogue, per-column partial sums and
// the partial of the next sweep's d.  All operands are padded and 16-byte aligned.
template <int T, bool F64>
struct BT {
    typedef typename std::conditional<F64, double, float>::type E;
    static constexpr int BK = F64 ? 16 : 32;
    static constexpr int VE = 16 / (int)sizeof(E);  // elements per 16-byte chunk
    static constexpr int CPA = BK / VE;              // chunks per A row (8)
    static constexpr int RPA = 256 / CPA;            // A rows per pass (32)
    static constexpr int PA = T / RPA;               // A passes per thread
    static constexpr int TPB = 256 / BK;             // threads per B row
    static constexpr int PB = (T / VE) / TPB;        // B chunks per thread
    // LDS pitches (elements) chosen so that the MFMA operand reads -- 16 rows x 4 k of A,
    // 4 k rows x 16 columns of B per wave -- fall on distinct banks
    static constexpr int LDA = F64 ? BK + 2 : BK + 4;
    static constexpr int LDB = T + 16;
    static constexpr int SMEM = 2 * T * LDA * (int)sizeof(E) + 2 * BK * LDB * (int)sizeof(E);
    static_assert(PA >= 1 && PB >= 1, "tile too small for the loader");
};

template <int T>
constexpr int bsmem() {
    return BT<T, true>::SMEM > BT<T, false>::SMEM ? BT<T, true>::SMEM : BT<T, false>::SMEM;
}

template <int T, bool F64>
__device__ __forceinline__ void btile(char *smem, int32_t *scol, const BArgs &a, const BatchMeta &m, int b, int tm,
                                      int tn, int32_t t, int32_t acx) {
    typedef BT<T, F64> C;
    typedef typename C::E E;
    constexpr int BK = C::BK, VE = C::VE, CPA = C::CPA, RPA = C::RPA, PA = C::PA, LDA = C::LDA, LDB = C::LDB;
    constexpr int MI = T / 32;  // 16 x 16 MFMA blocks per wave and dimension (waves are 2 x 2)
    typedef E ATile[T][LDA];
    typedef E BTile[BK][LDB];
    ATile *As = (ATile *)smem;
    BTile *Bs = (BTile *)(smem + 2 * sizeof(ATile));
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv >> 1, wn = wv & 1;
    const int n = m.n, np = m.np;
    int32_t q, pc;
    acx_phase(acx, t, q, pc);
    const int32_t in_buf = acx ? q : (t - 1) & 1, out_buf = acx ? q + 1 : in_buf ^ 1;
    const double *Ad = a.dpad + m.offz;
    const double *zin = a.zs[in_buf] + m.offz;
    double *zout = a.zs[out_buf] + m.offz;
    const E *Ag, *Bg;
    if constexpr (F64) {
        Ag = Ad;
        Bg = zin;
    } else {
        Ag = a.d32 + m.offz;
        Bg = (in_buf ? a.zlo1 : a.zlo0) + m.offz;
    }
    // packed column positions p0 .. p0 + T - 1 of the problem's active list
    const int r0 = tm * T, p0 = tn * T;
    const int32_t *al = a.col.alist + m.offc;
    const int kact = a.col.kact[b];
    const E *Ab = Ag + (int64_t)r0 * np;
    const int a_r = tid / CPA, a_c = (tid % CPA) * VE;
    // The tile's gathered iterate columns (-1 past the active list).  B loader: each
    // thread owns one column (lanes run over consecutive packed columns) and RB-strided
    // rows of the K slice.
    for (int i = tid; i < T; i += 256) scol[i] = p0 + i < kact ? al[p0 + i] : -1;
    __syncthreads();
    constexpr int RB = 256 / T, NB = BK / RB;  // row stride and rows per thread of the B slice
    const int b_c = tid % T, b_r = tid / T;
    const int cg = scol[b_c];
    uint4 ra[PA];
    E rb[NB];
    union Chunk {
        uint4 u;
        E e[VE];
    };
#define IPT_BLOAD(K0)                                                                                   \
    do {                                                                                                \
        _Pragma("unroll") for (int q = 0; q < PA; ++q) ra[q] =                                          \
            *(const uint4 *)(Ab + (int64_t)(a_r + RPA * q) * np + (K0) + a_c);                          \
        const E *bcol = Bg + (int64_t)((K0) + b_r) * np + (cg >= 0 ? cg : 0);                           \
        _Pragma("unroll") for (int q = 0; q < NB; ++q) rb[q] = cg >= 0 ? bcol[(int64_t)RB * q * np] : (E)0; \
    } while (0)
#define IPT_BSTORE(S)                                                                                   \
    do {                                                                                                \
        _Pragma("unroll") for (int q = 0; q < PA; ++q) {                                                \
            Chunk ch;                                                                                   \
            ch.u = ra[q];                                                                               \
            _Pragma("unroll") for (int e2 = 0; e2 < VE; ++e2) As[S][a_r + RPA * q][a_c + e2] = ch.e[e2]; \
        }                                                                                               \
        _Pragma("unroll") for (int q = 0; q < NB; ++q) Bs[S][b_r + RB * q][b_c] = rb[q];                \
    } while (0)
    // 16 x 16 blocks of this wave past the problem's rows or the tile's packed columns
    // are skipped (wave-uniform bounds: scalar branches around their MFMAs)
    const int wmu = __builtin_amdgcn_readfirstlane(wm), wnu = __builtin_amdgcn_readfirstlane(wn);
    const int rows_live = n - r0 - wmu * (T / 2);
    const int cols_live = (kact - p0 < T ? kact - p0 : T) - wnu * (T / 2);
    typedef typename std::conditional<F64, d4_t, f4_t>::type ACC;
    ACC acc[MI][MI];
#pragma unroll
    for (int x = 0; x < MI; ++x)
#pragma unroll
        for (int y = 0; y < MI; ++y) acc[x][y] = ACC{0, 0, 0, 0};
    const int nk = np / BK;
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
                    if (16 * x >= rows_live || 16 * y >= cols_live) continue;
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
    // Epilogue (column c continues e_c).  The accumulators go through LDS (in two
    // halves of T/2 rows when the whole tile does not fit: the waves of row half h write
    // theirs), and each thread then owns one packed column and every (256/T)-th row, so
    // that a wave's loads and stores run along rows (coalesced for contiguous packed
    // columns) and a thread issues the loads of up to 8 rows before their arithmetic.
    // Addresses are always valid (rows < np lie in the padded buffers, empty slots read
    // column 0, theta is clamped to row n - 1); the arithmetic skips what is not there.
    typedef typename std::conditional<F64, double, float>::type Acc;
    constexpr int YP = T + 1;                                  // LDS pitch of the staged rows
    constexpr int NH = (T * YP * (int)sizeof(Acc) <= C::SMEM) ? 1 : 2;  // staging passes
    constexpr int RH = T / NH;                                 // rows staged per pass
    constexpr int G = 256 / T;                                 // threads per column
    constexpr int RPT = RH / G;                                // rows per thread and pass
    constexpr int LB = RPT < 4 ? RPT : 4;                      // rows per load batch
    static_assert(RH * YP * (int)sizeof(Acc) <= C::SMEM, "staged rows must fit in the operand LDS");
    static_assert(G * T * (NPART + 1) * 8 <= C::SMEM, "epilogue reduction must fit in the operand LDS");
    static_assert(RPT % LB == 0, "row batches");
    Acc(*ys)[YP] = (Acc(*)[YP])smem;
    const double *tb = a.theta + m.offt;
    float *zlo_out = F64 ? nullptr : (in_buf ? a.zlo0 : a.zlo1) + m.offz;
    // Delta_cj of the next d: for an exactly symmetric Delta_b it is the coalesced Delta_jc
    const bool sym = a.col.asym[b] == 0;
    const bool need_jc = !F64 || sym;
    const int cc = tid % T, rg = tid / T;
    const int c_raw = p0 + cc < kact ? al[p0 + cc] : -1;
    const bool act = c_raw >= 0 && a.col.state[m.offc + c_raw] == COL_ACTIVE;
    const int c = act ? c_raw : 0;
    const double ti = act ? tb[c] : 0.0, dd = act ? a.col.d[m.offc + c] : 0.0;
    double sums[NPART + 1];
#pragma unroll
    for (int q2 = 0; q2 < NPART + 1; ++q2) sums[q2] = 0.0;
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        if (NH == 1 || wm == h) {
#pragma unroll
            for (int x = 0; x < MI; ++x)
#pragma unroll
                for (int y = 0; y < MI; ++y)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        // f64 MFMA: row 4r + l/16; f32 MFMA: row 4(l/16) + r (within the wave's 16-row block)
                        const int lr = F64 ? (16 * x + 4 * r + (lane >> 4)) : (16 * x + 4 * (lane >> 4) + r);
                        const int row = (NH == 1 ? wm * (T / 2) : 0) + lr;
                        ys[row][wn * (T / 2) + 16 * y + (lane & 15)] = acc[x][y][r];
                    }
        }
        __syncthreads();
#pragma unroll
        for (int q0 = 0; q0 < RPT; q0 += LB) {
            double zv[LB], av[LB], tj[LB];
            Acc yv[LB];
#pragma unroll
            for (int q1 = 0; q1 < LB; ++q1) {
                const int row = rg + G * (q0 + q1);
                const int j = r0 + h * RH + row;  // < np
                const int64_t e = (int64_t)j * np + c;
                tj[q1] = tb[j < n ? j : n - 1];
                zv[q1] = zin[e];
                av[q1] = need_jc ? Ad[e] : 0.0;
                yv[q1] = ys[row][cc];
            }
#pragma unroll
            for (int q1 = 0; q1 < LB; ++q1) {
                const int j = r0 + h * RH + rg + G * (q0 + q1);
                if (!act || j >= n) continue;
                const int64_t e = (int64_t)j * np + c;
                const double z = zv[q1];
                double wvv, st, gs, de;
                if (j == c) {
                    wvv = 1.0;
                    st = wvv - z;
                    gs = 0.0;
                    de = 0.0;
                } else {
                    const double acv = (double)yv[q1];
                    const double yy = F64 ? acv : av[q1] + acv;  // split form: Delta E exact
                    const double gap = tj[q1] - ti;
                    wvv = (z * dd - yy) / gap;
                    st = wvv - z;
                    gs = gap * st;
                    de = wvv;
                }
                zout[e] = wvv;
                if constexpr (!F64) zlo_out[e] = (float)(j == c ? 0.0 : wvv);
                sums[0] += st * st;
                sums[1] += z * z;
                sums[2] += gs * gs;
                sums[3] += de * de;
                sums[4] += (sym ? av[q1] : Ad[(int64_t)c * np + j]) * wvv;  // next sweep's d_c
            }
        }
        __syncthreads();
    }
    // per-column sums over the G row groups, in a fixed order
    double(*red)[T][NPART + 1] = (double(*)[T][NPART + 1])smem;
#pragma unroll
    for (int q2 = 0; q2 < NPART + 1; ++q2) red[rg][cc][q2] = sums[q2];
    __syncthreads();
    if (tid < T && c_raw >= 0) {
        double v[NPART + 1];
#pragma unroll
        for (int q2 = 0; q2 < NPART + 1; ++q2) {
            v[q2] = red[0][tid][q2];
#pragma unroll
            for (int g = 1; g < G; ++g) v[q2] += red[g][tid][q2];
        }
#pragma unroll
        for (int q2 = 0; q2 < NPART; ++q2) a.part[m.offp + ((int64_t)tm * n + c_raw) * NPART + q2] = v[q2];
        a.dpart[m.offq + (int64_t)tm * n + c_raw] = v[NPART];
    }
    __syncthreads();
}

// Narrow tiles (at most 16 packed columns: late sweeps, when few columns of a problem
// are left) stream the tile's Delta rows: each wave takes 16 rows and the whole K
// range, its Delta operand loaded straight into registers (32 contiguous bytes per
// lane, one K chunk ahead) and the <= 16 iterate columns staged through LDS in K chunks.
// Within a chunk the MFMA's K order is permuted -- lane group g holds k = 4g .. 4g + 3
// of each 16-wide sub-block and the MFMA of step e takes their e-th element -- and the
// B operand follows the same order.  Rows pass 64 at a time (T = 128: two passes;
// T = 32: two waves).  Needs np % 64 == 0.
constexpr int SK_KC = 64;  // K chunk of the narrow path
template <bool F64>
struct SkCfg {
    typedef typename std::conditional<F64, double, float>::type E;
    typedef typename std::conditional<F64, d4_t, f4_t>::type V4;
    static constexpr int SMEM = 2 * SK_KC * 16 * (int)sizeof(E) + 4 * 16 * (NPART + 1) * 8;
};

// Four consecutive Delta entries of a narrow-tile row at element offset k0 (32 or 16 bytes).
template <bool F64>
__device__ __forceinline__ typename SkCfg<F64>::V4 sk_load_a(const typename SkCfg<F64>::E *arow, int k0) {
    typedef typename SkCfg<F64>::V4 V4;
    if constexpr (F64) {
        const double2 *pp = (const double2 *)(arow + k0);
        const double2 lo = pp[0], hi = pp[1];
        return V4{lo.x, lo.y, hi.x, hi.y};
    } else {
        const float4 f = *(const float4 *)(arow + k0);
        return V4{f.x, f.y, f.z, f.w};
    }
}

template <bool F64>
__device__ __forceinline__ void btile_skinny(char *smem, int32_t *scol, const BArgs &a, const BatchMeta &m, int b,
                                             int tm, int tn, int32_t t, int32_t acx) {
    typedef SkCfg<F64> C;
    typedef typename C::E E;
    typedef typename C::V4 V4;
    const int T = m.T;
    E(*Bs)[SK_KC][16] = (E(*)[SK_KC][16])smem;
    double(*red)[16][NPART + 1] = (double(*)[16][NPART + 1])(smem + 2 * SK_KC * 16 * sizeof(E));
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 4, lc = lane & 15;
    const int n = m.n, np = m.np;
    int32_t q, pc;
    acx_phase(acx, t, q, pc);
    const int32_t in_buf = acx ? q : (t - 1) & 1, out_buf = acx ? q + 1 : in_buf ^ 1;
    const double *Ad = a.dpad + m.offz;
    const double *zin = a.zs[in_buf] + m.offz;
    double *zout = a.zs[out_buf] + m.offz;
    const E *Ag = F64 ? (const E *)Ad : (const E *)(a.d32 + m.offz);
    const E *Bg = F64 ? (const E *)zin : (const E *)((in_buf ? a.zlo1 : a.zlo0) + m.offz);
    float *zlo_out = F64 ? nullptr : (in_buf ? a.zlo0 : a.zlo1) + m.offz;
    const int r0 = tm * T;
    (void)tn;
    const double *tb = a.theta + m.offt;
    const bool sym = a.col.asym[b] == 0;
    const bool need_jc = !F64 || sym;
    // this lane's epilogue column, and the B column of this thread (the same: tid % 16),
    // from the tile's column list the plan wrote
    const int32_t *nc = a.ncols + (int64_t)b * 16;
    const int c_raw = nc[lc];
    const bool act = c_raw >= 0 && a.col.state[m.offc + c_raw] == COL_ACTIVE;
    const int c = act ? c_raw : 0;
    const double ti = act ? tb[c] : 0.0, dd = act ? a.col.d[m.offc + c] : 0.0;
    // B staging: thread -> (k row (tid + 256 i) / 16, column tid % 16), four entries per chunk
    const int bcol = c_raw;
    double sums[NPART + 1];
#pragma unroll
    for (int q2 = 0; q2 < NPART + 1; ++q2) sums[q2] = 0.0;
    const int nch = np / SK_KC;
    const int PASSES = T >= 64 ? T / 64 : 1;
    const bool wave_rows = wv * 16 < T;  // T = 32: waves 2 and 3 hold no rows
    for (int pass = 0; pass < PASSES; ++pass) {
        const int rw = r0 + pass * 64 + wv * 16;  // first row of this wave
        const E *arow = Ag + (int64_t)(wave_rows ? rw + lc : r0) * np + 4 * g;
        V4 acc = V4{0, 0, 0, 0};
        V4 av[4];
        E bv[4];
        auto load_b = [&](int ch) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int kr = (tid + 256 * i) >> 4;
                bv[i] = bcol >= 0 ? Bg[(int64_t)(ch * SK_KC + kr) * np + bcol] : (E)0;
            }
        };
        // sub-block s2 of a chunk in av[s2], refilled with the next chunk's sub-block right
        // after the MFMAs that read it
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) av[s2] = sk_load_a<F64>(arow, 16 * s2);
        load_b(0);
#pragma unroll
        for (int i = 0; i < 4; ++i) Bs[0][(tid + 256 * i) >> 4][(tid + 256 * i) & 15] = bv[i];
        __syncthreads();
        for (int ch = 0; ch < nch; ++ch) {
            const int cur = ch & 1, nxt = ch + 1 < nch ? ch + 1 : ch;
            load_b(nxt);
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) {
                if (wave_rows) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const E fb = Bs[cur][16 * s2 + 4 * g + e][lc];
                        if constexpr (F64)
                            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s2][e], fb, acc, 0, 0, 0);
                        else
                            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s2][e], fb, acc, 0, 0, 0);
                    }
                }
                av[s2] = sk_load_a<F64>(arow, nxt * SK_KC + 16 * s2);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) Bs[cur ^ 1][(tid + 256 * i) >> 4][(tid + 256 * i) & 15] = bv[i];
            __syncthreads();
        }
        if (!wave_rows) continue;
        // epilogue of the wave's 16 rows x 16 columns: lane holds 4 rows of column lc
        double zv[4], ajc[4], tj[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int lr = F64 ? (4 * r + g) : (4 * g + r);
            const int j = rw + lr;  // < np
            const int64_t e = (int64_t)j * np + c;
            tj[r] = tb[j < n ? j : n - 1];
            zv[r] = zin[e];
            ajc[r] = need_jc ? Ad[e] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int lr = F64 ? (4 * r + g) : (4 * g + r);
            const int j = rw + lr;
            if (!act || j >= n) continue;
            const int64_t e = (int64_t)j * np + c;
            const double z = zv[r];
            double wvv, st, gs, de;
            if (j == c) {
                wvv = 1.0;
                st = wvv - z;
                gs = 0.0;
                de = 0.0;
            } else {
                const double acv = (double)acc[r];
                const double yy = F64 ? acv : ajc[r] + acv;  // split form: Delta E exact
                const double gap = tj[r] - ti;
                wvv = (z * dd - yy) / gap;
                st = wvv - z;
                gs = gap * st;
                de = wvv;
            }
            zout[e] = wvv;
            if constexpr (!F64) zlo_out[e] = (float)(j == c ? 0.0 : wvv);
            sums[0] += st * st;
            sums[1] += z * z;
            sums[2] += gs * gs;
            sums[3] += de * de;
            sums[4] += (sym ? ajc[r] : Ad[(int64_t)c * np + j]) * wvv;  // next sweep's d_c
        }
    }
    // per-column sums: the 4 lane groups, then the waves in order
#pragma unroll
    for (int q2 = 0; q2 < NPART + 1; ++q2) {
        double v = sums[q2];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (g == 0) red[wv][lc][q2] = v;
    }
    __syncthreads();
    if (tid < 16) {
        const int cc = nc[tid];
        if (cc >= 0) {
            double v[NPART + 1];
#pragma unroll
            for (int q2 = 0; q2 < NPART + 1; ++q2) v[q2] = ((red[0][tid][q2] + red[1][tid][q2]) + red[2][tid][q2]) + red[3][tid][q2];
#pragma unroll
            for (int q2 = 0; q2 < NPART; ++q2) a.part[m.offp + ((int64_t)tm * n + cc) * NPART + q2] = v[q2];
            a.dpart[m.offq + (int64_t)tm * n + cc] = v[NPART];
        }
    }
    __syncthreads();
}

// Next work item of a persistent GEMM block (thread 0): its own die's segment first,
// then the others in turn; a drained segment is left for good.  -1 when none is left.
__device__ inline int32_t next_item(const int32_t *counts, int32_t *tickets, int32_t segcap, int &x, int &left) {
    while (left > 0) {
        const int32_t cnt = counts[x];
        // a segment seen drained (tickets only grow) is skipped without an atomic
        if (__hip_atomic_load(&tickets[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < cnt) {
            const int32_t tk = atomicAdd(&tickets[x], 1);
            if (tk < cnt) return x * segcap + tk;
        }
        x = (x + 1) % NXCD;
        --left;
    }
    return -1;
}

// Items of a class in the running sweep (all segments): a block of an empty launch
// leaves at once.
__device__ inline bool class_empty(const int32_t *counts) {
    __shared__ int32_t s_total;
    if (threadIdx.x == 0) {
        int32_t tot = 0;
        for (int x = 0; x < NXCD; ++x) tot += counts[x];
        s_total = tot;
    }
    __syncthreads();
    return s_total == 0;
}

// Persistent GEMM over the narrow-tile list (items of any tile size).
__global__ __launch_bounds__(256, 4) void k_bnarrow(const Ctrl *ctrl, BArgs a, BatchLists lists, int32_t acx) {
    if (ctrl->error || ctrl->done) return;
    const int32_t t = cur_sweep(ctrl);
    const int4 *items = lists.l[CLS_NARROW][t & 1];
    const int32_t *counts = lists.counts + (2 * CLS_NARROW + (t & 1)) * NXCD;
    int32_t *tickets = lists.tickets + CLS_NARROW * NXCD;
    constexpr int SM = SkCfg<true>::SMEM > SkCfg<false>::SMEM ? SkCfg<true>::SMEM : SkCfg<false>::SMEM;
    __shared__ __attribute__((aligned(16))) char smem[SM];
    __shared__ int32_t scol[16];
    __shared__ int32_t cur_item;
    if (class_empty(counts)) return;
    int x = blockIdx.x % NXCD, left = NXCD;
    const int32_t segcap = lists.segcap[CLS_NARROW];
    if (threadIdx.x == 0) cur_item = next_item(counts, tickets, segcap, x, left);
    __syncthreads();
    for (;;) {
        const int32_t it = __builtin_amdgcn_readfirstlane(cur_item);  // uniform: the item lives in scalar registers
        if (it < 0) break;
        // the ticket of the following item is taken now; its latency hides behind this item
        int32_t tk = 0;
        if (threadIdx.x == 0) tk = atomicAdd(&tickets[x], 1);
        const int4 w = items[it];
        const BatchMeta m = a.meta[w.x];
        if (w.w == PREC_F64) btile_skinny<true>(smem, scol, a, m, w.x, w.y, w.z, t, acx);
        else btile_skinny<false>(smem, scol, a, m, w.x, w.y, w.z, t, acx);
        // (the tile ends with a barrier: every thread has read cur_item)
        if (threadIdx.x == 0) {
            if (tk < counts[x]) {
                cur_item = x * segcap + tk;
            } else {  // this segment is drained: the other dies' segments in turn
                x = (x + 1) % NXCD;
                --left;
                cur_item = next_item(counts, tickets, segcap, x, left);
            }
        }
        __syncthreads();
    }
}

template <int T>
__global__ __launch_bounds__(256, (T == 128 ? 2 : (T == 64 ? 4 : 5))) void k_bgemm(const Ctrl *ctrl, BArgs a,
                                                                                   BatchLists lists, int32_t acx) {
    if (ctrl->error || ctrl->done) return;
    constexpr int C = tile_class<T>();
    const int32_t t = cur_sweep(ctrl);
    const int4 *items = lists.l[C][t & 1];
    const int32_t *counts = lists.counts + (2 * C + (t & 1)) * NXCD;
    int32_t *tickets = lists.tickets + C * NXCD;
    __shared__ __attribute__((aligned(16))) char smem[bsmem<T>()];
    __shared__ int32_t scol[T];
    __shared__ int32_t cur_item;
    if (class_empty(counts)) return;
    int x = blockIdx.x % NXCD, left = NXCD;
    const int32_t segcap = lists.segcap[C];
    if (threadIdx.x == 0) cur_item = next_item(counts, tickets, segcap, x, left);
    __syncthreads();
    for (;;) {
        const int32_t it = __builtin_amdgcn_readfirstlane(cur_item);  // uniform: the item lives in scalar registers
        if (it < 0) break;
        // the ticket of the following item is taken now; its latency hides behind this item
        int32_t tk = 0;
        if (threadIdx.x == 0) tk = atomicAdd(&tickets[x], 1);
        const int4 w = items[it];
        const BatchMeta m = a.meta[w.x];
        if (a.tflag[m.offf + w.z] == (uint32_t)PREC_F64) btile<T, true>(smem, scol, a, m, w.x, w.y, w.z, t, acx);
        else btile<T, false>(smem, scol, a, m, w.x, w.y, w.z, t, acx);
        // (the tile ends with a barrier: every thread has read cur_item)
        if (threadIdx.x == 0) {
            if (tk < counts[x]) {
                cur_item = x * segcap + tk;
            } else {  // this segment is drained: the other dies' segments in turn
                x = (x + 1) % NXCD;
                --left;
                cur_item = next_item(counts, tickets, segcap, x, left);
            }
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------- finalize
// Per column of every problem: reduce its problem's row-tile partials in order, form
// s_c, decide (only an FP64 or product-free sweep certifies); a column that stays
// active gets its next d (the epilogue partials, in row-tile order) and stamps its
// column tile with the precision it needs next.  The first stamp of a tile in a sweep
// enqueues the tile's row tiles for the next sweep (one list append per block and
// tile class).  Batch counters go to per-block partials, reduced by the control
// kernel in block order.
enum { BP_MAXSTEP, BP_DECSTEP, BP_STILL, BP_CONV, BP_DIV, BP_NC, BP_F32, BP_WORDS = 8 };

__global__ __launch_bounds__(256) void k_bfinalize(Ctrl *ctrl, DevOpts o, BArgs a, int64_t total_cols) {
    if (ctrl->error || ctrl->done) return;
    const int32_t t = cur_sweep(ctrl);
    const int64_t gc = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool inb = gc < total_cols;
    int32_t decided = -1, prec = 0;
    double s = 0.0;
    bool act = false, still = false;
    uint32_t want = 0;
    int64_t prob_key = -1;
    uint64_t norm_v = 0;
    BatchMeta m{};
    int c = 0;
    if (inb) {
        const int b = a.col.prob[gc];
        m = a.meta[b];
        c = (int)(gc - m.offc);
        prob_key = b;
        const int nt = m.np / m.T;
        if (t == 1) {  // |M_b|_1 from the first sweep's column sums
            double cs = 0.0;
            for (int q = 0; q < nt; ++q) cs += a.normpart[m.offq + (int64_t)q * m.n + c];
            norm_v = dbits(cs);
        }
        act = a.col.state[gc] == COL_ACTIVE;
        if (act) {
            double p[NPART] = {0.0, 0.0, 0.0, 0.0};
            for (int rt = 0; rt < nt; ++rt) {
                const double4 v = *(const double4 *)&a.part[m.offp + ((int64_t)rt * m.n + c) * NPART];
                p[0] += v.x;
                p[1] += v.y;
                p[2] += v.z;
                p[3] += v.w;
            }
            s = sqrt(p[0]) / sqrt(p[1]);
            const double dist = sqrt(p[3]);
            prec = (t == 1) ? PREC_EXACT_FIRST : a.col.cprec[gc];
            const bool exact = prec == PREC_F64 || prec == PREC_EXACT_FIRST;
            const double resid = sqrt(p[2]) / sqrt(p[1]);  // normalised by |M_b|_1 at copy-out
            // IPT-ACX: only the first application of a cycle is tested (slot 0 -> 1)
            int32_t q, pc;
            acx_phase(o.acx, t, q, pc);
            const int32_t in_par = (t == 1) ? PAR_UNIT : (o.acx ? PAR_BUF0 : ((t - 1) & 1));
            const int32_t out_par = o.acx ? PAR_BUF1 : (t & 1);
            const double prev = a.col.prev[gc];
            if (q != 0) {
                // mid-cycle application: no decision
            } else if (exact && s <= o.tol) {
                decided = COL_CONVERGED;
                a.col.par[gc] = in_par;
            } else {
                const bool bad = !isfinite(s) || !(dist <= o.div_norm);
                int32_t grow = a.col.grow[gc];
                if (exact) {
                    grow = (s > prev) ? grow + 1 : 0;
                    a.col.grow[gc] = grow;
                }
                if (bad || grow >= o.div_growth) {
                    decided = COL_DIVERGED;
                    a.col.par[gc] = out_par;
                } else if (t + pc > o.max_iter) {
                    decided = COL_NOT_CONVERGED;
                    a.col.par[gc] = out_par;
                }
            }
            if (q == 0) a.col.prev[gc] = s;
            if (decided >= 0) {
                a.col.state[gc] = decided;
                a.col.sweeps[gc] = t;
                a.col.step[gc] = s;
                a.col.lam[gc] = a.theta[m.offt + c] + a.col.d[gc];
                a.col.resid[gc] = resid;
            } else {
                still = true;
                double dn = 0.0;
                for (int r2 = 0; r2 < nt; ++r2) dn += a.dpart[m.offq + (int64_t)r2 * m.n + c];
                if (o.acx) {  // d of every slot of the cycle, for the extrapolated iterate's d
                    if (q == 0) a.col.dslot[gc] = a.col.d[gc];
                    a.col.dslot[(int64_t)(q + 1) * total_cols + gc] = dn;
                }
                a.col.d[gc] = dn;
                want = PREC_F64;
                if (o.ladder && prec != PREC_F64) want = (s <= o.tau_32 || !(s < prev)) ? PREC_F64 : PREC_F32;
                a.col.want[gc] = (int32_t)want;
            }
        }
    }
    if (t == 1) {
        bool nl;
        const uint64_t nv = seg_max(prob_key, norm_v, nl);
        if (nl && inb) atomicMax((unsigned long long *)&a.col.norm_bits[prob_key], (unsigned long long)nv);
    }
    // batch counters: wave reductions, then a per-block partial
    uint64_t v = act ? dbits(s) : 0;
    uint64_t dv = decided >= 0 ? dbits(s) : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t q1 = (uint64_t)__shfl_xor((unsigned long long)v, off);
        const uint64_t q2 = (uint64_t)__shfl_xor((unsigned long long)dv, off);
        v = q1 > v ? q1 : v;
        dv = q2 > dv ? q2 : dv;
    }
    __shared__ uint64_t s_w[4][BP_WORDS];
    if (lane == 0) {
        s_w[wave][BP_MAXSTEP] = v;
        s_w[wave][BP_DECSTEP] = dv;
    }
    const uint64_t m_still = __ballot(still), m_conv = __ballot(decided == COL_CONVERGED),
                   m_div = __ballot(decided == COL_DIVERGED), m_nc = __ballot(decided == COL_NOT_CONVERGED),
                   m_f32 = __ballot(act && prec == PREC_F32);
    if (lane == 0) {
        s_w[wave][BP_STILL] = __popcll(m_still);
        s_w[wave][BP_CONV] = __popcll(m_conv);
        s_w[wave][BP_DIV] = __popcll(m_div);
        s_w[wave][BP_NC] = __popcll(m_nc);
        s_w[wave][BP_F32] = m_f32 ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x < BP_WORDS) {
        const int q = threadIdx.x;
        uint64_t r;
        if (q <= BP_DECSTEP || q == BP_F32) {
            r = s_w[0][q];
            for (int w2 = 1; w2 < 4; ++w2) r = s_w[w2][q] > r ? s_w[w2][q] : r;
        } else {
            r = s_w[0][q] + s_w[1][q] + s_w[2][q] + s_w[3][q];
        }
        if (q == BP_WORDS - 1) r = 0;
        a.bpart[(int64_t)blockIdx.x * BP_WORDS + q] = r;
    }
}

// Plan of the next sweep, one block per problem: the still-active columns in
// ascending order (packed positions), the precision of each packed column tile (the
// highest its columns ask for), each column's precision, and the work items (row
// tile, packed column tile) appended to the next sweep's list of its tile class.
__global__ __launch_bounds__(256) void k_bplan(const Ctrl *ctrl, BArgs a, BatchLists lists) {
    if (ctrl->error || ctrl->done) return;
    const int32_t t = cur_sweep(ctrl);  // the sweep just finalized
    const int b = blockIdx.x;
    const BatchMeta m = a.meta[b];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ int s_w[4];
    __shared__ int s_base, s_items, s_items2;
    __shared__ uint32_t s_tprec[128];  // n <= 4096, T >= 32
    for (int i = threadIdx.x; i < 128; i += 256) s_tprec[i] = 0;
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    int32_t *al = a.col.alist + m.offc;
    for (int c0 = 0; c0 < m.n; c0 += 256) {
        const int c = c0 + threadIdx.x;
        const bool act = c < m.n && a.col.state[m.offc + c] == COL_ACTIVE;
        const int inc = wave_incl_scan(act ? 1 : 0);
        if (lane == 63) s_w[wave] = inc;
        __syncthreads();
        int pos = s_base + inc - (act ? 1 : 0);
        for (int w2 = 0; w2 < wave; ++w2) pos += s_w[w2];
        if (act) {
            al[pos] = c;
            atomicMax(&s_tprec[pos / m.T], (uint32_t)a.col.want[m.offc + c]);
        }
        __syncthreads();
        if (threadIdx.x == 0) s_base += s_w[0] + s_w[1] + s_w[2] + s_w[3];
        __syncthreads();
    }
    const int kact = s_base;
    const int tiles = (kact + m.T - 1) / m.T, nt = m.np / m.T;
    for (int pos = threadIdx.x; pos < kact; pos += 256) a.col.cprec[m.offc + al[pos]] = (int32_t)s_tprec[pos / m.T];
    for (int tn = threadIdx.x; tn < tiles; tn += 256) a.tflag[m.offf + tn] = s_tprec[tn];
    const int cl = tile_class_of(m.T), nx = (t + 1) & 1;
    // a last column tile of at most 16 columns goes to the narrow list (only the last
    // one can be: every tile before it is full)
    const bool narrow = tiles > 0 && kact - (tiles - 1) * m.T <= 16 && m.np % SK_KC == 0;
    const int wide = narrow ? tiles - 1 : tiles;
    if (threadIdx.x == 0) {
        a.col.kact[b] = kact;
        s_items = wide ? atomicAdd(&lists.counts[(2 * cl + nx) * NXCD + m.xcd], wide * nt) : 0;
        s_items2 = narrow ? atomicAdd(&lists.counts[(2 * CLS_NARROW + nx) * NXCD + m.xcd], nt) : 0;
    }
    __syncthreads();
    int4 *lst = lists.l[cl][nx] + (int64_t)m.xcd * lists.segcap[cl];
    for (int e = threadIdx.x; e < wide * nt; e += 256) lst[s_items + e] = make_int4(b, e % nt, e / nt, 0);
    if (narrow) {
        // the narrow items carry the tile's precision; its columns go to ncols
        const int p0 = (tiles - 1) * m.T;
        if (threadIdx.x < 16) a.ncols[(int64_t)b * 16 + threadIdx.x] = p0 + threadIdx.x < kact ? al[p0 + threadIdx.x] : -1;
        int4 *ln = lists.l[CLS_NARROW][nx] + (int64_t)m.xcd * lists.segcap[CLS_NARROW];
        const int prec = (int)s_tprec[tiles - 1];
        for (int e = threadIdx.x; e < nt; e += 256) ln[s_items2 + e] = make_int4(b, e, tiles - 1, prec);
    }
}

// Sweep bookkeeping of the batch: reduce the finalize blocks' partials in block
// order, then history, done flag, device sweep counter, and reset of the work-list
// counters and tickets this sweep consumed.  One block.
__global__ __launch_bounds__(256) void k_bcontrol(Ctrl *ctrl, DevOpts o, BArgs a, int32_t nblk, BatchLists lists) {
    if (ctrl->error || ctrl->done) return;
    __shared__ uint64_t r[256][BP_WORDS];
    uint64_t acc[BP_WORDS] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int bi = threadIdx.x; bi < nblk; bi += 256) {
        const uint64_t *p = a.bpart + (int64_t)bi * BP_WORDS;
#pragma unroll
        for (int q = 0; q < BP_WORDS; ++q) {
            const uint64_t x = p[q];
            if (q <= BP_DECSTEP || q == BP_F32) acc[q] = x > acc[q] ? x : acc[q];
            else acc[q] += x;
        }
    }
#pragma unroll
    for (int q = 0; q < BP_WORDS; ++q) r[threadIdx.x][q] = acc[q];
    __syncthreads();
    for (int half = 128; half > 0; half >>= 1) {
        if (threadIdx.x < half) {
#pragma unroll
            for (int q = 0; q < BP_WORDS; ++q) {
                const uint64_t x = r[threadIdx.x + half][q], y = r[threadIdx.x][q];
                r[threadIdx.x][q] = (q <= BP_DECSTEP || q == BP_F32) ? (x > y ? x : y) : x + y;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const int32_t t = cur_sweep(ctrl);
    const double ms = bitsd(r[0][BP_MAXSTEP]);
    if (r[0][BP_DECSTEP] > ctrl->dec_maxstep) ctrl->dec_maxstep = r[0][BP_DECSTEP];
    ctrl->n_conv += (int32_t)r[0][BP_CONV];
    ctrl->n_div += (int32_t)r[0][BP_DIV];
    ctrl->n_notconv += (int32_t)r[0][BP_NC];
    // a sweep counts as FP32 when any of its tiles ran in FP32
    const int32_t prec = (t == 1) ? PREC_EXACT_FIRST : (r[0][BP_F32] ? PREC_F32 : PREC_F64);
    if (t - 1 < IPT_HIST) {
        ctrl->hist_prec[t - 1] = prec;
        ctrl->hist_active[t - 1] = ctrl->active;
        ctrl->hist_step[t - 1] = ms;
    }
    if (t > 1) ctrl->matvecs += ctrl->active;
    ctrl->active = (int32_t)r[0][BP_STILL];
    ctrl->sweeps = t;
    if (ctrl->active == 0 || t >= o.max_iter) ctrl->done = 1;
    for (int cl = 0; cl < NCLS; ++cl)
        for (int x = 0; x < NXCD; ++x) {
            lists.counts[(2 * cl + (t & 1)) * NXCD + x] = 0;
            lists.tickets[cl * NXCD + x] = 0;
        }
}

// Outputs: the final iterate of each column into z_pool (row-major, leading dimension
// n_b), lambda, status; the eigen-residual is normalised by |M_b|_1 here.  Item =
// (problem, row tile, 64 columns), as for the first sweep.
__global__ __launch_bounds__(256) void k_bcopyout(const Ctrl *ctrl, BArgs a, const int4 *items, int64_t nitems,
                                                  double *z_pool, double *lambda_pool, int32_t *status_pool,
                                                  double *max_resid_out, int32_t *ci_sweeps, double *ci_step,
                                                  double *ci_resid) {
    if (ctrl->error) return;
    const int cx = threadIdx.x & 63, ry = threadIdx.x >> 6;
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int4 w = items[__builtin_amdgcn_readfirstlane((int32_t)it)];
        const BatchMeta m = a.meta[w.x];
        const int n = m.n, np = m.np, tm = w.y;
        const int c = w.z * 64 + cx;
        const bool ok = c < n;
        const int64_t gc = m.offc + c;
        if (ok) {
            const int32_t par = a.col.par[gc];
            const double *src = a.zs[par == PAR_BUF1 ? 1 : 0] + m.offz;
            double *dst = z_pool + m.offo;
            const int j1 = min(n, tm * m.T + m.T);
            // eight rows' loads in flight before their stores (rows < np are inside the
            // padded buffer, so the loads need no bounds check)
            for (int j0 = tm * m.T + ry; j0 < j1; j0 += 32) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int j = j0 + 4 * u;
                    v[u] = (par == PAR_UNIT) ? (j == c ? 1.0 : 0.0) : src[(int64_t)(j < np ? j : np - 1) * np + c];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (j0 + 4 * u < j1) dst[(int64_t)(j0 + 4 * u) * n + c] = v[u];
            }
        }
        if (tm == 0 && ry == 0) {  // one wave per item: per-column outputs
            uint64_t rb = 0;
            if (ok) {
                lambda_pool[m.offt + c] = a.col.lam[gc];
                const int32_t st = a.col.state[gc];
                status_pool[m.offt + c] = st == COL_ACTIVE ? IPT_NOT_CONVERGED : st;
                const double nrm = bitsd(a.col.norm_bits[w.x]);
                const double r = a.col.resid[gc] / (nrm > 0.0 ? nrm : 1.0);
                a.col.resid[gc] = r;
                if (st == COL_CONVERGED) rb = dbits(r);
                if (ci_sweeps) ci_sweeps[m.offt + c] = a.col.sweeps[gc];
                if (ci_step) ci_step[m.offt + c] = a.col.step[gc];
                if (ci_resid) ci_resid[m.offt + c] = r;
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const uint64_t q = (uint64_t)__shfl_xor((unsigned long long)rb, off);
                rb = q > rb ? q : rb;
            }
            if (cx == 0 && rb) atomicMax((unsigned long long *)max_resid_out, (unsigned long long)rb);
        }
    }
}

// ------------------------------------------------------------------ IPT-ACX
// After the last application of a cycle of order p (sweep t = ctrl->sweeps), every
// active column moves to z + sum_q binom(p, q) sigma^q D^q (D^q the forward
// differences of its slots z, F(z), ..., F^p(z); sigma = |<D^p, D^(p-1)>| / |D^p|^2,
// 1 when D^p = 0), and its d follows by linearity from the d of the slots.  The
// tiles are those of the next sweep's work lists (every tile holding an active
// column); a tile's partial sums go to the per-row-tile arrays dpart (dot) and
// normpart (squared norm), free at this point of the sweep.
__device__ inline bool acx_cycle_end(const Ctrl *ctrl, int32_t &t, int32_t &pc) {
    if (ctrl->error || ctrl->done) return false;
    t = ctrl->sweeps;
    int32_t q;
    acx_phase(1, t, q, pc);
    return q == pc - 1;
}

// Item it of the next sweep's work, counted over the classes and die segments in turn.
__device__ inline bool acx_item(const BatchLists &lists, int32_t t, int64_t it, int4 &w) {
    const int nx = (t + 1) & 1;
    int64_t base = 0;
    for (int cl = 0; cl < NCLS; ++cl)
        for (int x = 0; x < NXCD; ++x) {
            const int64_t cnt = lists.counts[(2 * cl + nx) * NXCD + x];
            if (it < base + cnt) {
                w = lists.l[cl][nx][(int64_t)x * lists.segcap[cl] + (it - base)];
                return true;
            }
            base += cnt;
        }
    return false;
}

__device__ inline int64_t acx_total(const BatchLists &lists, int32_t t) {
    const int nx = (t + 1) & 1;
    int64_t total = 0;
    for (int cl = 0; cl < NCLS; ++cl)
        for (int x = 0; x < NXCD; ++x) total += lists.counts[(2 * cl + nx) * NXCD + x];
    return total;
}

__device__ inline void acx_diffs(int32_t p, double z, double a1, double a2, double a3, double &d1, double &d2,
                                 double &d3) {
    d1 = a1 - z;
    d2 = (a2 - 2.0 * a1) + z;
    d3 = p == 3 ? ((a3 - 3.0 * a2) + 3.0 * a1) - z : 0.0;
}

__global__ __launch_bounds__(256) void k_bacx_dots(const Ctrl *ctrl, BArgs a, BatchLists lists) {
    int32_t t, pc;
    if (!acx_cycle_end(ctrl, t, pc)) return;
    __shared__ double sh[2][256];
    const int64_t total = acx_total(lists, t);
    for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
        int4 w;
        acx_item(lists, t, it, w);
        const BatchMeta m = a.meta[w.x];
        const int T = m.T, n = m.n, np = m.np;
        const int cc = threadIdx.x % T, rg = threadIdx.x / T, ngr = 256 / T;
        const int pi = w.z * T + cc;
        const int c = pi < a.col.kact[w.x] ? a.col.alist[m.offc + pi] : -1;
        const bool act = c >= 0 && a.col.state[m.offc + c] == COL_ACTIVE;
        double dot = 0.0, nrm = 0.0;
        if (act) {
            const int j1 = min(n, w.y * T + T);
            for (int j = w.y * T + rg; j < j1; j += ngr) {
                const int64_t e = m.offz + (int64_t)j * np + c;
                double d1, d2, d3;
                acx_diffs(pc, a.zs[0][e], a.zs[1][e], a.zs[2][e], pc == 3 ? a.zs[3][e] : 0.0, d1, d2, d3);
                const double hi = pc == 3 ? d3 : d2, lo = pc == 3 ? d2 : d1;
                dot += hi * lo;
                nrm += hi * hi;
            }
        }
        sh[0][threadIdx.x] = dot;
        sh[1][threadIdx.x] = nrm;
        __syncthreads();
        if (rg == 0 && act) {
            double sd = 0.0, sn = 0.0;
            for (int g = 0; g < ngr; ++g) {
                sd += sh[0][g * T + cc];
                sn += sh[1][g * T + cc];
            }
            a.dpart[m.offq + (int64_t)w.y * n + c] = sd;
            a.normpart[m.offq + (int64_t)w.y * n + c] = sn;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_bacx_update(const Ctrl *ctrl, BArgs a, BatchLists lists, int64_t total_cols) {
    int32_t t, pc;
    if (!acx_cycle_end(ctrl, t, pc)) return;
    const int64_t total = acx_total(lists, t);
    for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
        int4 w;
        acx_item(lists, t, it, w);
        const BatchMeta m = a.meta[w.x];
        const int T = m.T, n = m.n, np = m.np, nt = np / T;
        const int cc = threadIdx.x % T, rg = threadIdx.x / T, ngr = 256 / T;
        const int pi = w.z * T + cc;
        const int c = pi < a.col.kact[w.x] ? a.col.alist[m.offc + pi] : -1;
        if (c < 0 || a.col.state[m.offc + c] != COL_ACTIVE) continue;
        double sd = 0.0, sn = 0.0;
        for (int r = 0; r < nt; ++r) {
            sd += a.dpart[m.offq + (int64_t)r * n + c];
            sn += a.normpart[m.offq + (int64_t)r * n + c];
        }
        const double sg = sn > 0.0 ? fabs(sd) / sn : 1.0;
        const int j1 = min(n, w.y * T + T);
        for (int j = w.y * T + rg; j < j1; j += ngr) {
            const int64_t e = m.offz + (int64_t)j * np + c;
            const double z = a.zs[0][e];
            double d1, d2, d3;
            acx_diffs(pc, z, a.zs[1][e], a.zs[2][e], pc == 3 ? a.zs[3][e] : 0.0, d1, d2, d3);
            a.zs[0][e] = pc == 3 ? ((z + 3.0 * sg * d1) + 3.0 * (sg * sg) * d2) + (sg * sg * sg) * d3
                                 : (z + 2.0 * sg * d1) + (sg * sg) * d2;
        }
        if (w.y == 0 && rg == 0) {
            const int64_t gc = m.offc + c;
            const double *ds = a.col.dslot;
            double d1, d2, d3;
            const double d0 = ds[gc];
            acx_diffs(pc, d0, ds[total_cols + gc], ds[2 * total_cols + gc], pc == 3 ? ds[3 * total_cols + gc] : 0.0,
                      d1, d2, d3);
            a.col.d[gc] = pc == 3 ? ((d0 + 3.0 * sg * d1) + 3.0 * (sg * sg) * d2) + (sg * sg * sg) * d3
                                  : (d0 + 2.0 * sg * d1) + (sg * sg) * d2;
        }
    }
}

}  // namespace

// ------------------------------------------------------------- launchers
int bgemm_grid(int tile) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 512;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    hipError_t e = tile == 32   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_bgemm<32>, 256, 0)
                   : tile == 64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_bgemm<64>, 256, 0)
                                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_bgemm<128>, 256, 0);
    if (e != hipSuccess || per <= 0) per = 1;
    return cus * per;
}

int bfinalize_blocks(int64_t total_cols) { return (int)((total_cols + 255) / 256); }

hipError_t launch_binit(hipStream_t s, Ctrl *ctrl, const BatchLaunch &L, int32_t count, int32_t start_prec) {
    k_binit<<<count, 256, 0, s>>>(ctrl, L, start_prec);
    return hipGetLastError();
}

hipError_t launch_bsweep1(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, const int4 *items, int64_t nitems,
                          int32_t ladder, int32_t acx) {
    const int g = nitems < 8192 ? (int)nitems : 8192;
    k_bsweep1<<<g > 0 ? g : 1, 256, 0, s>>>(ctrl, L, items, nitems, ladder, acx);
    return hipGetLastError();
}

int bnarrow_grid() {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 512;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_bnarrow, 256, 0) != hipSuccess || per <= 0) per = 1;
    return cus * per;
}

hipError_t launch_bnarrow(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, const BatchLists &lists, int grid,
                         int32_t acx) {
    k_bnarrow<<<grid, 256, 0, s>>>(ctrl, L, lists, acx);
    return hipGetLastError();
}

hipError_t launch_bgemm(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, const BatchLists &lists, int tile,
                        int grid, int32_t acx) {
    if (tile == 32) k_bgemm<32><<<grid, 256, 0, s>>>(ctrl, L, lists, acx);
    else if (tile == 64) k_bgemm<64><<<grid, 256, 0, s>>>(ctrl, L, lists, acx);
    else k_bgemm<128><<<grid, 256, 0, s>>>(ctrl, L, lists, acx);
    return hipGetLastError();
}

hipError_t launch_bacx(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, const BatchLists &lists,
                       int64_t total_cols) {
    k_bacx_dots<<<4096, 256, 0, s>>>(ctrl, L, lists);
    k_bacx_update<<<4096, 256, 0, s>>>(ctrl, L, lists, total_cols);
    return hipGetLastError();
}

hipError_t launch_bfinalize(hipStream_t s, Ctrl *ctrl, const DevOpts &o, const BatchLaunch &L, int64_t total_cols,
                            const BatchLists &lists) {
    (void)lists;
    k_bfinalize<<<bfinalize_blocks(total_cols), 256, 0, s>>>(ctrl, o, L, total_cols);
    return hipGetLastError();
}

hipError_t launch_bplan(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, const BatchLists &lists, int32_t count) {
    k_bplan<<<count, 256, 0, s>>>(ctrl, L, lists);
    return hipGetLastError();
}

hipError_t launch_bcontrol(hipStream_t s, Ctrl *ctrl, const DevOpts &o, const BatchLaunch &L, int64_t total_cols,
                           const BatchLists &lists) {
    k_bcontrol<<<1, 256, 0, s>>>(ctrl, o, L, bfinalize_blocks(total_cols), lists);
    return hipGetLastError();
}

hipError_t launch_bcopyout(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, const int4 *items, int64_t nitems,
                           double *z_pool, double *lambda_pool, int32_t *status_pool, double *max_resid_out,
                           int32_t *ci_sweeps, double *ci_step, double *ci_resid) {
    const int g = nitems < 8192 ? (int)nitems : 8192;
    k_bcopyout<<<g > 0 ? g : 1, 256, 0, s>>>(ctrl, L, items, nitems, z_pool, lambda_pool, status_pool, max_resid_out,
                                            ci_sweeps, ci_step, ci_resid);
    return hipGetLastError();
}

}  // namespace ipt
