// The product Y = Delta Z of an IPT sweep on the gfx950 matrix cores, with the rest
// of the sweep fused into the epilogue:
//   W_jc = (Z_jc d_c - Y_jc) / (theta_j - theta_i)  (j != i),  W_ic = 1      (eq. dyn)
// plus the per-column partial sums of |W - Z|^2, |Z|^2, |(theta_j - theta_i)(W - Z)|^2
// and |W - e_i|^2 over each 128-row tile (reduced in a fixed order by the finalize
// kernel).  By F(Z) - Z = -G o (M Z - Z Lambda), the third sum is the squared
// eigen-residual |M z - lambda z|^2 of the column.  Optionally the epilogue also
// forms sum_j Delta_ij W_jc over its rows: the finalize adds these into d of the next
// sweep (lambda = theta + diag(Delta Z) with Z = W), so that sweep needs no separate
// pass over Delta and Z for its d.
//
// Column tiles run over the packed active columns (ColState::alist, rebuilt after
// every finalize), so frozen columns cost nothing; the B operand gathers them.
//
// One kernel per sweep; the precision of the sweep is read from the device control
// block (the ladder is decided on the device, so the host never waits between
// sweeps) and selects one of two bodies:
//  * FP64: v_mfma_f64_16x16x4f64, 128x128 block tile, 4 waves of 64x64, BK = 16,
//    double-buffered LDS.  Delta (padded to a multiple of 128) and Z are read in place.
//  * low precision (BF16 / FP16 with v_mfma_f32_16x16x32_*, FP32 with
//    v_mfma_f32_16x16x4f32), FP32 accumulation, "NT" operands: Delta_lo row-major and
//    the transposed shadow of the split iterate Z - E.  The epilogue adds back
//    Delta E exactly in FP64 (Y = Delta[:, i] + Delta_lo (Z - E)_lo), so only the small
//    correction Z - E sees low precision.
#include <math.h>

#include <type_traits>

#include "ipt_internal.h"

namespace ipt {

namespace {

constexpr int BM = TILE_M, BN = TILE_N;

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));

// Block -> (row tile, column tile).  Workgroups are dispatched round-robin over the
// 8 XCDs; consecutive block ids are first regrouped per XCD so that each XCD works
// on a compact patch of tiles (8 row tiles wide) sharing Delta rows and Z columns
// in its own L2.
__device__ inline void tile_of(int bid, int nblocks, int ntm, int ntn, int &tm, int &tn) {
    const int full = nblocks & ~7;
    int pid = bid;
    if (bid < full) pid = (bid & 7) * (full >> 3) + (bid >> 3);
    constexpr int GM = 8;
    const int per_group = GM * ntn;
    const int group = pid / per_group;
    const int first_m = group * GM;
    const int gsz = (ntm - first_m) < GM ? (ntm - first_m) : GM;
    const int in = pid - group * per_group;
    tm = first_m + in % gsz;
    tn = in / gsz;
}

// Everything a sweep GEMM needs (one struct keeps the kernel signature short).
struct GemmArgs {
    const double *delta;  // FP64 Delta (padded to np rows when copied), leading dimension lda
    int64_t lda;
    const void *dlo;      // low-precision Delta shadow (np x np, leading dimension np)
    const float *d32;     // FP32 Delta shadow (np x np)
    const void *zt;       // transposed shadow of Z - E (kp x np)
    const double *zin;    // iterate Z (np x kp)
    double *zout;         // W = F(Z)
    const double *theta;
    ColState cs;
    const double *dvec;   // d_c
    double *part;         // partial sums [row tile][column][NPART]
    int64_t n, np, kp;
    int32_t low_type;     // LT_BF16 or LT_F16
    double *ypart;        // split-K partial products of narrow sweeps
    int32_t nblk;         // blocks that fill the chip (2 per CU)
    double *dnp;          // NULL, or [row tile][column] partials of d for the next sweep
    // FP32-class rung as three FP16 products (mid_x3): hi/lo FP16 shadows of the scaled
    // Delta (np x np each) and of the scaled transposed Z - E (kp x np each)
    const _Float16 *dmh, *dml, *zth, *ztl;
    int32_t mid_x3;
};

// Epilogue reduction slots: the NPART sums of the finalize, then the partial of
// d' = (Delta W)_{i,c}, the d of the next sweep (W is its input).
constexpr int NRED = NPART + 1;

// Narrow sweeps: when the packed active columns give fewer tiles than nblk, the K
// range is split S ways (S >= 2); each split writes its FP64 partial tile and a
// separate kernel sums the partials in split order and runs the epilogue.
constexpr int SPLIT_MAX = 16;
struct SplitPlan {
    int nct, S;
};
__host__ __device__ inline SplitPlan split_plan(int64_t kact, int ntm, int64_t np, int nblk) {
    SplitPlan sp;
    sp.nct = (int)((kact + BN - 1) / BN);
    const int64_t reg = (int64_t)ntm * sp.nct;
    int64_t S = reg > 0 && reg < nblk ? (nblk + reg - 1) / reg : 1;
    if (S > SPLIT_MAX) S = SPLIT_MAX;
    if (S > np / 64) S = np / 64;
    sp.S = S >= 2 ? (int)S : 1;
    return sp;
}

// The packed columns of one column tile: position i (< BN) holds column cols[i] when
// i < lim, no column otherwise.
struct PackedCols {
    const int32_t *cols;
    int32_t lim;
    __device__ int32_t operator[](int i) const { return i < lim ? cols[i] : -1; }
};

// Column blocks (16 columns each) of wave column wn that hold packed columns.  Narrow
// sweeps (the split path) skip the MFMAs of the others.
__device__ inline int live_col_blocks(int32_t lim, int wn) {
    const int v = (lim - wn * 64 + 15) >> 4;
    return v < 0 ? 0 : (v > 4 ? 4 : v);
}

constexpr int SMEM_F64 = 2 * BM * (16 + 1) * 8 + 2 * 16 * BN * 8;
constexpr int SMEM_LOW16 = 2 * 2 * BM * (64 + 8) * 2;
constexpr int SMEM_LOW32 = 2 * 2 * BM * (32 + 1) * 4;
constexpr int X3_BK = 32, X3_LDP = X3_BK;  // unpadded rows; 16-byte chunks XOR-swizzled by row
constexpr int SMEM_X3 = 2 * 4 * BM * X3_LDP * 2;  // two stages of A hi/lo and B hi/lo
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int SMEM_MAIN = cmax(cmax(SMEM_F64, SMEM_X3), cmax(SMEM_LOW16, SMEM_LOW32));

// Shared epilogue.  Each lane holds 4 column blocks (jb) x 16 rows of the block
// tile; row_of(ib, r) gives the tile row of accumulator (ib, r), which depends on
// the MFMA family.  y_of(ib, jb, r, dji) returns the FP64 product value (dji =
// Delta_ji, loaded for a low-precision product, LOW).  WANT_D: also the partials of
// the next sweep's d (e.dnp).  Both are template flags so that the unrolled loop
// carries no branches around its loads.
template <bool LOW, bool WANT_D, class RowOf, class YOf>
__device__ inline void sweep_epilogue(const GemmArgs &e, const PackedCols scol, int tm, int wm, int wn, int lane,
                                      RowOf row_of, YOf y_of, double (*red)[BN][NRED], bool sym) {
    // The loads of one row (4 column blocks) issue together before its arithmetic, at
    // addresses that are always valid (empty packed slots read column 0, rows past n
    // the zero padding, theta clamps to n - 1); the arithmetic then skips what is not
    // there.  One element at a time would leave each load's latency exposed.
    int32_t cols[4], ii[4];
    double ti[4], dd[4];
    bool act[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int32_t c = scol[wn * 64 + 16 * jb + (lane & 15)];  // packed position -> column
        act[jb] = c >= 0 && e.cs.state[c] == COL_ACTIVE;
        cols[jb] = act[jb] ? c : 0;
        ii[jb] = act[jb] ? e.cs.idx[c] : 0;
        ti[jb] = act[jb] ? e.theta[ii[jb]] : 0.0;
        dd[jb] = act[jb] ? e.dvec[c] : 0.0;
    }
    const int64_t ldzb = e.kp;
    double sums[4][NRED];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int q = 0; q < NRED; ++q) sums[jb][q] = 0.0;
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t j = (int64_t)tm * BM + wm * 64 + row_of(ib, r, lane);
            const bool rok = j < e.n;
            const double tj = e.theta[rok ? j : e.n - 1];
            double zv[4], dji[4], dij[4];
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                const int64_t a_ji = j * e.lda + ii[jb], a_ij = (int64_t)ii[jb] * e.lda + j;
                zv[jb] = e.zin[j * ldzb + cols[jb]];
                dji[jb] = LOW ? e.delta[a_ji] : 0.0;
                // Delta_ij of d'; for an exactly symmetric Delta, Delta_ji (coalesced
                // across the lanes' columns) holds the same value
                dij[jb] = WANT_D ? e.delta[sym ? a_ji : a_ij] : 0.0;
            }
            if (!rok) continue;
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                if (!act[jb]) continue;
                const double z = zv[jb];
                double w, st, gs, de;
                if (j == ii[jb]) {
                    w = 1.0;
                    st = w - z;
                    gs = 0.0;
                    de = 0.0;
                } else {
                    const double gap = tj - ti[jb];
                    w = fma(z, dd[jb], -y_of(ib, jb, r, dji[jb])) / gap;
                    st = w - z;
                    gs = gap * st;
                    de = w;
                }
                e.zout[j * ldzb + cols[jb]] = w;
                sums[jb][0] = fma(st, st, sums[jb][0]);
                sums[jb][1] = fma(z, z, sums[jb][1]);
                sums[jb][2] = fma(gs, gs, sums[jb][2]);
                sums[jb][3] = fma(de, de, sums[jb][3]);
                if constexpr (WANT_D) sums[jb][NPART] = fma(dij[jb], w, sums[jb][NPART]);
            }
        }
    // Reduce over the 4 lane groups holding the same columns (fixed pattern), then
    // over the two waves that share the column block, in a fixed order.
    constexpr int nq = WANT_D ? NRED : NPART;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int q = 0; q < nq; ++q) {
            double v = sums[jb][q];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            sums[jb][q] = v;
        }
    if (lane < 16) {
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
            for (int q = 0; q < nq; ++q) red[wm][wn * 64 + 16 * jb + lane][q] = sums[jb][q];
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < BN) {
        const int32_t c = scol[t];
        if (c >= 0) {
#pragma unroll
            for (int q = 0; q < NPART; ++q)
                e.part[((int64_t)tm * e.kp + c) * NPART + q] = red[0][t][q] + red[1][t][q];
            if constexpr (WANT_D) e.dnp[(int64_t)tm * e.kp + c] = red[0][t][NPART] + red[1][t][NPART];
        }
    }
}

// ------------------------------------------------------------------- FP64
constexpr int BK64 = 16;

template <bool SPLIT>
__device__ __forceinline__ void gemm_f64_body(char *smem, double (*red)[BN][NRED], const PackedCols scol,
                                              const GemmArgs &g, int tm, int64_t k0, int64_t k1, double *yp,
                                              bool sym) {
    typedef double ATile[BM][BK64 + 1];
    typedef double BTile[BK64][BN];
    ATile *As = (ATile *)smem;
    BTile *Bs = (BTile *)(smem + 2 * sizeof(ATile));

    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, wm = wv >> 1, wn = wv & 1;
    const int64_t lda = g.lda, ldzb = g.kp;
    const double *Ab = g.delta + (int64_t)tm * BM * lda;
    // B loader.  Contiguous packed columns (every column of the tile active, the usual
    // case): thread -> column pair 2cp, 2cp + 1 and rows rg + 4q, 16-byte loads.
    // Otherwise one gathered column per thread, rows b_r + 2q.
    const int a_r = t >> 3, a_k = 2 * (t & 7);
    const int b_c = t & (BN - 1), b_r = t >> 7;
    const int cp = t & 63, rg = t >> 6;
    const int32_t c_first = scol[0];
    const bool contig = scol.lim >= BN && scol[BN - 1] == c_first + BN - 1;
    const int32_t cg = contig ? c_first + 2 * cp : scol[b_c];
    const double *Bc = g.zin + (cg >= 0 ? cg : 0);
    const int nj = SPLIT ? live_col_blocks(scol.lim, wn) : 4;

    d4_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};

    // Register staging of the next K slice: issued before the MFMAs of the current
    // slice, written to the idle LDS stage after them (one barrier per slice).  The
    // last iteration re-reads its own slice into the idle stage, which keeps the
    // loop free of branches.
    double2 ra[4];
    double rb[8];
    const int nk = (int)((k1 - k0) / BK64);
#pragma unroll
    for (int q = 0; q < 4; ++q) ra[q] = *(const double2 *)(Ab + (int64_t)(a_r + 32 * q) * lda + k0 + a_k);
#define IPT_F64_BLOAD(K)                                                                        \
    do {                                                                                        \
        if (contig) {                                                                           \
            _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                     \
                const double2 v = *(const double2 *)(Bc + ((K) + rg + 4 * q) * ldzb);          \
                rb[2 * q] = v.x;                                                                \
                rb[2 * q + 1] = v.y;                                                            \
            }                                                                                   \
        } else {                                                                                \
            _Pragma("unroll") for (int q = 0; q < 8; ++q) rb[q] =                               \
                cg >= 0 ? Bc[((K) + b_r + 2 * q) * ldzb] : 0.0;                                 \
        }                                                                                       \
    } while (0)
#define IPT_F64_BSTORE(S)                                                                       \
    do {                                                                                        \
        if (contig) {                                                                           \
            _Pragma("unroll") for (int q = 0; q < 4; ++q)                                       \
                *(double2 *)&Bs[S][rg + 4 * q][2 * cp] = double2{rb[2 * q], rb[2 * q + 1]};     \
        } else {                                                                                \
            _Pragma("unroll") for (int q = 0; q < 8; ++q) Bs[S][b_r + 2 * q][b_c] = rb[q];      \
        }                                                                                       \
    } while (0)
    IPT_F64_BLOAD(k0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        As[0][a_r + 32 * q][a_k] = ra[q].x;
        As[0][a_r + 32 * q][a_k + 1] = ra[q].y;
    }
    IPT_F64_BSTORE(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        const int64_t kn = k0 + (int64_t)(kt + 1 < nk ? kt + 1 : kt) * BK64;
#pragma unroll
        for (int q = 0; q < 4; ++q) ra[q] = *(const double2 *)(Ab + (int64_t)(a_r + 32 * q) * lda + kn + a_k);
        IPT_F64_BLOAD(kn);
#pragma unroll
        for (int kk = 0; kk < BK64 / 4; ++kk) {
            double fa[4], fb[4];
#pragma unroll
            for (int ib = 0; ib < 4; ++ib) fa[ib] = As[cur][wm * 64 + 16 * ib + (lane & 15)][4 * kk + (lane >> 4)];
#pragma unroll
            for (int jb = 0; jb < 4; ++jb)
                fb[jb] = (!SPLIT || jb < nj) ? Bs[cur][4 * kk + (lane >> 4)][wn * 64 + 16 * jb + (lane & 15)] : 0.0;
#pragma unroll
            for (int ib = 0; ib < 4; ++ib)
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
                    if (!SPLIT || jb < nj)
                        acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[ib], fb[jb], acc[ib][jb], 0, 0, 0);
        }
        const int nx = cur ^ 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            As[nx][a_r + 32 * q][a_k] = ra[q].x;
            As[nx][a_r + 32 * q][a_k + 1] = ra[q].y;
        }
        IPT_F64_BSTORE(nx);
        __syncthreads();
    }
#undef IPT_F64_BLOAD
#undef IPT_F64_BSTORE

    // v_mfma_f64_16x16x4f64: lane l, register r holds row 4r + l/16, column l%16.
    auto row_of = [](int ib, int r, int l) { return 16 * ib + 4 * r + (l >> 4); };
    if constexpr (SPLIT) {
#pragma unroll
        for (int ib = 0; ib < 4; ++ib)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
                    if (wn * 64 + 16 * jb + (lane & 15) < scol.lim)  // empty packed columns: never read
                        yp[(int64_t)(wm * 64 + row_of(ib, r, lane)) * BN + wn * 64 + 16 * jb + (lane & 15)] =
                            acc[ib][jb][r];
    } else {
        auto y_of = [&](int ib, int jb, int r, double) { return acc[ib][jb][r]; };
        if (g.dnp) sweep_epilogue<false, true>(g, scol, tm, wm, wn, lane, row_of, y_of, red, sym);
        else sweep_epilogue<false, false>(g, scol, tm, wm, wn, lane, row_of, y_of, red, sym);
    }
}

// ------------------------------------------------------------ low precision
template <typename T>
struct LowCfg;
template <>
struct LowCfg<__bf16> {
    static constexpr int BK = 64, KSTEP = 32, VEC = 8, PAD = 8;
};
template <>
struct LowCfg<_Float16> {
    static constexpr int BK = 64, KSTEP = 32, VEC = 8, PAD = 8;
};
template <>
struct LowCfg<float> {
    static constexpr int BK = 32, KSTEP = 4, VEC = 1, PAD = 1;
};

template <typename T>
__device__ inline f4_t mfma_low(const T *a, const T *b, f4_t c);
template <>
__device__ inline f4_t mfma_low<__bf16>(const __bf16 *a, const __bf16 *b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(*(const bf8_t *)a, *(const bf8_t *)b, c, 0, 0, 0);
}
template <>
__device__ inline f4_t mfma_low<_Float16>(const _Float16 *a, const _Float16 *b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(*(const h8_t *)a, *(const h8_t *)b, c, 0, 0, 0);
}
template <>
__device__ inline f4_t mfma_low<float>(const float *a, const float *b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(*a, *b, c, 0, 0, 0);
}

// Staged 16-byte chunks -> LDS tile rows (row l_r + 32 q, elements l_c ..).
template <typename T, int EPC, int LDP>
__device__ __forceinline__ void lds_put(T (*as)[LDP], T (*bs)[LDP], const uint4 *ra, const uint4 *rb, int l_r,
                                        int l_c) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if constexpr ((LDP * sizeof(T)) % 16 == 0) {
            *(uint4 *)&as[l_r + 32 * q][l_c] = ra[q];
            *(uint4 *)&bs[l_r + 32 * q][l_c] = rb[q];
        } else {
            union {
                uint4 u;
                T e[EPC];
            } ua, ub;
            ua.u = ra[q];
            ub.u = rb[q];
#pragma unroll
            for (int e2 = 0; e2 < EPC; ++e2) {
                as[l_r + 32 * q][l_c + e2] = ua.e[e2];
                bs[l_r + 32 * q][l_c + e2] = ub.e[e2];
            }
        }
    }
}

template <typename T, bool SPLIT>
__device__ __forceinline__ void gemm_low_body(char *smem, double (*red)[BN][NRED], const PackedCols scol,
                                              const GemmArgs &g, const T *dlo, double unscale, int tm, int64_t k0,
                                              int64_t k1, double *yp, bool sym) {
    using C = LowCfg<T>;
    constexpr int BK = C::BK, LDP = C::BK + C::PAD;
    typedef T Tile[BM][LDP];
    Tile *As = (Tile *)smem;
    Tile *Bs = (Tile *)(smem + 2 * sizeof(Tile));

    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, wm = wv >> 1, wn = wv & 1;
    // Each block row of BK elements is 128 bytes = 8 chunks of 16 bytes; 256 threads
    // move 32 rows' worth of chunks per pass, 4 passes cover 128 rows.
    constexpr int EPC = 16 / sizeof(T);  // elements per 16-byte chunk
    const int l_r = t >> 3, l_c = (t & 7) * EPC;
    const int64_t ldd = g.np, ldt = g.np;
    const T *Ab = dlo + (int64_t)tm * BM * ldd;
    // B rows are the transposed shadows of the tile's packed columns (-1: zeros)
    const T *zt = (const T *)g.zt;
    int64_t boff[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int32_t cg = scol[l_r + 32 * q];
        boff[q] = cg >= 0 ? (int64_t)cg * ldt + l_c : -1;
    }
    const int nj = SPLIT ? live_col_blocks(scol.lim, wn) : 4;

    f4_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f4_t{0.f, 0.f, 0.f, 0.f};

    uint4 ra[4], rb[4];
    const int nk = (int)((k1 - k0) / BK);
#pragma unroll
    for (int q = 0; q < 4; ++q) ra[q] = *(const uint4 *)(Ab + (int64_t)(l_r + 32 * q) * ldd + k0 + l_c);
#pragma unroll
    for (int q = 0; q < 4; ++q)
        rb[q] = boff[q] >= 0 ? *(const uint4 *)(zt + boff[q] + k0) : uint4{0u, 0u, 0u, 0u};
    lds_put<T, EPC, LDP>(As[0], Bs[0], ra, rb, l_r, l_c);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        const int64_t kn = k0 + (int64_t)(kt + 1 < nk ? kt + 1 : kt) * BK;
#pragma unroll
        for (int q = 0; q < 4; ++q) ra[q] = *(const uint4 *)(Ab + (int64_t)(l_r + 32 * q) * ldd + kn + l_c);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            rb[q] = boff[q] >= 0 ? *(const uint4 *)(zt + boff[q] + kn) : uint4{0u, 0u, 0u, 0u};
#pragma unroll
        for (int kk = 0; kk < BK / C::KSTEP; ++kk) {
            const int koff = kk * C::KSTEP + C::VEC * (lane >> 4);
#pragma unroll
            for (int ib = 0; ib < 4; ++ib)
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
                    if (!SPLIT || jb < nj)
                        acc[ib][jb] = mfma_low<T>(&As[cur][wm * 64 + 16 * ib + (lane & 15)][koff],
                                                  &Bs[cur][wn * 64 + 16 * jb + (lane & 15)][koff], acc[ib][jb]);
        }
        lds_put<T, EPC, LDP>(As[cur ^ 1], Bs[cur ^ 1], ra, rb, l_r, l_c);
        __syncthreads();
    }

    // f32-accumulating 16x16 MFMAs: lane l, register r holds row 4(l/16) + r, column l%16.
    auto row_of = [](int ib, int r, int l) { return 16 * ib + 4 * (l >> 4) + r; };
    if constexpr (SPLIT) {
#pragma unroll
        for (int ib = 0; ib < 4; ++ib)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
                    if (wn * 64 + 16 * jb + (lane & 15) < scol.lim)  // empty packed columns: never read
                        yp[(int64_t)(wm * 64 + row_of(ib, r, lane)) * BN + wn * 64 + 16 * jb + (lane & 15)] =
                            unscale * (double)acc[ib][jb][r];
    } else {
        auto y_of = [&](int ib, int jb, int r, double dji) { return dji + unscale * (double)acc[ib][jb][r]; };
        if (g.dnp) sweep_epilogue<true, true>(g, scol, tm, wm, wn, lane, row_of, y_of, red, sym);
        else sweep_epilogue<true, false>(g, scol, tm, wm, wn, lane, row_of, y_of, red, sym);
    }
}

// ------------------------------------------------ FP32-class rung, 3 x FP16
// The correction product (Delta)(Z - E) of an FP32-class sweep from FP16 matrix-core
// products: with A = s_d Delta and B = s_z (Z - E) scaled by powers of two, each split
// into FP16 hi + lo (lo = the rounding remainder, so hi + lo carries about 22 bits),
// A B ~ Ah Bh + Ah Bl + Al Bh accumulated in FP32 (the dropped Al Bl is 2^-22
// relative).  v_mfma_f32_16x16x32_f16 runs 16 times the FP32 matrix rate, so the three
// products cost less than a fifth of one FP32 product.  BK = 32; each 16-byte chunk
// holds 8 elements, 4 chunks per 64-byte tile row, 256 threads cover 64 rows per pass.
// Chunk c of row r sits at position c ^ ((r >> 2) & 3), so the eight rows that one
// 16-byte fragment read serves per cycle fall on distinct banks without padding.
template <bool SPLIT>
__device__ __forceinline__ void gemm_x3_body(char *smem, double (*red)[BN][NRED], const PackedCols scol,
                                             const GemmArgs &g, double unscale, int tm, int64_t k0, int64_t k1,
                                             double *yp, bool sym) {
    typedef _Float16 Tile[BM][X3_LDP];
    Tile *S = (Tile *)smem;  // stage s: S[4 s + 0..3] = A hi, A lo, B hi, B lo

    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, wm = wv >> 1, wn = wv & 1;
    const int l_r = t >> 2, l_c = (t & 3) * 8;
    const int64_t ldd = g.np, ldt = g.np;
    const _Float16 *Ah = g.dmh + (int64_t)tm * BM * ldd, *Al = g.dml + (int64_t)tm * BM * ldd;
    int64_t boff[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int32_t cg = scol[l_r + 64 * q];
        boff[q] = cg >= 0 ? (int64_t)cg * ldt + l_c : -1;
    }
    const int nj = SPLIT ? live_col_blocks(scol.lim, wn) : 4;

    f4_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f4_t{0.f, 0.f, 0.f, 0.f};

    // Two register stages: the chunks of K step kt + 2 are loaded while step kt is
    // multiplied out of LDS and step kt + 1 waits in the other stage, so a load has two
    // steps of matrix work to arrive in.  st[p][m][q]: stage p, operand m (A hi, A lo,
    // B hi, B lo), row l_r + 64 q; every index is a constant after unrolling.
    // (a native vector type: the register arrays of HIP's uint4 struct were left in scratch)
    typedef unsigned int u4v __attribute__((ext_vector_type(4)));
    u4v st[2][4][2];
    const int nk = (int)((k1 - k0) / X3_BK);
    const int klast = nk > 0 ? nk - 1 : 0;
    auto swz = [](int r, int chunk) { return 8 * (chunk ^ ((r >> 2) & 3)); };
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int64_t k = k0 + (int64_t)(p < klast ? p : klast) * X3_BK;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int64_t ao = (int64_t)(l_r + 64 * q) * ldd + k + l_c;
            st[p][0][q] = *(const u4v *)(Ah + ao);
            st[p][1][q] = *(const u4v *)(Al + ao);
            st[p][2][q] = boff[q] >= 0 ? *(const u4v *)(g.zth + boff[q] + k) : u4v{0u, 0u, 0u, 0u};
            st[p][3][q] = boff[q] >= 0 ? *(const u4v *)(g.ztl + boff[q] + k) : u4v{0u, 0u, 0u, 0u};
        }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q)
            *(u4v *)&S[m][l_r + 64 * q][swz(l_r + 64 * q, l_c >> 3)] = st[0][m][q];
    __syncthreads();
    const int kc = lane >> 4;  // this lane's 16-byte chunk of the K slice
    // K ranges are multiples of 64 (two steps): step kt + p sits in LDS stage p; the
    // stage is a template constant, so every index into st is one
    int kt = 0;
    auto half = [&](auto pc) {
        constexpr int p = decltype(pc)::value;
        {
            // stage p of the registers was stored to LDS: load step kt + p + 2 into it
            const int kn = kt + p + 2;
            const int64_t k = k0 + (int64_t)(kn < klast ? kn : klast) * X3_BK;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int64_t ao = (int64_t)(l_r + 64 * q) * ldd + k + l_c;
                st[p][0][q] = *(const u4v *)(Ah + ao);
                st[p][1][q] = *(const u4v *)(Al + ao);
                st[p][2][q] = boff[q] >= 0 ? *(const u4v *)(g.zth + boff[q] + k) : u4v{0u, 0u, 0u, 0u};
                st[p][3][q] = boff[q] >= 0 ? *(const u4v *)(g.ztl + boff[q] + k) : u4v{0u, 0u, 0u, 0u};
            }
            h8_t ah[4], al[4];
#pragma unroll
            for (int ib = 0; ib < 4; ++ib) {
                const int r = wm * 64 + 16 * ib + (lane & 15);
                ah[ib] = *(const h8_t *)&S[4 * p + 0][r][swz(r, kc)];
                al[ib] = *(const h8_t *)&S[4 * p + 1][r][swz(r, kc)];
            }
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                if (SPLIT && jb >= nj) continue;
                const int r = wn * 64 + 16 * jb + (lane & 15);
                const h8_t bh = *(const h8_t *)&S[4 * p + 2][r][swz(r, kc)];
                const h8_t bl = *(const h8_t *)&S[4 * p + 3][r][swz(r, kc)];
#pragma unroll
                for (int ib = 0; ib < 4; ++ib) {
                    acc[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[ib], bh, acc[ib][jb], 0, 0, 0);
                    acc[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[ib], bl, acc[ib][jb], 0, 0, 0);
                    acc[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[ib], bh, acc[ib][jb], 0, 0, 0);
                }
            }
            // step kt + p + 1 (register stage p ^ 1) to the other LDS stage
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    *(u4v *)&S[4 * (p ^ 1) + m][l_r + 64 * q][swz(l_r + 64 * q, l_c >> 3)] = st[p ^ 1][m][q];
            __syncthreads();
        }
    };
    for (; kt < nk; kt += 2) {
        half(std::integral_constant<int, 0>{});
        half(std::integral_constant<int, 1>{});
    }

    // f32-accumulating 16x16 MFMAs: lane l, register r holds row 4(l/16) + r, column l%16.
    auto row_of = [](int ib, int r, int l) { return 16 * ib + 4 * (l >> 4) + r; };
    if constexpr (SPLIT) {
#pragma unroll
        for (int ib = 0; ib < 4; ++ib)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
                    if (wn * 64 + 16 * jb + (lane & 15) < scol.lim)  // empty packed columns: never read
                        yp[(int64_t)(wm * 64 + row_of(ib, r, lane)) * BN + wn * 64 + 16 * jb + (lane & 15)] =
                            unscale * (double)acc[ib][jb][r];
    } else {
        auto y_of = [&](int ib, int jb, int r, double dji) { return dji + unscale * (double)acc[ib][jb][r]; };
        if (g.dnp) sweep_epilogue<true, true>(g, scol, tm, wm, wn, lane, row_of, y_of, red, sym);
        else sweep_epilogue<true, false>(g, scol, tm, wm, wn, lane, row_of, y_of, red, sym);
    }
}

// The sweep's product over the K range [k0, k1), in the precision the ladder chose;
// SPLIT writes the partial tile instead of running the epilogue.  X3: the three-product
// FP32-class rung, which has a kernel of its own (k_sweep_x3).
template <bool SPLIT, bool X3>
__device__ __forceinline__ void sweep_tile(const Ctrl *ctrl, const GemmArgs &g, char *smem, double (*red)[BN][NRED],
                                           const PackedCols scol, int tm, int64_t k0, int64_t k1, double *yp) {
    const int32_t prec = ctrl->prec;
    const bool sym = ctrl->sym != 0;
    if constexpr (X3) {
        gemm_x3_body<SPLIT>(smem, red, scol, g, 1.0 / (ctrl->dscale * ctrl->zscale), tm, k0, k1, yp, sym);
    } else if (prec == PREC_F64) {
        gemm_f64_body<SPLIT>(smem, red, scol, g, tm, k0, k1, yp, sym);
    } else if (prec == PREC_F32) {
        gemm_low_body<float, SPLIT>(smem, red, scol, g, g.d32, 1.0, tm, k0, k1, yp, sym);
    } else if (prec == PREC_LOW) {
        if (g.low_type == LT_F16)
            gemm_low_body<_Float16, SPLIT>(smem, red, scol, g, (const _Float16 *)g.dlo,
                                           1.0 / (ctrl->dscale * ctrl->zscale), tm, k0, k1, yp, sym);
        else
            gemm_low_body<__bf16, SPLIT>(smem, red, scol, g, (const __bf16 *)g.dlo, 1.0, tm, k0, k1, yp, sym);
    }
}

// One sweep's product.  Sweeps with enough tiles: block -> (row tile, packed column
// tile), whole K range, fused epilogue.  Narrow sweeps: block -> (split s, packed
// column tile, row tile) over a K range, partial tile written for k_sweep_split_epi.
template <bool X3>
__device__ __forceinline__ void sweep_gemm(const Ctrl *ctrl, const GemmArgs &g, int32_t regular_blocks) {
    const int ntm = (int)(g.np / BM), ntn = (int)(g.kp / BN);
    const int32_t kact = ctrl->kact;
    const SplitPlan sp = split_plan(kact, ntm, g.np, g.nblk);
    __shared__ __attribute__((aligned(16))) char smem[SMEM_MAIN];
    // The epilogue's reduction area reuses the operand stages: every wave has passed
    // the K loop's last barrier, after its last operand read, before it is written.
    static_assert(sizeof(double) * 2 * BN * NRED <= SMEM_MAIN, "reduction area exceeds the operand stages");
    double (*red)[BN][NRED] = (double (*)[BN][NRED])smem;
    if (sp.S < 2) {
        if ((int)blockIdx.x >= regular_blocks) return;
        int tm, tn;
        tile_of(blockIdx.x, regular_blocks, ntm, ntn, tm, tn);
        // column tiles run over the packed active columns; tiles past them have no work
        if ((int64_t)tn * BN >= kact) return;
        const PackedCols scol{g.cs.alist + (int64_t)tn * BN, (int32_t)(kact - (int64_t)tn * BN)};
        sweep_tile<false, X3>(ctrl, g, smem, red, scol, tm, 0, g.np, nullptr);
    } else {
        const int64_t per = (int64_t)ntm * sp.nct;
        if ((int64_t)blockIdx.x >= per * sp.S) return;
        const int s = (int)(blockIdx.x / per), rest = (int)(blockIdx.x % per);
        const int tn = rest / ntm, tm = rest % ntm;
        const int64_t nk64 = g.np / 64;
        const int64_t k0 = (int64_t)s * nk64 / sp.S * 64, k1 = (int64_t)(s + 1) * nk64 / sp.S * 64;
        const PackedCols scol{g.cs.alist + (int64_t)tn * BN, (int32_t)(kact - (int64_t)tn * BN)};
        double *yp = g.ypart + (((int64_t)s * sp.nct + tn) * ntm + tm) * (int64_t)(BM * BN);
        sweep_tile<true, X3>(ctrl, g, smem, nullptr, scol, tm, k0, k1, yp);
    }
}

// The sweep's product in FP64, BF16/FP16 or FP32; a three-product FP32-class sweep is
// left to k_sweep_x3, launched beside it (the precision is decided on the device).
__global__ __launch_bounds__(256, 2) void k_sweep_gemm(const Ctrl *ctrl, GemmArgs g, int32_t regular_blocks) {
    if (ctrl->error || ctrl->done) return;
    if (g.mid_x3 && ctrl->prec == PREC_F32) return;
    sweep_gemm<false>(ctrl, g, regular_blocks);
}

// The three-product FP32-class sweep: a kernel of its own so that the K loop is not
// held to the FP64 body's register budget (it keeps two staged loads in flight).
__global__ __launch_bounds__(256, 2) void k_sweep_x3(const Ctrl *ctrl, GemmArgs g, int32_t regular_blocks) {
    if (ctrl->error || ctrl->done || ctrl->prec != PREC_F32) return;
    sweep_gemm<true>(ctrl, g, regular_blocks);
}

// Narrow sweep, epilogue: Y of the tile = the split partials summed in split order.
// The block first sums the partials of the tile's live columns into split slot 0
// (coalesced rows, every split's load in flight at once), then runs the epilogue on
// that sum.  A small grid walks the tiles, so that sweeps with enough tiles pay
// little for it.
__global__ __launch_bounds__(256, 1) void k_sweep_split_epi(const Ctrl *ctrl, GemmArgs g) {
    if (ctrl->error || ctrl->done) return;
    const int ntm = (int)(g.np / BM);
    const int32_t kact = ctrl->kact;
    const SplitPlan sp = split_plan(kact, ntm, g.np, g.nblk);
    if (sp.S < 2) return;
    __shared__ double red[2][BN][NRED];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, wm = wv >> 1, wn = wv & 1;
    const bool low = ctrl->prec != PREC_F64, sym = ctrl->sym != 0;
    const int64_t tile = (int64_t)BM * BN, stride = (int64_t)sp.nct * ntm * tile;
    auto row_of = [](int ib, int r, int l) { return 16 * ib + 4 * r + (l >> 4); };
    for (int64_t bt = blockIdx.x; bt < (int64_t)ntm * sp.nct; bt += gridDim.x) {
        const int tn = (int)(bt / ntm), tm = (int)(bt % ntm);
        const PackedCols scol{g.cs.alist + (int64_t)tn * BN, (int32_t)(kact - (int64_t)tn * BN)};
        double *y0 = g.ypart + ((int64_t)tn * ntm + tm) * tile;
        // (row, live column) pairs spread over all threads, consecutive threads on
        // consecutive columns of a row
        const int live = scol.lim < BN ? scol.lim : BN;
#pragma unroll 2
        for (int p = t; p < BM * live; p += 256) {
            const int r = p / live, cl = p - r * live;
            const int64_t e = (int64_t)r * BN + cl;
            double v[SPLIT_MAX];
#pragma unroll
            for (int q = 0; q < SPLIT_MAX; ++q) v[q] = q < sp.S ? y0[q * stride + e] : 0.0;
            double y = 0.0;
#pragma unroll
            for (int q = 0; q < SPLIT_MAX; ++q)
                if (q < sp.S) y += v[q];
            y0[e] = y;
        }
        __syncthreads();
        auto y_of = [&](int ib, int jb, int r, double dji) {
            const double y = y0[(int64_t)(wm * 64 + row_of(ib, r, lane)) * BN + wn * 64 + 16 * jb + (lane & 15)];
            return low ? dji + y : y;  // low precision: split form, Delta E exact
        };
        if (low) {
            if (g.dnp) sweep_epilogue<true, true>(g, scol, tm, wm, wn, lane, row_of, y_of, red, sym);
            else sweep_epilogue<true, false>(g, scol, tm, wm, wn, lane, row_of, y_of, red, sym);
        } else {
            if (g.dnp) sweep_epilogue<false, true>(g, scol, tm, wm, wn, lane, row_of, y_of, red, sym);
            else sweep_epilogue<false, false>(g, scol, tm, wm, wn, lane, row_of, y_of, red, sym);
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_sweep_gemm(hipStream_t s, const Ctrl *ctrl, const double *delta, int64_t lda, const void *dlo,
                             const float *d32, const void *zt, const double *zin, double *zout, const double *theta,
                             ColState cs, const double *dvec, double *part, int64_t n, int64_t np, int64_t kp,
                             int32_t sweep, int32_t low_type, double *ypart, int nblk, double *dnp, int32_t mid_x3) {
    // three-product rung: the FP16 hi/lo shadows live where the FP32 shadows would
    const _Float16 *dmh = (const _Float16 *)d32, *dml = dmh ? dmh + np * np : nullptr;
    const _Float16 *zth = (const _Float16 *)zt, *ztl = zth ? zth + kp * np : nullptr;
    GemmArgs g{delta, lda, dlo, d32, zt, zin, zout, theta, cs, dvec, part, n, np, kp, low_type, ypart, nblk, dnp,
               dmh, dml, zth, ztl, mid_x3};
    (void)sweep;
    const int blocks = (int)((np / BM) * (kp / BN));
    const SplitBounds b = split_bounds(np, kp, nblk);
    const int64_t grid = b.split_blocks > blocks ? b.split_blocks : blocks;
    k_sweep_gemm<<<(unsigned)grid, 256, 0, s>>>(ctrl, g, blocks);
    if (mid_x3) k_sweep_x3<<<(unsigned)grid, 256, 0, s>>>(ctrl, g, blocks);
    if (b.split_blocks > 0) {
        const int64_t eg = b.epi_blocks < nblk / 2 ? b.epi_blocks : nblk / 2;
        k_sweep_split_epi<<<(unsigned)(eg > 0 ? eg : 1), 256, 0, s>>>(ctrl, g);
    }
    return hipGetLastError();
}

SplitBounds split_bounds(int64_t np, int64_t kp, int nblk) {
    SplitBounds b{0, 0, 0};
    const int ntm = (int)(np / BM);
    for (int64_t nct = 1; nct <= kp / BN; ++nct) {
        const SplitPlan sp = split_plan(nct * BN, ntm, np, nblk);
        if (sp.S < 2) continue;
        const int64_t blocks = (int64_t)ntm * nct * sp.S;
        if (blocks > b.split_blocks) b.split_blocks = blocks;
        if ((int64_t)ntm * nct > b.epi_blocks) b.epi_blocks = (int64_t)ntm * nct;
        if (blocks > b.ypart_tiles) b.ypart_tiles = blocks;
    }
    return b;
}

}  // namespace ipt
