// Small MLP that predicts warm starts Z0 for a parametrised family M(eps) = D + eps R,
// trained and evaluated with the kernels of this file.
//
// Network: x (in) -> [Linear -> tanh] x depth -> Linear -> y (out).  Parameters are
// stored layer by layer as W_l (out_l x in_l, row-major) followed by b_l (out_l), in
// FP32 (the Adam master copy); the GEMMs read BF16 copies.
//
// Every GEMM is C[M x N] = A[M x K] B[N x K]^T on BF16 operands whose reduction
// dimension is contiguous (16-byte loads, no transposed reads), with v_mfma_f32_16x16x32_bf16
// and FP32 accumulation.  The layouts each product needs are written by the producer:
// the forward epilogue stores H and H^T, the loss epilogue g and g^T, the Adam epilogue
// W and W^T, so that
//   forward      H_l = act(H_{l-1} W_l^T + b_l)          A = H_{l-1},  B = W_l
//   input grad   dH_{l-1} = G_l W_l                      A = G_l,      B = W_l^T   (split K)
//   weight grad  dW_l = G_l^T H_{l-1}                    A = G_l^T,    B = H_{l-1}^T
// All dimensions are zero-padded to multiples of 128; padding stays zero.  Reductions
// (split K, column sums, loss) run in a fixed order, so results are bit-reproducible.
#include <math.h>

#include "ipt_internal.h"

namespace ipt {

namespace {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef double d2_t __attribute__((ext_vector_type(2)));

constexpr int GT = MLP_TILE;   // tile rows and columns
constexpr int GK = 32;         // K step
constexpr int WARM_REG_ORDER = 4;  // warm-start series orders held in registers
constexpr int GLD = GK + 8;    // LDS pitch of an operand row in BF16 (80 bytes: 16 rows hit distinct banks)
constexpr int OLD = GT + 8;    // LDS pitch of an output row in BF16 (272 bytes)
constexpr int STAGE = 2 * GT * GLD;             // A and B of one stage
constexpr int SMEM_BF16 = 2 * STAGE;            // two stages (40 KB); the output tile reuses it
static_assert(GT * OLD <= SMEM_BF16, "output tile must fit the operand buffers");

__device__ inline uint16_t bf16_bits(float v) {
    const __bf16 b = (__bf16)v;
    return __builtin_bit_cast(uint16_t, b);
}
__device__ inline float bits_f32(uint16_t u) { return (float)__builtin_bit_cast(__bf16, u); }

// The 128 x 128 BF16 tile in LDS (out[r * OLD + c], values already zero outside the
// valid region) goes to C (row-major) and C^T.  For C^T, lane l of a wave reads column
// l of the tile (consecutive 2-byte LDS words) and writes 8 consecutive rows of it.
__device__ void store_tile(const uint16_t *out, const MlpEpi &e, int m0, int n0) {
    const int t = threadIdx.x;
    if (e.c16) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int u = t + 256 * i, r = u >> 4, ch = u & 15;
            *(u16x8 *)(e.c16 + (int64_t)(m0 + r) * e.ldc16 + n0 + ch * 8) = *(const u16x8 *)(out + r * OLD + ch * 8);
        }
    }
    if (e.ct16) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int u = t + 256 * i, c = u & (GT - 1), ch = u >> 7;
            u16x8 v;
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = out[(ch * 8 + q) * OLD + c];
            *(u16x8 *)(e.ct16 + (int64_t)(n0 + c) * e.ldct16 + m0 + ch * 8) = v;
        }
    }
}

// a / b and a % b for non-negative a, b > 0, in 32 bits when both fit (a 64-bit
// division is several times longer)
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

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Adam (beta 0.9 / 0.999, eps 1e-8) on one weight; returns the new weight.  c1, c2 are
// the bias corrections 1 - beta^step of the step (computed once per thread).
constexpr float ADAM_B1 = 0.9f, ADAM_B2 = 0.999f;
__device__ inline float adam_update(float *w, float *m, float *v, float g, float lr, float c1, float c2) {
    const float b1 = ADAM_B1, b2 = ADAM_B2, eps = 1e-8f;
    const float mv = b1 * *m + (1.f - b1) * g;
    const float vv = b2 * *v + (1.f - b2) * g * g;
    *m = mv;
    *v = vv;
    const float nw = *w - lr * (mv / c1) / (sqrtf(vv / c2) + eps);
    *w = nw;
    return nw;
}

// The loss and Adam epilogues read FP32 data per output (targets; weights and moments):
// their accumulators go through LDS in two halves of 64 rows (FP32, after the BF16
// output tile), and each thread then takes 4 consecutive columns of a row at a time,
// so those reads and the Adam writes are 16-byte accesses along rows, four rows' loads
// in flight before their arithmetic.
constexpr int FLD = GT + 4;                                   // FP32 half-tile pitch (floats)
constexpr int SMEM_STAGED = GT * OLD + 2 * (GT / 2) * FLD;    // BF16 tile + FP32 half (in BF16 units)
template <int MODE>
constexpr int mlp_smem() {
    return (MODE == MLP_EPI_MSE || MODE == MLP_EPI_ADAM || MODE == MLP_EPI_WARM)
               ? (SMEM_STAGED > SMEM_BF16 ? SMEM_STAGED : SMEM_BF16)
               : SMEM_BF16;
}

// The warm-start epilogue (MLP_EPI_WARM) of a 128 x 128 output tile held as the
// four waves' 64 x 64 quarters (acc of wave (wm, wn), cbase = 64 wn + lane % 16): the
// network's output y of member p and entry q = j kcols + c is the standardised remainder
// after the analytic series start, so Z0_jc = sum_{l <= order} eps^l T_l + eps^(order+1)
// (mu + sigma (y + bias)), and 1 at the requested entry of each column.  fh: 64 x FLD
// floats of LDS; every thread of the block calls it (it holds barriers).
__device__ __forceinline__ void warm_epilogue(const f4_t (&acc)[4][4], const MlpEpi &e, float (*fh)[FLD], int m0,
                                              int n0, int t, int lane, int wm, int cbase) {
    // accumulators through LDS (two halves of 64 rows, FP32); each thread then takes 4
    // consecutive outputs q of a member row at a time (consecutive columns c of Z0)
    const int32_t ord = e.order;
    const int cq = t & 31, rp = t >> 5;
    // When kcols is a multiple of 4 (so is nvalid = n kcols), the four outputs of a
    // thread are four consecutive columns of one row of Z0, all in range or all out;
    // with even strides and a 16-byte aligned Z0 they leave as two 16-byte stores, and
    // the series terms T_l (they do not depend on the member) sit in registers.  The
    // arithmetic is the same in both forms.
    const bool vec = (e.kcols & 3) == 0 && (e.ldz0 & 1) == 0 && (e.pstride & 1) == 0 &&
                     ((uintptr_t)e.z0 & 15) == 0 && ord <= WARM_REG_ORDER;
    int64_t jj[4], cc[4];
    bool qok[4], unit[4];
    double bv[4], mu[4], sg[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int q = n0 + 4 * cq + u;
        qok[u] = q < e.nvalid;
        const int qq = qok[u] ? q : 0;
        divmod_nn(qq, e.kcols, jj[u], cc[u]);
        unit[u] = jj[u] == e.idx[cc[u]];
        bv[u] = e.bias ? (double)e.bias[qq] : 0.0;
        mu[u] = e.mu[qq];
        sg[u] = e.sigma[qq];
    }
    double tr[WARM_REG_ORDER][4];
#pragma unroll
    for (int l = 0; l < WARM_REG_ORDER; ++l)
#pragma unroll
        for (int u = 0; u < 4; ++u)
            tr[l][u] = (vec && l < ord && qok[u]) ? e.terms[(int64_t)l * e.nvalid + n0 + 4 * cq + u] : 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (wm == h) {
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y)
#pragma unroll
                    for (int r = 0; r < 4; ++r) fh[4 * (lane >> 4) + 16 * x + r][cbase + 16 * y] = acc[x][y][r];
        }
        __syncthreads();
        if (vec) {
            if (qok[0]) {
                double epr[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int p = m0 + h * 64 + rp + 8 * i;
                    epr[i] = p < e.mvalid ? e.eps[p] : 0.0;
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int lrow = rp + 8 * i, p = m0 + h * 64 + lrow;
                    if (p >= e.mvalid) continue;
                    const double ep = epr[i];
                    const f4_t a4 = *(const f4_t *)&fh[lrow][4 * cq];
                    d2_t v[2];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        double vu = 1.0;
                        if (!unit[u]) {
                            double base = 0.0, pw = 1.0;
#pragma unroll
                            for (int l = 0; l < WARM_REG_ORDER; ++l)
                                if (l < ord) {
                                    pw *= ep;
                                    base += pw * tr[l][u];
                                }
                            vu = base + pw * ep * (mu[u] + sg[u] * ((double)a4[u] + bv[u]));
                        }
                        v[u >> 1][u & 1] = vu;
                    }
                    d2_t *dst = (d2_t *)(e.z0 + (int64_t)p * e.pstride + jj[0] * e.ldz0 + cc[0]);
                    dst[0] = v[0];
                    dst[1] = v[1];
                }
            }
        } else {
#pragma unroll 2
            for (int i = 0; i < 8; ++i) {
                const int lrow = rp + 8 * i, p = m0 + h * 64 + lrow;
                if (p >= e.mvalid) continue;
                const double ep = e.eps[p];
                const f4_t a4 = *(const f4_t *)&fh[lrow][4 * cq];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (!qok[u]) continue;
                    const int q = n0 + 4 * cq + u;
                    double v = 1.0;
                    if (!unit[u]) {
                        double base = 0.0, pw = 1.0;
                        for (int l = 1; l <= ord; ++l) {
                            pw *= ep;
                            base += pw * e.terms[(int64_t)(l - 1) * e.nvalid + q];
                        }
                        v = base + pw * ep * (mu[u] + sg[u] * ((double)a4[u] + bv[u]));
                    }
                    e.z0[(int64_t)p * e.pstride + jj[u] * e.ldz0 + cc[u]] = v;
                }
            }
        }
        __syncthreads();
    }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_mlp_gemm(const __bf16 *__restrict__ A, int64_t lda,
                                                  const __bf16 *__restrict__ B, int64_t ldb, int Kc, int M, int N,
                                                  MlpEpi e) {
    __shared__ __attribute__((aligned(16))) uint16_t smem[mlp_smem<MODE>()];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, wm = wv >> 1, wn = wv & 1;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int64_t kbeg = (int64_t)blockIdx.z * Kc;
    const __bf16 *Ab = A + (int64_t)m0 * lda + kbeg;
    const __bf16 *Bb = B + (int64_t)n0 * ldb + kbeg;
    // loader: 16-byte chunk u = t + 256 r of a 128 x 32 tile: row u / 4, k offset 8 (u % 4)
    const int lr0 = t >> 2, lk = (t & 3) * 8;
    u16x8 ra[2], rb[2];
    f4_t acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = f4_t{0.f, 0.f, 0.f, 0.f};
    const int nk = Kc / GK;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        ra[r] = *(const u16x8 *)(Ab + (int64_t)(lr0 + 64 * r) * lda + lk);
        rb[r] = *(const u16x8 *)(Bb + (int64_t)(lr0 + 64 * r) * ldb + lk);
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        *(u16x8 *)(smem + (lr0 + 64 * r) * GLD + lk) = ra[r];
        *(u16x8 *)(smem + GT * GLD + (lr0 + 64 * r) * GLD + lk) = rb[r];
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) {
            const int64_t ko = (int64_t)(kt + 1) * GK + lk;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                ra[r] = *(const u16x8 *)(Ab + (int64_t)(lr0 + 64 * r) * lda + ko);
                rb[r] = *(const u16x8 *)(Bb + (int64_t)(lr0 + 64 * r) * ldb + ko);
            }
        }
        const uint16_t *as = smem + (kt & 1) * STAGE, *bs = as + GT * GLD;
        bf8_t af[4], bfg[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) af[x] = *(const bf8_t *)(as + (wm * 64 + 16 * x + (lane & 15)) * GLD + 8 * (lane >> 4));
#pragma unroll
        for (int y = 0; y < 4; ++y) bfg[y] = *(const bf8_t *)(bs + (wn * 64 + 16 * y + (lane & 15)) * GLD + 8 * (lane >> 4));
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[x], bfg[y], acc[x][y], 0, 0, 0);
        if (kt + 1 < nk) {
            uint16_t *ns = smem + ((kt + 1) & 1) * STAGE;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                *(u16x8 *)(ns + (lr0 + 64 * r) * GLD + lk) = ra[r];
                *(u16x8 *)(ns + GT * GLD + (lr0 + 64 * r) * GLD + lk) = rb[r];
            }
        }
        __syncthreads();
    }

    // lane l, register r of block (x, y): row 16 x + 4 (l / 16) + r, column 16 y + l % 16
    // of the wave's 64 x 64 quarter
    const int rbase = wm * 64 + 4 * (lane >> 4), cbase = wn * 64 + (lane & 15);
    if (MODE == MLP_EPI_SPLIT) {
        float *p = e.c32 + (int64_t)blockIdx.z * M * N;
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    p[(int64_t)(m0 + rbase + 16 * x + r) * N + n0 + cbase + 16 * y] = acc[x][y][r];
        return;
    }
    if (MODE == MLP_EPI_F32 || MODE == MLP_EPI_GRAD) {
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                const int gc = n0 + cbase + 16 * y;
                if (gc >= e.nvalid) continue;
                const float bv = (MODE == MLP_EPI_F32 && e.bias) ? e.bias[gc] : 0.f;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gr = m0 + rbase + 16 * x + r;
                    if (gr < e.mvalid) e.c32[(int64_t)gr * e.ldc32 + gc] = acc[x][y][r] + bv;
                }
            }
        return;
    }
    if (MODE == MLP_EPI_WARM) {
        warm_epilogue(acc, e, (float(*)[FLD])(smem + GT * OLD), m0, n0, t, lane, wm, cbase);
        return;
    }

    // the BF16-output epilogues: values into the LDS tile, then store_tile
    uint16_t *out = smem;  // the last K step ended with a barrier
    float lsum = 0.f;
    float c1 = 1.f, c2 = 1.f;
    if (MODE == MLP_EPI_ADAM) {
        const float step = (float)(*e.adam_t + 1);
        c1 = 1.f - powf(ADAM_B1, step);
        c2 = 1.f - powf(ADAM_B2, step);
    }
    if constexpr (MODE == MLP_EPI_MSE || MODE == MLP_EPI_ADAM) {
        float(*fh)[FLD] = (float(*)[FLD])(smem + GT * OLD);
        const int cq = t & 31, rp = t >> 5;  // columns 4 cq .. 4 cq + 3, rows rp, rp + 8, ...
        const int lc0 = 4 * cq, gc0 = n0 + lc0;
        // the 4 columns: all valid (16-byte path) or checked one by one
        const bool vec = gc0 + 4 <= e.nvalid &&
                         (MODE == MLP_EPI_MSE ? (e.ldt & 3) == 0 && ((uintptr_t)e.tgt & 15) == 0
                                              : (e.nvalid & 3) == 0 &&
                                                    (((uintptr_t)e.w | (uintptr_t)e.am | (uintptr_t)e.av) & 15) == 0);
        float bv[4] = {0.f, 0.f, 0.f, 0.f};
        if (MODE == MLP_EPI_MSE && e.bias)
#pragma unroll
            for (int q = 0; q < 4; ++q) bv[q] = gc0 + q < e.nvalid ? e.bias[gc0 + q] : 0.f;
        float csv[4] = {0.f, 0.f, 0.f, 0.f};  // column sums of the stored values over this thread's rows
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (wm == h) {
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y)
#pragma unroll
                        for (int r = 0; r < 4; ++r) fh[4 * (lane >> 4) + 16 * x + r][cbase + 16 * y] = acc[x][y][r];
            }
            __syncthreads();
#pragma unroll
            for (int i0 = 0; i0 < 8; i0 += 4) {
                f4_t ld0[4], ld1[4], ld2[4];  // targets, or weights / moments
                float rw[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int lrow = h * 64 + rp + 8 * (i0 + i), gr = m0 + lrow;
                    const bool rok = gr < e.mvalid;
                    rw[i] = 1.f;
                    if (MODE == MLP_EPI_MSE) {
                        if (rok && e.roww) rw[i] = e.roww[gr];
                        const float *tp = e.tgt + (int64_t)(rok ? gr : 0) * e.ldt + gc0;
                        if (vec) {
                            ld0[i] = *(const f4_t *)tp;
                        } else {
#pragma unroll
                            for (int q = 0; q < 4; ++q) ld0[i][q] = gc0 + q < e.nvalid ? tp[q] : 0.f;
                        }
                    } else {
                        const int64_t wi = (int64_t)(rok ? gr : 0) * e.nvalid + gc0;
                        if (vec) {
                            ld0[i] = *(const f4_t *)(e.w + wi);
                            ld1[i] = *(const f4_t *)(e.am + wi);
                            ld2[i] = *(const f4_t *)(e.av + wi);
                        } else {
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                const bool ok = gc0 + q < e.nvalid;
                                ld0[i][q] = ok ? e.w[wi + q] : 0.f;
                                ld1[i][q] = ok ? e.am[wi + q] : 0.f;
                                ld2[i][q] = ok ? e.av[wi + q] : 0.f;
                            }
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int lrow = h * 64 + rp + 8 * (i0 + i), gr = m0 + lrow;
                    const bool rok = gr < e.mvalid;
                    const f4_t a4 = *(const f4_t *)&fh[lrow - h * 64][lc0];
                    f4_t nw = f4_t{0.f, 0.f, 0.f, 0.f}, nm = nw, nv = nw;
                    uint16_t b[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const bool ok = rok && gc0 + q < e.nvalid;
                        float v = a4[q] + bv[q];
                        if (MODE == MLP_EPI_MSE) {
                            const float ws = (ok && e.roww) ? rw[i] : 1.f;
                            const float d = ok ? (v - ld0[i][q]) * ws : 0.f;
                            lsum += d * d;
                            v = (e.scale * ws) * d;
                        } else if (ok) {
                            float w = ld0[i][q], m = ld1[i][q], vv = ld2[i][q];
                            v = adam_update(&w, &m, &vv, v, e.lr, c1, c2);
                            nw[q] = w;
                            nm[q] = m;
                            nv[q] = vv;
                        }
                        b[q] = ok ? bf16_bits(v) : (uint16_t)0;
                        csv[q] += bits_f32(b[q]);
                    }
                    if (MODE == MLP_EPI_ADAM && rok) {
                        const int64_t wi = (int64_t)gr * e.nvalid + gc0;
                        if (vec) {
                            *(f4_t *)(e.w + wi) = nw;
                            *(f4_t *)(e.am + wi) = nm;
                            *(f4_t *)(e.av + wi) = nv;
                        } else {
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                if (gc0 + q < e.nvalid) {
                                    e.w[wi + q] = nw[q];
                                    e.am[wi + q] = nm[q];
                                    e.av[wi + q] = nv[q];
                                }
                        }
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) out[lrow * OLD + lc0 + q] = b[q];
                }
            }
            __syncthreads();
        }
        if (e.colp) {
            // the 8 row phases in order, through LDS (the FP32 half is free again)
            float(*cred)[GT] = (float(*)[GT])(smem + GT * OLD);
#pragma unroll
            for (int q = 0; q < 4; ++q) cred[rp][lc0 + q] = csv[q];
            __syncthreads();
            if (t < GT) {
                float v = cred[0][t];
#pragma unroll
                for (int g = 1; g < 8; ++g) v += cred[g][t];
                e.colp[(int64_t)(m0 / GT) * e.ldcolp + n0 + t] = v;
            }
        }
        if (MODE == MLP_EPI_MSE) {
            __shared__ double red[4];
            const double ws = wave_sum_d((double)lsum);
            if (lane == 0) red[wv] = ws;
            __syncthreads();
            if (t == 0) e.lossp[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
        }
        __syncthreads();
        store_tile(out, e, m0, n0);
        return;
    }
    float csum[4] = {0.f, 0.f, 0.f, 0.f};  // column sums of the stored values over this lane's rows
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int lc = cbase + 16 * y, gc = n0 + lc;
            const bool cok = gc < e.nvalid;
            const float bv = (e.bias && cok && MODE != MLP_EPI_ADAM) ? e.bias[gc] : 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int lrow = rbase + 16 * x + r, gr = m0 + lrow;
                const bool ok = cok && gr < e.mvalid;
                float v = acc[x][y][r] + bv;
                if (MODE == MLP_EPI_ACT) {
                    if (e.tanh_act) v = tanhf(v);
                } else if (MODE == MLP_EPI_MSE) {
                    const float ws = (ok && e.roww) ? e.roww[gr] : 1.f;
                    const float d = ok ? (v - e.tgt[(int64_t)gr * e.ldt + gc]) * ws : 0.f;
                    lsum += d * d;
                    v = (e.scale * ws) * d;
                } else if (MODE == MLP_EPI_ADAM) {
                    if (ok) {
                        const int64_t wi = (int64_t)gr * e.nvalid + gc;
                        v = adam_update(e.w + wi, e.am + wi, e.av + wi, v, e.lr, c1, c2);
                    }
                }
                const uint16_t b = ok ? bf16_bits(v) : (uint16_t)0;
                out[lrow * OLD + lc] = b;
                csum[y] += bits_f32(b);
            }
        }
    if (e.colp) {
        // the 4 row groups of the wave (lane / 16), then the two waves sharing columns
        __shared__ float cred[2][GT];
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            float v = csum[y];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (lane < 16) cred[wm][cbase + 16 * y] = v;
        }
        __syncthreads();
        if (t < GT) e.colp[(int64_t)(m0 / GT) * e.ldcolp + n0 + t] = cred[0][t] + cred[1][t];
    }
    if (MODE == MLP_EPI_MSE) {
        __shared__ double red[4];
        const double ws = wave_sum_d((double)lsum);
        if (lane == 0) red[wv] = ws;
        __syncthreads();
        if (t == 0) e.lossp[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
    }
    __syncthreads();
    store_tile(out, e, m0, n0);
}

// Split-K sum in split order over a slab of MLP_SLAB rows x 128 columns per block
// (thread t sums column t % 128 of 4 rows, its loads for 8 splits at a time in
// flight), then the layer's epilogue: the tanh derivative (1 - h^2) of the stored
// activation (MLP_EPI_SPLIT: hidden gradients), bias and tanh (MLP_EPI_ACT), or Adam on
// the weights (MLP_EPI_ADAM); BF16 C row by row, then C^T (8 consecutive rows of a
// column per 16-byte store) and the slab's column sums through LDS.
template <int MODE>
__global__ __launch_bounds__(256) void k_split_reduce(const float *part, int splits, int M, int N, MlpEpi e) {
    __shared__ uint16_t slab[MLP_SLAB][GT];
    const int t = threadIdx.x, c = t & (GT - 1), rq = (t >> 7) * 4;
    const int m0 = blockIdx.y * MLP_SLAB, n0 = blockIdx.x * GT, gc = n0 + c;
    const int64_t mn = (int64_t)M * N;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    const float *p = part + (int64_t)(m0 + rq) * N + gc;
    int z = 0;
    for (; z + 8 <= splits; z += 8) {
        float v[8][4];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) v[u][r] = p[(z + u) * mn + (int64_t)r * N];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] += v[u][r];
    }
    for (; z < splits; ++z)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] += p[z * mn + (int64_t)r * N];
    float c1 = 1.f, c2 = 1.f;
    if (MODE == MLP_EPI_ADAM) {
        const float step = (float)(*e.adam_t + 1);
        c1 = 1.f - powf(ADAM_B1, step);
        c2 = 1.f - powf(ADAM_B2, step);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gr = m0 + rq + r;
        const bool ok = gr < e.mvalid && gc < e.nvalid;
        float v = acc[r];
        if (MODE == MLP_EPI_SPLIT) {
            const float hv = (float)e.h[(int64_t)gr * e.ldh + gc];
            v *= 1.f - hv * hv;
        } else if (MODE == MLP_EPI_ACT) {
            if (ok) v = tanhf(v + e.bias[gc]);
        } else if (MODE == MLP_EPI_ADAM) {
            if (ok) {
                const int64_t wi = (int64_t)gr * e.nvalid + gc;
                v = adam_update(e.w + wi, e.am + wi, e.av + wi, v, e.lr, c1, c2);
            }
        }
        const uint16_t b = ok ? bf16_bits(v) : (uint16_t)0;
        slab[rq + r][c] = b;
        *(uint16_t *)(e.c16 + (int64_t)gr * e.ldc16 + gc) = b;
    }
    __syncthreads();
    if (t < GT) {
        u16x8 v;
        float cs = 0.f;
#pragma unroll
        for (int q = 0; q < MLP_SLAB; ++q) {
            v[q] = slab[q][t];
            cs += bits_f32(v[q]);
        }
        if (e.ct16) *(u16x8 *)(e.ct16 + (int64_t)(n0 + t) * e.ldct16 + m0) = v;
        if (e.colp) e.colp[(int64_t)(m0 / MLP_SLAB) * e.ldcolp + n0 + t] = cs;
    }
}

// Every hidden layer of a narrow network (padded widths <= MLP_FUSED_W) in one launch:
// a block owns 16 rows of the batch and keeps their activations in LDS from layer to
// layer.  Layer l: H_l = tanh(H_{l-1} W_l^T + b_l); wave w computes columns 64 w ..
// 64 w + 63 of the 16 rows with v_mfma_f32_16x16x32_bf16 over the whole K (A from LDS,
// B = rows of W_l straight from global memory), FP32 accumulation, then
// bias, tanh and the BF16 rounding of the split-K path; H_l goes to LDS for the next
// layer and to H_l (row-major) and H_l^T in global memory for the backward products.
// Rows past the batch and columns past the layer's width are zero, as in the GEMM path.
constexpr int MLP_FUSED_W = 256;
constexpr int FP_LD = MLP_FUSED_W + 8;  // LDS pitch of an activation row (BF16): 528 bytes
// The hidden layers of the 16 batch rows m0.. (hs: two LDS activation buffers).  The
// input is the packed BF16 f.xb, or with x non-null the BF16 of x [batch x in] with the
// packer's zero padding; H_l^T is stored only with store_t.
__device__ __forceinline__ void hidden_slab(const MlpFused &f, const float *x, int in, int batch, int bp, int m0,
                                            uint16_t (*hs)[16][FP_LD], bool store_t) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    // every B fragment of a layer and its bias are loaded before the layer's first
    // product, so a layer waits for one round of loads, not one per K step; the next
    // layer's round is issued as soon as the products have consumed this one, and its
    // latency hides behind this layer's tanh and stores
    constexpr int KS = MLP_FUSED_W / 32;
    bf8_t bq[KS][4];
    float bb[4];
    auto load_layer = [&](int l) {
        const int K = f.linp[l];
        if (wv * 64 >= f.loutp[l]) return;  // the wave's 64 columns hold no data
        const uint16_t *W = (const uint16_t *)f.w[l];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
            if (32 * ks < K)
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
                    bq[ks][jb] = *(const bf8_t *)(W + (int64_t)(wv * 64 + 16 * jb + (lane & 15)) * K + 32 * ks +
                                                  8 * (lane >> 4));
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
            const int n = wv * 64 + 16 * jb + (lane & 15);
            bb[jb] = n < f.lout[l] ? f.bias[l][n] : 0.f;
        }
    };
    load_layer(0);
    if (!x) {
        // the packed BF16 input rows (zero-padded to ip by the packer)
        for (int e = t; e < 16 * (f.ip / 8); e += 256) {
            const int r = e / (f.ip / 8), c8 = (e % (f.ip / 8)) * 8;
            *(u16x8 *)&hs[0][r][c8] = *(const u16x8 *)((const uint16_t *)f.xb + (int64_t)(m0 + r) * f.ip + c8);
        }
    } else {
        // as the packer: BF16 of x, zero past the batch and the input width (zeros first,
        // then one load per thread and pass, so that a thread's loads do not queue)
        for (int e = t; e < 16 * (f.ip / 8); e += 256) {
            const int r = e / (f.ip / 8), c8 = (e % (f.ip / 8)) * 8;
            *(u16x8 *)&hs[0][r][c8] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
        }
        __syncthreads();
        for (int e = t; e < 16 * in; e += 256) {
            const int r = e / in, i = e - r * in;
            if (m0 + r < batch) hs[0][r][i] = bf16_bits(x[(int64_t)(m0 + r) * in + i]);
        }
    }
    __syncthreads();
    for (int l = 0; l < f.depth; ++l) {
        const int cur = l & 1, K = f.linp[l], N = f.loutp[l];
        const bool live = wv * 64 < N;  // the wave's 64 columns hold data
        f4_t acc[4];
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) acc[jb] = f4_t{0.f, 0.f, 0.f, 0.f};
        if (live) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                if (32 * ks < K) {
                    const bf8_t a = *(const bf8_t *)&hs[cur][lane & 15][32 * ks + 8 * (lane >> 4)];
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb)
                        acc[jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bq[ks][jb], acc[jb], 0, 0, 0);
                }
#pragma unroll
            for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[jb][r] += bb[jb];
        }
        if (l + 1 < f.depth) load_layer(l + 1);
        // lane l, register r of block jb: row 4 (l / 16) + r, column 64 w + 16 jb + l % 16
        if (live) {
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                const int n = wv * 64 + 16 * jb + (lane & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 4 * (lane >> 4) + r;
                    const bool ok = m0 + row < batch && n < f.lout[l];
                    const uint16_t b = ok ? bf16_bits(tanhf(acc[jb][r])) : (uint16_t)0;
                    hs[cur ^ 1][row][n] = b;
                    *((uint16_t *)f.hb[l] + (int64_t)(m0 + row) * f.hp + n) = b;
                }
            }
        }
        __syncthreads();
        // H_l^T: column n holds the block's 16 rows contiguously (two 16-byte stores)
        for (int e = t; store_t && e < 2 * N; e += 256) {
            const int n = e >> 1, h8 = (e & 1) * 8;
            u16x8 v;
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = hs[cur ^ 1][h8 + q][n];
            *(u16x8 *)((uint16_t *)f.ht[l] + (int64_t)n * bp + m0 + h8) = v;
        }
    }
}

__global__ __launch_bounds__(256) void k_mlp_hidden_fused(MlpFused f, const float *x, int in, int batch, int bp,
                                                          int store_t) {
    __shared__ __attribute__((aligned(16))) uint16_t hs[2][16][FP_LD];
    hidden_slab(f, x, in, batch, bp, blockIdx.x * 16, hs, store_t != 0);
}

__global__ void k_pack_weights(const float *w, int lout, int lin, __bf16 *wb, __bf16 *wbt, int loutp, int linp) {
    const int64_t total = (int64_t)loutp * linp;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < total; u += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(u / linp), c = (int)(u - (int64_t)r * linp);
        const float v = (r < lout && c < lin) ? w[(int64_t)r * lin + c] : 0.f;
        wb[u] = (__bf16)v;
        wbt[(int64_t)c * loutp + r] = (__bf16)v;
    }
}

__global__ void k_pack_x(const float *x, int batch, int in, __bf16 *xb, __bf16 *xt, int bp, int ip) {
    const int64_t total = (int64_t)bp * ip;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < total; u += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(u / ip), i = (int)(u - (int64_t)b * ip);
        const float v = (b < batch && i < in) ? x[(int64_t)b * in + i] : 0.f;
        xb[u] = (__bf16)v;
        xt[(int64_t)i * bp + b] = (__bf16)v;
    }
}

__global__ void k_bias_step(MlpBiasLayers L, int adam, float *w, float *g, float *am, float *av,
                            const int32_t *adam_t, float lr) {
    int64_t total = 0;
    for (int l = 0; l < L.count; ++l) total += L.lout[l];
    float c1 = 1.f, c2 = 1.f;
    if (adam) {
        const float step = (float)(*adam_t + 1);
        c1 = 1.f - powf(ADAM_B1, step);
        c2 = 1.f - powf(ADAM_B2, step);
    }
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < total; u += (int64_t)gridDim.x * blockDim.x) {
        int l = 0;
        int64_t o = u;
        while (o >= L.lout[l]) {
            o -= L.lout[l];
            ++l;
        }
        float db = 0.f;
        const float *cp = L.colp[l] + o;
        const int64_t ld = L.ldcolp[l];
        int mt = 0;
        for (; mt + 8 <= L.mtiles[l]; mt += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = cp[(int64_t)(mt + u) * ld];
#pragma unroll
            for (int u = 0; u < 8; ++u) db += v[u];
        }
        for (; mt < L.mtiles[l]; ++mt) db += cp[(int64_t)mt * ld];
        const int64_t wi = L.boff[l] + o;
        if (adam)
            adam_update(w + wi, am + wi, av + wi, db, lr, c1, c2);
        else
            g[wi] = db;
    }
}

__global__ void k_loss_step(const double *lossp, int nparts, double inv_count, float *loss, int32_t *adam_t,
                            int adam) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nparts; b += 256) acc += lossp[b];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *loss = (float)(sh[0] * inv_count);
        if (adam) *adam_t += 1;
    }
}

// Targets for problem p and output q = j k + c: the remainder of Z_p after the base
// E + sum_{l <= order} eps_p^l T_l, divided by eps_p^(order + 1), standardised over the
// batch (mean and deviation summed in problem order).
__global__ void k_targets(const double *z, int32_t batch, int64_t n, int64_t k, int64_t ldz, int64_t pstride,
                          const int32_t *idx, const double *eps, int32_t order, const double *terms,
                          const double *weights, float *targets, float *mu, float *sigma) {
    const int64_t nk = n * k;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nk; q += (int64_t)gridDim.x * blockDim.x) {
        int64_t j, c;
        divmod_nn(q, k, j, c);
        const double e0 = (j == idx[c]) ? 1.0 : 0.0;
        auto rem = [&](int32_t p) {
            const double ep = eps[p];
            double base = e0, pw = 1.0;
            for (int l = 1; l <= order; ++l) {
                pw *= ep;
                base += pw * terms[(int64_t)(l - 1) * nk + q];
            }
            return (z[p * pstride + j * ldz + c] - base) / (pw * ep);
        };
        // weighted by weights[p]^2 (uniform when weights is NULL)
        double s = 0.0, sw = 0.0;
        for (int32_t p = 0; p < batch; ++p) {
            const double w2 = weights ? weights[p] * weights[p] : 1.0;
            s += w2 * rem(p);
            sw += w2;
        }
        const double mean = s / sw;
        double v = 0.0;
        for (int32_t p = 0; p < batch; ++p) {
            const double w2 = weights ? weights[p] * weights[p] : 1.0;
            const double r = rem(p) - mean;
            v += w2 * (r * r);
        }
        double sd = sqrt(v / sw);
        if (!(sd >= 1e-300)) sd = 1.0;
        mu[q] = (float)mean;
        sigma[q] = (float)sd;
        for (int32_t p = 0; p < batch; ++p) targets[(int64_t)p * nk + q] = (float)((rem(p) - mean) / sd);
    }
}

inline int capped(int64_t count) {
    int64_t b = (count + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace

// ------------------------------------------------------------------ host side
hipError_t mlp_gemm(hipStream_t s, int mode, const __bf16 *A, int64_t lda, const __bf16 *B, int64_t ldb, int M, int N,
                    int K, int splits, const MlpEpi &e) {
    if (M % GT || N % GT || splits < 1 || K % (GK * splits)) return hipErrorInvalidValue;
    if (mode != MLP_EPI_SPLIT && splits != 1) return hipErrorInvalidValue;
    const dim3 g(N / GT, M / GT, splits);
    const int Kc = K / splits;
    switch (mode) {
        case MLP_EPI_ACT: k_mlp_gemm<MLP_EPI_ACT><<<g, 256, 0, s>>>(A, lda, B, ldb, Kc, M, N, e); break;
        case MLP_EPI_MSE: k_mlp_gemm<MLP_EPI_MSE><<<g, 256, 0, s>>>(A, lda, B, ldb, Kc, M, N, e); break;
        case MLP_EPI_F32: k_mlp_gemm<MLP_EPI_F32><<<g, 256, 0, s>>>(A, lda, B, ldb, Kc, M, N, e); break;
        case MLP_EPI_GRAD: k_mlp_gemm<MLP_EPI_GRAD><<<g, 256, 0, s>>>(A, lda, B, ldb, Kc, M, N, e); break;
        case MLP_EPI_ADAM: k_mlp_gemm<MLP_EPI_ADAM><<<g, 256, 0, s>>>(A, lda, B, ldb, Kc, M, N, e); break;
        case MLP_EPI_SPLIT: k_mlp_gemm<MLP_EPI_SPLIT><<<g, 256, 0, s>>>(A, lda, B, ldb, Kc, M, N, e); break;
        case MLP_EPI_WARM: k_mlp_gemm<MLP_EPI_WARM><<<g, 256, 0, s>>>(A, lda, B, ldb, Kc, M, N, e); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool mlp_fused_fits(int depth, const int *linp, const int *loutp) {
    if (depth < 1 || depth > MLP_MAX_LAYERS) return false;
    for (int l = 0; l < depth; ++l)
        if (linp[l] > MLP_FUSED_W || loutp[l] > MLP_FUSED_W || linp[l] % 32) return false;
    return true;
}

hipError_t mlp_hidden_fused(hipStream_t s, const MlpFused &f, int batch, int bp, const float *x, int in) {
    if (bp % 16 || !mlp_fused_fits(f.depth, f.linp, f.loutp) || (x && (in < 1 || in > f.linp[0])))
        return hipErrorInvalidValue;
    k_mlp_hidden_fused<<<(unsigned)(bp / 16), 256, 0, s>>>(f, x, in, batch, bp, x ? 0 : 1);
    return hipGetLastError();
}

int mlp_split_count(int M, int N, int K) {
    // enough blocks for the chip (about 256) without splitting K below two K steps
    const int tiles = (M / GT) * (N / GT);
    int want = tiles >= 256 ? 1 : 256 / tiles;
    int best = 1;
    for (int sp = 1; sp <= want; ++sp)
        if (K % (GK * sp) == 0 && K / sp >= 2 * GK) best = sp;
    return best;
}

hipError_t mlp_split_reduce(hipStream_t s, int mode, const float *part, int splits, int M, int N, const MlpEpi &e) {
    if (M % GT || N % GT || !e.c16) return hipErrorInvalidValue;
    const dim3 g(N / GT, M / MLP_SLAB);
    switch (mode) {
        case MLP_EPI_SPLIT: k_split_reduce<MLP_EPI_SPLIT><<<g, 256, 0, s>>>(part, splits, M, N, e); break;
        case MLP_EPI_ACT: k_split_reduce<MLP_EPI_ACT><<<g, 256, 0, s>>>(part, splits, M, N, e); break;
        case MLP_EPI_ADAM: k_split_reduce<MLP_EPI_ADAM><<<g, 256, 0, s>>>(part, splits, M, N, e); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t mlp_pack_weights(hipStream_t s, const float *w, int lout, int lin, __bf16 *wb, __bf16 *wbt, int loutp,
                            int linp) {
    k_pack_weights<<<capped((int64_t)loutp * linp), 256, 0, s>>>(w, lout, lin, wb, wbt, loutp, linp);
    return hipGetLastError();
}

hipError_t mlp_pack_x(hipStream_t s, const float *x, int batch, int in, __bf16 *xb, __bf16 *xt, int bp, int ip) {
    k_pack_x<<<capped((int64_t)bp * ip), 256, 0, s>>>(x, batch, in, xb, xt, bp, ip);
    return hipGetLastError();
}

hipError_t mlp_bias_step(hipStream_t s, const MlpBiasLayers &L, int adam, float *w, float *g, float *am, float *av,
                         const int32_t *adam_t, float lr) {
    int64_t total = 0;
    for (int l = 0; l < L.count; ++l) total += L.lout[l];
    k_bias_step<<<capped(total), 256, 0, s>>>(L, adam, w, g, am, av, adam_t, lr);
    return hipGetLastError();
}

hipError_t mlp_loss_step(hipStream_t s, const double *lossp, int nparts, double inv_count, float *loss,
                         int32_t *adam_t, int adam) {
    k_loss_step<<<1, 256, 0, s>>>(lossp, nparts, inv_count, loss, adam_t, adam);
    return hipGetLastError();
}

hipError_t mlp_targets(hipStream_t s, const double *z, int32_t batch, int64_t n, int64_t k, int64_t ldz,
                       int64_t pstride, const int32_t *idx, const double *eps, int32_t order, const double *terms,
                       const double *weights, float *targets, float *mu, float *sigma) {
    k_targets<<<capped(n * k), 256, 0, s>>>(z, batch, n, k, ldz, pstride, idx, eps, order, terms, weights, targets, mu,
                                            sigma);
    return hipGetLastError();
}

}  // namespace ipt
