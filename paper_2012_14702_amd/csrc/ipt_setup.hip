// Setup, first-sweep, diagonal, finalize, control and copy-out kernels of the IPT
// sweep (everything except the products Delta x Z).
//
// Notation: theta = diag(D), i = idx[c] the index column c continues, Z is the
// current iterate (row-major, buffer leading dimension ldzb, padded to np rows and
// kp columns with zeros), W = F(Z) its image under the map of eq. dyn.
#include <math.h>

#include <type_traits>

#include "ipt_internal.h"

namespace ipt {

namespace {


__device__ inline uint64_t dbits(double x) {
    // Bit pattern of a non-negative double (NaN mapped to +inf) so that unsigned
    // integer max equals floating-point max; used for order-independent maxima.
    if (!(x >= 0.0)) x = INFINITY;
    return (uint64_t)__double_as_longlong(x);
}

__device__ inline double bitsd(uint64_t b) { return __longlong_as_double((long long)b); }

// Control block reset (every solve starts with all k columns active, in order: the
// packed list k_init_cols writes), and optionally the zeroed duplicate-index bitmap.
__global__ void k_ctrl_init(Ctrl *ctrl, int32_t start_prec, int64_t k, int32_t sym0, double cont_alpha,
                            uint32_t *bitmap, int64_t bitmap_words) {
    uint32_t *w = (uint32_t *)ctrl;
    constexpr int words = (int)(sizeof(Ctrl) / sizeof(uint32_t));
    for (int q = threadIdx.x; q < words; q += blockDim.x) w[q] = 0u;
    for (int64_t q = threadIdx.x; q < bitmap_words; q += blockDim.x) bitmap[q] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        ctrl->prec = start_prec;
        ctrl->active = (int32_t)k;
        ctrl->kact = (int32_t)k;
        ctrl->sym = sym0;
        ctrl->prev_maxstep = INFINITY;
        ctrl->dscale = 1.0;
        ctrl->zscale = 1.0;
        // continuation: sweep 1 applies the map of D + (1 - alpha) Delta
        ctrl->apow = cont_alpha;
        ctrl->escale = 1.0 - cont_alpha;
    }
}

__global__ void k_fill_u32(uint32_t *p, int64_t count, uint32_t v) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = v;
}

// Column state of a solve (the requested indices checked: in range, no repeats); with
// cs.alist the packed list of the first sweep (column c at position c), and with theta
// the order check of theta (finite; k_theta_order's flags) over the same grid.
__device__ inline void theta_order_flags(Ctrl *ctrl, const double *theta, int64_t n, int64_t j0, int64_t stride) {
    int32_t bits = 0;
    bool bad = false;
    for (int64_t j = j0; j < n; j += stride) {
        const double a = theta[j];
        bad |= !isfinite(a);
        if (j + 1 < n) {
            const double b = theta[j + 1];
            if (!(b > a)) bits |= 1;
            if (!(b < a)) bits |= 2;
        }
    }
    // one atomic per block and flag, and none for a flag another block has already set
    // (atomics on one word serialise: one per wave cost tens of microseconds at n = 2e5)
    const bool any_bad = __syncthreads_or(bad) != 0;
    const int32_t wbits = (__syncthreads_or(bits & 1) ? 1 : 0) | (__syncthreads_or(bits & 2) ? 2 : 0);
    if (threadIdx.x == 0) {
        if (any_bad) atomicMax(&ctrl->error, (int32_t)IPT_EINVAL);
        if (wbits & ~__hip_atomic_load(&ctrl->theta_order, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicOr(&ctrl->theta_order, wbits);
    }
}

__global__ void k_init_cols(Ctrl *ctrl, ColState cs, const int32_t *idx_user, int64_t n, int64_t k, int64_t kp,
                            uint32_t *bitmap, int32_t ntiles, int32_t start_stamp, const double *theta) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (theta) theta_order_flags(ctrl, theta, n, c, (int64_t)gridDim.x * blockDim.x);
    if (c < ntiles) cs.tile_stamp[c] = start_stamp;
    if (c >= kp) return;
    if (cs.alist) cs.alist[c] = (int32_t)c;  // positions past k are never read (kact = k)
    int32_t state = COL_PAD, i = 0;
    if (c < k) {
        const int64_t ii = idx_user ? (int64_t)idx_user[c] : c;
        if (ii < 0 || ii >= n) {
            atomicMax(&ctrl->error, (int32_t)IPT_EINVAL);
        } else {
            if (idx_user) {  // the default columns 0 .. k-1 cannot repeat
                const uint32_t bit = 1u << (ii & 31);
                const uint32_t old = atomicOr(&bitmap[ii >> 5], bit);
                if (old & bit) atomicMax(&ctrl->error, (int32_t)IPT_EINVAL);  // duplicate index
            }
            i = (int32_t)ii;
        }
        state = COL_ACTIVE;
    }
    cs.idx[c] = i;
    cs.state[c] = state;
    cs.sweeps[c] = 0;
    cs.grow[c] = 0;
    cs.par[c] = PAR_BUF0;
    cs.prev[c] = INFINITY;
    cs.step[c] = INFINITY;
    cs.lam[c] = 0.0;
    cs.resid[c] = 0.0;
}

// theta must be finite, and theta_j != theta_i for every j != i = idx[c]: the
// inverse gaps G_ji are then defined for every requested column.  A strictly monotone
// theta (k_theta_order: one comparison per adjacent pair) has distinct entries, and
// the pairwise check then returns at once.
__global__ void k_theta_order(Ctrl *ctrl, const double *theta, int64_t n) {
    theta_order_flags(ctrl, theta, n, blockIdx.x * (int64_t)blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

__global__ void k_check_theta(Ctrl *ctrl, const double *theta, const int32_t *idx, int64_t n, int64_t k) {
    if (ctrl->theta_order != 3) return;  // strictly monotone (and finite, checked with the order)
    __shared__ double ti[256];
    __shared__ int32_t ii[256];
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.y * 256;
    const int64_t cc = c0 + threadIdx.x;
    if (cc < k) {
        ii[threadIdx.x] = idx[cc];
        ti[threadIdx.x] = theta[idx[cc]];
    }
    __syncthreads();
    if (j >= n) return;
    const double tj = theta[j];
    if (blockIdx.y == 0 && !isfinite(tj)) atomicMax(&ctrl->error, (int32_t)IPT_EINVAL);
    const int64_t cend = (k - c0 < 256) ? (k - c0) : 256;
    bool degen = false;
    for (int64_t q = 0; q < cend; ++q) degen |= (tj == ti[q]) && (j != ii[q]);
    if (degen) atomicMax(&ctrl->error, (int32_t)IPT_EDEGENERATE);
}

// Conversions to the shadow element types (round to nearest even).
template <typename T>
__device__ inline T to_low(double x);
template <>
__device__ inline float to_low<float>(double x) { return (float)x; }
template <>
__device__ inline __bf16 to_low<__bf16>(double x) { return (__bf16)(float)x; }
template <>
__device__ inline _Float16 to_low<_Float16>(double x) { return (_Float16)(float)x; }

__device__ inline uint64_t wave_max_u64(uint64_t v);              // max over the wave (below)
__device__ inline void wave_atomic_max(uint64_t *p, uint64_t v);  // one atomic max per wave (below)
__device__ inline void block_atomic_max(uint64_t *p, uint64_t v);  // one atomic max per block (below)

// Row-major pass over Delta: a zero-padded FP64 copy (when Delta is not tile
// aligned), the BF16 and FP32 shadows of the ladder, per-block maxima of |Delta_jl|
// (for the scale of the FP16 shadows, which k_scan_delta writes; reduced by
// k_set_dscale, so no two blocks write the same word), and per-chunk partial column
// sums of |M| for |M|_1 = max_c sum_j |M_jc|, M = diag(theta) + Delta.  Block: 256 columns x
// PREP_ROWS rows; thread (cx, ry) holds columns 4cx..4cx+3 (16-byte loads) and walks
// rows ry, ry + 4, ..., four rows in flight.
constexpr int PREP_ROWS = 32;

template <typename TL>
__global__ __launch_bounds__(256) void k_prep_delta(Ctrl *ctrl, const double *theta, const double *delta,
                                                    int64_t lda, int64_t n, int64_t np, double *dpad, TL *dlo,
                                                    float *d32, double *colpart, uint64_t *bmax) {
    typedef TL tl4_t __attribute__((ext_vector_type(4)));
    __shared__ double sh[4][256];
    __shared__ uint64_t wmax[4];
    const int cx = threadIdx.x & 63, ry = threadIdx.x >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * 256 + 4 * cx;
    const int64_t r0 = (int64_t)blockIdx.y * PREP_ROWS;
    const bool vec = ((lda & 1) == 0) && (((uintptr_t)delta & 15) == 0) && c0 + 4 <= n;
    const bool live = c0 < np;  // np is a multiple of 128, so c0 + 4 <= np
    double acc[4] = {0.0, 0.0, 0.0, 0.0}, th[4], vmax = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) th[e] = c0 + e < n ? theta[c0 + e] : 0.0;
    // Loads read a clamped (valid) row and column and are masked afterwards, so the
    // four rows' loads issue back to back without branches between them.
    auto walk = [&](auto vec_tag) {
        constexpr bool VEC = decltype(vec_tag)::value;
        for (int q0 = 0; q0 < PREP_ROWS / 4; q0 += 4) {
            double v[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t j = r0 + ry + 4 * (q0 + u);
                const int64_t jc = j < n ? j : n - 1;
                if constexpr (VEC) {
                    const double2 x = *(const double2 *)(delta + jc * lda + c0);
                    const double2 y = *(const double2 *)(delta + jc * lda + c0 + 2);
                    v[u][0] = x.x;
                    v[u][1] = x.y;
                    v[u][2] = y.x;
                    v[u][3] = y.y;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int64_t cc = c0 + e < n ? c0 + e : n - 1;
                        v[u][e] = delta[jc * lda + cc];
                    }
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (!(j < n && c0 + e < n)) v[u][e] = 0.0;
            }
            if (!live) continue;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t j = r0 + ry + 4 * (q0 + u);
                if (j >= np) continue;
                const int64_t o = j * np + c0;
                if (dpad) {
                    *(double2 *)(dpad + o) = double2{v[u][0], v[u][1]};
                    *(double2 *)(dpad + o + 2) = double2{v[u][2], v[u][3]};
                }
                if (dlo)
                    *(tl4_t *)(dlo + o) = tl4_t{to_low<TL>(v[u][0]), to_low<TL>(v[u][1]), to_low<TL>(v[u][2]),
                                                to_low<TL>(v[u][3])};
#pragma unroll
                for (int e = 0; e < 4; ++e) vmax = fmax(vmax, fabs(v[u][e]));
                if (d32)
                    *(float4 *)(d32 + o) = float4{(float)v[u][0], (float)v[u][1], (float)v[u][2], (float)v[u][3]};
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    acc[e] += fabs(j == c0 + e ? v[u][e] + th[e] : v[u][e]);  // padding adds 0
            }
        }
    };
    if (vec) walk(std::true_type{});
    else walk(std::false_type{});
    if (bmax) {
        const uint64_t v = wave_max_u64(dbits(vmax));
        if (cx == 0) wmax[ry] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint64_t m01 = wmax[0] > wmax[1] ? wmax[0] : wmax[1], m23 = wmax[2] > wmax[3] ? wmax[2] : wmax[3];
            bmax[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = m01 > m23 ? m01 : m23;
        }
    }
    if (!colpart) return;
#pragma unroll
    for (int e = 0; e < 4; ++e) sh[ry][4 * cx + e] = acc[e];
    __syncthreads();
    if (ry == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t c = c0 + e;
            const int x = 4 * cx + e;
            if (c < n) colpart[(int64_t)blockIdx.y * n + c] = ((sh[0][x] + sh[1][x]) + sh[2][x]) + sh[3][x];
        }
    }
}

__global__ void k_norm1_reduce(Ctrl *ctrl, const double *colpart, int64_t n, int64_t chunks) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= n) return;
    double acc = 0.0;
    int64_t q = 0;
    for (; q + 8 <= chunks; q += 8) {  // eight loads in flight, added in chunk order
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = colpart[(q + u) * n + c];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; q < chunks; ++q) acc += colpart[q * n + c];
    atomicMax((unsigned long long *)&ctrl->norm1_bits, (unsigned long long)dbits(acc));
}

// CSR column sums: off-diagonal |Delta_jc| go to scratch[c], diagonal entries of
// Delta to scratch[n + c] (added to theta_c before taking the modulus).  Double
// atomics: the norm is a diagnostic (it scales the reported eigen-residual) and
// takes no part in any decision, so the order of the sums is free.  (An exact check
// that |M| is symmetric, which would turn the column sums into row sums, reads a
// random line of row_ptr, col and val per entry and costs as much as the atomics.)
// |M|_1 of a CSR matrix: the column sums of |Delta| off the diagonal are accumulated
// as fixed-point integers (deterministic in any order), at a power-of-two scale from
// S = sum |val| that keeps every column sum below 2^62:
//   k_csr_abs_sum  : per-block sums of |val| (and clears the integer column sums),
//   k_csr_abs_scale: S and the scale 2^(62 - ceil(log2 S)) (0 when S is not finite),
//   k_csr_colsum   : one 64-bit integer atomic add per off-diagonal entry,
//   k_norm1_csr_reduce: per column, the sum / scale + |theta_j + Delta_jj| (the diagonal
//                    entries of row j, in storage order), maximum over columns.
// Complex entries (cplx: val holds (re, im) pairs, theta_im the imaginary parts of
// theta) enter by their modulus.
constexpr int CSR_SUM_BLOCKS = 1024;
__device__ inline double csr_abs(const double *val, int64_t p, int32_t cplx) {
    if (!cplx) return fabs(val[p]);
    const double re = val[2 * p], im = val[2 * p + 1];
    return sqrt(re * re + im * im);
}

__global__ __launch_bounds__(256) void k_csr_abs_sum(const Ctrl *ctrl, const double *val, int64_t nnz,
                                                     uint64_t *acc, int64_t n, double *part, int32_t cplx) {
    if (ctrl->error) return;
    __shared__ double sh[256];
    double a = 0.0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
        a += csr_abs(val, p, cplx);
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        acc[j] = 0;
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_csr_abs_scale(const Ctrl *ctrl, const double *part, int nb, double *scale) {
    if (ctrl->error) return;
    __shared__ double sh[256];
    double a = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) a += part[b];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double S = sh[0];
        *scale = !isfinite(S) ? 0.0 : (S > 0.0 ? exp2(fmin(62.0 - ceil(log2(S)), 1000.0)) : 1.0);
    }
}

__global__ void k_csr_colsum(const Ctrl *ctrl, const int32_t *row_ptr, const int32_t *col, const double *val,
                             int64_t n, const double *scale, uint64_t *acc, int32_t cplx) {
    if (ctrl->error) return;  // the structure checks ran first; never walk a malformed matrix
    const double sc = *scale;
    if (!(sc > 0.0)) return;
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    for (int32_t p = row_ptr[j]; p < row_ptr[j + 1]; ++p) {
        const int32_t c = col[p];
        if (c != j)
            atomicAdd((unsigned long long *)&acc[c], (unsigned long long)llrint(csr_abs(val, p, cplx) * sc));
    }
}

// Block: grid-stride over columns, one atomic max per block.
__global__ __launch_bounds__(256) void k_norm1_csr_reduce(Ctrl *ctrl, const double *theta, const int32_t *row_ptr,
                                                          const int32_t *col, const double *val, const uint64_t *acc,
                                                          const double *scale, int64_t n, const double *theta_im) {
    if (ctrl->error) return;
    const double sc = *scale;
    const int32_t cplx = theta_im != nullptr;
    uint64_t m = 0;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        double dg = 0.0, dgi = 0.0;
        for (int32_t p = row_ptr[c]; p < row_ptr[c + 1]; ++p)
            if (col[p] == c) {
                dg += cplx ? val[2 * p] : val[p];
                if (cplx) dgi += val[2 * p + 1];
            }
        const double off = sc > 0.0 ? (double)acc[c] / sc : NAN;  // NaN (reported as +inf) for a non-finite Delta
        const double dre = theta[c] + dg, dim = cplx ? theta_im[c] + dgi : 0.0;
        const uint64_t b = dbits(off + (cplx ? sqrt(dre * dre + dim * dim) : fabs(dre)));
        m = b > m ? b : m;
    }
    block_atomic_max(&ctrl->norm1_bits, m);
}

// Z <- z0 with Z[idx[c], c] = 1 (chart U_i), or Z <- E when z0 is NULL; padding zero.
// Writes columns [0, kw) of rows [0, np) (grid-stride over the np x kw elements).
// Also records max |Z - E| in ctrl->acc_maxdist (when want_max), from which
// k_set_zscale scales the FP16 shadow of Z - E for a first sweep on that rung.
__global__ void k_load_z0(Ctrl *ctrl, const double *z0, int64_t ldz0, double *zb, int64_t ldzb, const int32_t *idx,
                          int64_t n, int64_t np, int64_t k, int64_t kw, int32_t want_max) {
    if (ctrl->error) return;
    const int64_t total = np * kw;
    double m = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / kw, c = e - j * kw;
        double v = 0.0;
        if (j < n && c < k) v = (j == idx[c]) ? 1.0 : (z0 ? z0[j * ldz0 + c] : 0.0);
        zb[j * ldzb + c] = v;
        if (j < n && c < k && j != idx[c]) m = fmax(m, fabs(v));
    }
    if (want_max) wave_atomic_max(&ctrl->acc_maxdist, dbits(isfinite(m) ? m : 0.0));
}

__global__ void k_set_zscale(Ctrl *ctrl) {
    const double md = bitsd(ctrl->acc_maxdist);
    ctrl->zscale = (md > 0.0 && isfinite(md)) ? exp2(floor(log2(8192.0 / md))) : 1.0;
    ctrl->acc_maxdist = 0;
}

// Zero the padding rows [n, np) and padding columns [k, kp) of a Z buffer.
__global__ void k_zero_pad(double *zb, int64_t ldzb, int64_t n, int64_t np, int64_t k, int64_t kp) {
    const int64_t total = np * kp;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / kp, c = e - j * kp;
        if (j >= n || c >= k) zb[j * ldzb + c] = 0.0;
    }
}

// Block-wide reduction of per-thread column partials laid out as 4 row groups of
// 64 columns: thread (cx = t & 63, ry = t >> 6).  Sums the 4 groups in a fixed order
// and writes part[rt][c][q].
__device__ inline void store_col_partials(double (*sh)[4][64], const double v[NPART], int cx, int ry, double *part,
                                          int64_t rt, int64_t kp, int64_t c) {
#pragma unroll
    for (int q = 0; q < NPART; ++q) sh[ry][q][cx] = v[q];
    __syncthreads();
    if (ry == 0) {
#pragma unroll
        for (int q = 0; q < NPART; ++q) {
            const double s = ((sh[0][q][cx] + sh[1][q][cx]) + sh[2][q][cx]) + sh[3][q][cx];
            part[(rt * kp + c) * NPART + q] = s;
        }
    }
}

// First sweep of a cold start (Z = I): W = F(I) needs no product because
// Delta I = Delta exactly.  W_jc = -Delta_ji / (theta_j - theta_i) for j != i,
// W_ic = 1, d_c = Delta_ii (eq. dyn at Z = I; the first-order RS term of
// eq. ARS-alpha).  Block: one row tile of TILE_M rows x 64 columns.
__global__ __launch_bounds__(256) void k_sweep1_dense(const Ctrl *ctrl, const double *theta, const double *delta,
                                                      int64_t lda, ColState cs, double *dvec, double *zout,
                                                      int64_t ldzb, double *part, int64_t n, int64_t kp, double *dnp) {
    if (ctrl->error || ctrl->done) return;
    __shared__ double sh[4][4][64];
    __shared__ double sdn[2][4][64];
    const int cx = threadIdx.x & 63, ry = threadIdx.x >> 6;
    const int64_t rt = blockIdx.y;
    const int64_t c = (int64_t)blockIdx.x * 64 + cx;
    const bool colok = cs.state[c] == COL_ACTIVE;
    const int32_t i = cs.idx[c];
    const double ti = theta[i];
    const bool sym = ctrl->sym != 0;
    double v[NPART] = {0.0, 0.0, 0.0, 0.0};
    // Partials of the next sweep's d = sum_j Delta_ij W_jc, in the FP64 sweep
    // epilogue's order: rows ry + 4q for q < 16 (q >= 16) are that epilogue's rows of
    // lane group ry in wave row 0 (1), in the same order.
    double dn[2] = {0.0, 0.0};
    for (int q = 0; q < TILE_M / 4; ++q) {
        const int64_t j = rt * TILE_M + ry + 4 * q;
        double w = 0.0;
        if (colok && j < n) {
            const double dji = delta[j * lda + i];
            if (j == i) {
                w = 1.0;
                v[1] += 1.0;  // z_ii^2
            } else {
                const double gap = theta[j] - ti;
                w = -dji / gap;
                const double st = w;  // z_jc = 0
                v[0] += st * st;
                v[2] += (gap * st) * (gap * st);
                v[3] += w * w;
            }
            if (dnp) {
                const double dij = sym ? dji : delta[(int64_t)i * lda + j];
                dn[q >> 4] = fma(dij, w, dn[q >> 4]);
            }
        }
        zout[j * ldzb + c] = w;
    }
    if (colok && rt == (int64_t)(i / TILE_M) && ry == 0) dvec[c] = delta[(int64_t)i * lda + i];
    if (dnp) {
        sdn[0][ry][cx] = dn[0];
        sdn[1][ry][cx] = dn[1];
    }
    store_col_partials(sh, v, cx, ry, part, rt, kp, c);  // synchronizes the block first
    if (dnp && ry == 0 && colok) {
        const double r0 = (sdn[0][0][cx] + sdn[0][1][cx]) + (sdn[0][2][cx] + sdn[0][3][cx]);
        const double r1 = (sdn[1][0][cx] + sdn[1][1][cx]) + (sdn[1][2][cx] + sdn[1][3][cx]);
        dnp[rt * kp + c] = r0 + r1;
    }
}

// Pairs of 64 x 64 tiles of Delta: block b takes the b-th pair (I, J), I >= J, in
// row-major lower-triangle order over the padded np x np (entries outside Delta are
// 0), compares Delta[I, J] with the transpose of Delta[J, I] bit for bit (the second
// tile goes through LDS; any difference clears ctrl->sym), and writes both tiles'
// FP16 shadows with the power-of-two scale ctrl->dscale: f16 = the FP16 low rung's
// shadow, hi (lo = hi + np^2) = the split of the three-product rung.  It runs right
// after the row-major pass over Delta, whose reads leave Delta in the last-level
// cache for these transposed ones.
__global__ __launch_bounds__(256) void k_scan_delta(Ctrl *ctrl, const double *delta, int64_t lda, int64_t n,
                                                    int64_t np, int64_t nb, int32_t want_sym, _Float16 *f16,
                                                    _Float16 *hi) {
    __shared__ double tb[64][65];
    __shared__ int32_t go;
    if (threadIdx.x == 0) go = want_sym && ctrl->sym;  // one read per block keeps the branch uniform
    __syncthreads();
    const bool cmp = go != 0;
    if (!cmp && !f16 && !hi) return;
    const int64_t b = blockIdx.x;
    // lower-triangle decode: bi (bi + 1) / 2 <= b < (bi + 1)(bi + 2) / 2
    int64_t bi = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= b) ++bi;
    while (bi * (bi + 1) / 2 > b) --bi;
    const int64_t bj = b - bi * (bi + 1) / 2;
    if (bi >= nb) return;
    // thread -> column pair 2 cp, 2 cp + 1 of rows ry + 8 q: both tiles' 16 loads issue
    // before any of them is used.  Entries outside Delta count as 0; their loads read a
    // valid address instead.  16-byte loads need an even n (a pair is then wholly
    // inside or outside Delta), an even lda and an aligned Delta.
    const int cp = threadIdx.x & 31, ry = threadIdx.x >> 5;
    const int64_t r0 = bi * 64, c0 = bj * 64;
    const bool pair = ((n & 1) == 0) && ((lda & 1) == 0) && (((uintptr_t)delta & 15) == 0);
    double2 va[8], vb[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int rr = ry + 8 * q;
        const int64_t ra = r0 + rr, ca = c0 + 2 * cp;  // Delta[I, J]
        const int64_t rb = c0 + rr, cb = r0 + 2 * cp;  // Delta[J, I]
        if (pair) {
            const bool oka = ra < n && ca < n, okb = rb < n && cb < n;
            const double2 x = *(const double2 *)(delta + (oka ? ra * lda + ca : 0));
            const double2 y = *(const double2 *)(delta + (okb ? rb * lda + cb : 0));
            va[q] = oka ? x : double2{0.0, 0.0};
            vb[q] = okb ? y : double2{0.0, 0.0};
        } else {
            double e[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t r = u < 2 ? ra : rb, c = (u < 2 ? ca : cb) + (u & 1);
                const bool ok = r < n && c < n;
                const double v = delta[ok ? r * lda + c : 0];
                e[u] = ok ? v : 0.0;
            }
            va[q] = double2{e[0], e[1]};
            vb[q] = double2{e[2], e[3]};
        }
    }
    if (f16 || hi) {
        typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
        const double ds = ctrl->dscale;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int rr = ry + 8 * q;
#pragma unroll
            for (int t2 = 0; t2 < 2; ++t2) {
                if (t2 == 1 && bi == bj) break;  // a diagonal tile is its own mirror
                const double2 v = t2 ? vb[q] : va[q];
                const int64_t o = t2 ? (c0 + rr) * np + r0 + 2 * cp : (r0 + rr) * np + c0 + 2 * cp;
                const double x0 = v.x * ds, x1 = v.y * ds;
                const h2_t h{to_low<_Float16>(x0), to_low<_Float16>(x1)};
                if (f16) *(h2_t *)(f16 + o) = h;
                if (hi) {
                    *(h2_t *)(hi + o) = h;
                    *(h2_t *)(hi + np * np + o) =
                        h2_t{to_low<_Float16>(x0 - (double)h[0]), to_low<_Float16>(x1 - (double)h[1])};
                }
            }
        }
    }
    if (!cmp) return;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        tb[ry + 8 * q][2 * cp] = vb[q].x;
        tb[ry + 8 * q][2 * cp + 1] = vb[q].y;
    }
    __syncthreads();
    bool diff = false;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int rr = ry + 8 * q;  // Delta[r0 + rr, c0 + 2cp + e] against Delta[c0 + 2cp + e, r0 + rr]
        diff |= __double_as_longlong(va[q].x) != __double_as_longlong(tb[2 * cp][rr]);
        diff |= __double_as_longlong(va[q].y) != __double_as_longlong(tb[2 * cp + 1][rr]);
    }
    if (__syncthreads_or(diff) && threadIdx.x == 0) ctrl->sym = 0;
}

// d_c = (Delta Z)_{i,c} = sum_l Delta_il Z_lc in FP64 for the active columns, as
// per-row-tile partials dnp[tm][c] (tiles of TILE_M rows) that k_diag_reduce adds.
// Each partial is summed in exactly the order in which the FP64 sweep epilogue forms
// the same quantity for the next sweep (rows held by wave row wm and lane group g:
// wm*64 + 16ib + 4r + g, in (ib, r) order, by fused multiply-adds; the four groups
// as (g0 + g1) + (g2 + g3); then wm 0 + wm 1), and k_diag_reduce adds the tiles in
// the finalize's order, so a solve resumed from a returned iterate computes bit for
// bit the d that the uninterrupted solve took from its epilogue.  Block: 64 columns
// x one row tile.  The 64 row segments Delta[idx[c], tile] are staged in LDS with
// coalesced loads; thread (cx, w) then sums the slots (wm, g) = 2w and 2w + 1.
__global__ __launch_bounds__(256) void k_diag_tiles(const Ctrl *ctrl, const double *delta, int64_t lda,
                                                    const double *zin, int64_t ldzb, ColState cs, double *dnp,
                                                    int64_t n, int64_t kp) {
    if (ctrl->error || ctrl->done) return;
    __shared__ double ds[64][TILE_M + 1];
    __shared__ double sh[8][64];
    __shared__ int32_t srow[64];
    const int cx = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * 64, c = c0 + cx;
    const int64_t tm = blockIdx.y, j0 = tm * TILE_M;
    const bool act = cs.state[c] == COL_ACTIVE;
    if (w == 0) srow[cx] = act ? cs.idx[c] : -1;
    if (!__syncthreads_or(act)) return;
    // Wave w stages rows 16w .. 16w + 15 of ds (one 128-entry segment of Delta row
    // idx[c] each); addresses are clamped into Delta and the values masked, so the
    // 32 loads of a lane issue without branches between them.
    const int64_t ja = j0 + cx < n ? j0 + cx : n - 1, jb = j0 + cx + 64 < n ? j0 + cx + 64 : n - 1;
    const bool oka = j0 + cx < n, okb = j0 + cx + 64 < n;
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
        const int row = 16 * w + rr;
        const int32_t i = srow[row];
        const double *drow = delta + (int64_t)(i >= 0 ? i : 0) * lda;
        const double va = drow[ja], vb = drow[jb];
        ds[row][cx] = (i >= 0 && oka) ? va : 0.0;
        ds[row][cx + 64] = (i >= 0 && okb) ? vb : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int slot = 2 * w + s, wm = slot >> 2, g = slot & 3;
        double acc = 0.0;
        if (act) {
            double z[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int64_t j = j0 + wm * 64 + 16 * (q >> 2) + 4 * (q & 3) + g;
                z[q] = zin[(j < n ? j : n - 1) * ldzb + c];
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) {  // q = 4 ib + r
                const int jl = wm * 64 + 16 * (q >> 2) + 4 * (q & 3) + g;
                const double nxt = fma(ds[cx][jl], z[q], acc);
                acc = (j0 + jl < n) ? nxt : acc;  // rows past n: skipped, as in the epilogue
            }
        }
        sh[slot][cx] = acc;
    }
    __syncthreads();
    if (w == 0 && act) {
        const double r0 = (sh[0][cx] + sh[1][cx]) + (sh[2][cx] + sh[3][cx]);
        const double r1 = (sh[4][cx] + sh[5][cx]) + (sh[6][cx] + sh[7][cx]);
        dnp[tm * kp + c] = r0 + r1;
    }
}

// d_c = the row-tile partials added exactly as the finalize adds them: group g sums
// tiles g, g + 4, ... in order, then ((s0 + s1) + s2) + s3.  Block: 64 columns x 4
// groups.
__global__ __launch_bounds__(256) void k_diag_reduce(const Ctrl *ctrl, ColState cs, const double *dnp, double *d,
                                                     int64_t nrt, int64_t kp) {
    if (ctrl->error || ctrl->done) return;
    __shared__ double sh[4][64];
    const int cx = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t c = (int64_t)blockIdx.x * 64 + cx;
    const bool act = cs.state[c] == COL_ACTIVE;
    double a = 0.0;
    if (act)
        for (int64_t rt = g; rt < nrt; rt += 4) a += dnp[rt * kp + c];
    sh[g][cx] = a;
    __syncthreads();
    if (g == 0 && act) d[c] = ((sh[0][cx] + sh[1][cx]) + sh[2][cx]) + sh[3][cx];
}

__device__ inline uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = (uint64_t)__shfl_xor((unsigned long long)v, off);
        v = o > v ? o : v;
    }
    return v;
}

// Adds the number of lanes with pred set to *p with one atomic per wave.
__device__ inline void wave_count(int32_t *p, bool pred) {
    const uint64_t m = __ballot(pred);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(p, (int32_t)__popcll(m));
}

__device__ inline void wave_atomic_max(uint64_t *p, uint64_t v) {
    v = wave_max_u64(v);
    if ((threadIdx.x & 63) == 0 && v) atomicMax((unsigned long long *)p, (unsigned long long)v);
}

// Every thread of the block must call it (blockDim.x a multiple of 64, at most 1024).
__device__ inline void block_atomic_max(uint64_t *p, uint64_t v) {
    __shared__ uint64_t wm[16];
    v = wave_max_u64(v);
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t m = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = wm[w] > m ? wm[w] : m;
        if (m) atomicMax((unsigned long long *)p, (unsigned long long)m);
    }
}

// Finalize sweep t for every active column: reduce the partial sums over row
// tiles in a fixed order, form s_c = |W_c - Z_c| / |Z_c| (Alg. 1 loop test,
// Euclidean norms), and decide.  Only an exact sweep (FP64 product, or the
// product-free first sweep) may certify a column; a certified column keeps its
// input iterate and lambda_c = theta_i + d_c of this sweep (Alg. 1/2 return steps).
// Block: 64 columns; thread (cx, g) sums row tiles g, g + 4, ...; wave 0 decides.
// The finalize of columns 64 blk .. 64 blk + 63 by one block of 256 threads (k_finalize
// runs one such group per block; the CSR sweep tail runs all groups in its last block).
__device__ void finalize_cols(Ctrl *ctrl, const DevOpts &o, ColState cs, double *dvec, const double *theta,
                              const double *part, int64_t nrt, int64_t kp, int32_t sweep, int32_t in_par,
                              int32_t out_par, const double *dnp, const double *theta_im, const double *dvec_im,
                              double *lam_im, int64_t blk) {
    __shared__ double sh[4][NPART + 1][64];
    const int cx = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t c = blk * 64 + cx;
    const bool act = cs.state[c] == COL_ACTIVE;
    double p[NPART] = {0.0, 0.0, 0.0, 0.0}, dn = 0.0;
    if (act) {
        for (int64_t rt = g; rt < nrt; rt += 4) {
            const double4 v = *(const double4 *)&part[(rt * kp + c) * NPART];
            p[0] += v.x;
            p[1] += v.y;
            p[2] += v.z;
            p[3] += v.w;
            if (dnp) dn += dnp[rt * kp + c];
        }
    }
#pragma unroll
    for (int q = 0; q < NPART; ++q) sh[g][q][cx] = p[q];
    sh[g][NPART][cx] = dn;
    __syncthreads();
    if (g != 0) {
        __syncthreads();  // sh is free again for the next group once wave 0 has read it
        return;
    }
#pragma unroll
    for (int q = 0; q < NPART; ++q) p[q] = ((sh[0][q][cx] + sh[1][q][cx]) + sh[2][q][cx]) + sh[3][q][cx];
    dn = ((sh[0][NPART][cx] + sh[1][NPART][cx]) + sh[2][NPART][cx]) + sh[3][NPART][cx];
    int32_t decided = -1;
    double s = 0.0;
    uint64_t res_bits = 0;
    // IPT-ACX: only the first application of a cycle is tested; the budget rule ends
    // a column whose cycle could not be followed by another test within max_iter
    // (with plain sweeps, p = 1: the last sweep).
    int32_t q, pc;
    acx_phase(o.acx, sweep, q, pc);
    // continuation sweep (scale es < 1): no column certifies, the growth rule restarts,
    // and |W - e| of the scaled iterate is es |F(Z) - e|
    const double es = ctrl->escale;
    const bool scaled = es < 1.0;
    if (act && q != 0) {
        s = sqrt(p[0]) / sqrt(p[1]);
        cs.tile_stamp[c / TILE_N] = sweep;
    } else if (act) {
        const double d = dvec[c];
        s = sqrt(p[0]) / sqrt(p[1]);
        const int32_t prec = ctrl->prec;
        const bool exact = (prec == PREC_F64) || (prec == PREC_EXACT_FIRST);
        const double nrm = bitsd(ctrl->norm1_bits);
        const double resid = sqrt(p[2]) / (nrm > 0.0 ? nrm : 1.0) / sqrt(p[1]);
        const int32_t i = cs.idx[c];
        int32_t par = 0;
        if (exact && !scaled && s <= o.tol) {
            decided = COL_CONVERGED;
            par = in_par;
            res_bits = dbits(resid);
        } else {
            const bool bad = !isfinite(s) || !((scaled ? es * sqrt(p[3]) : sqrt(p[3])) <= o.div_norm);
            int32_t grow = cs.grow[c];
            if (scaled) {
                grow = 0;
                cs.prev[c] = INFINITY;
                cs.grow[c] = 0;
            } else if (exact) {
                grow = (s > cs.prev[c]) ? grow + 1 : 0;
                cs.prev[c] = s;
                cs.grow[c] = grow;
            }
            if (bad || grow >= o.div_growth) {
                decided = COL_DIVERGED;
                par = out_par;
            } else if (sweep + pc > o.max_iter) {
                decided = COL_NOT_CONVERGED;
                par = out_par;
            }
        }
        if (decided >= 0) {
            cs.state[c] = decided;
            cs.par[c] = par;
            cs.sweeps[c] = sweep;
            cs.step[c] = s;
            cs.lam[c] = theta[i] + (scaled ? es * d : d);
            if (lam_im) lam_im[c] = theta_im[i] + (scaled ? es * dvec_im[c] : dvec_im[c]);  // complex solves
            cs.resid[c] = resid;
        } else {
            cs.tile_stamp[c / TILE_N] = sweep;
        }
    }
    const bool still = act && decided < 0;
    if (dnp && still) dvec[c] = dn;  // d of the next sweep, whose input is this sweep's W
    wave_atomic_max(&ctrl->acc_maxstep, act ? dbits(s) : 0);
    wave_atomic_max(&ctrl->acc_maxdist, still ? dbits(sqrt(p[3])) : 0);
    wave_atomic_max(&ctrl->acc_maxres, res_bits);
    wave_atomic_max(&ctrl->dec_maxstep, decided >= 0 ? dbits(s) : 0);
    wave_count(&ctrl->acc_active, still);
    wave_count(&ctrl->n_conv, decided == COL_CONVERGED);
    wave_count(&ctrl->n_div, decided == COL_DIVERGED);
    wave_count(&ctrl->n_notconv, decided == COL_NOT_CONVERGED);
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_finalize(Ctrl *ctrl, DevOpts o, ColState cs, double *dvec,
                                                  const double *theta, const double *part, int64_t nrt, int64_t kp,
                                                  int32_t sweep, int32_t in_par, int32_t out_par, const double *dnp,
                                                  const double *theta_im, const double *dvec_im, double *lam_im) {
    if (ctrl->error || ctrl->done) return;
    finalize_cols(ctrl, o, cs, dvec, theta, part, nrt, kp, sweep, in_par, out_par, dnp, theta_im, dvec_im, lam_im,
                  blockIdx.x);
}

__device__ void control_step(Ctrl *ctrl, const DevOpts &o, int32_t sweep);

// CSR sweep tail (plain sweeps), one block, after the per-column sums of the SpMM's
// row-tile partials: the finalize of every column, the next sweep's d for the columns
// still active (one wave per column, as k_diag_csr, on this sweep's output) and the
// control step.  One launch instead of three; the work itself is a few microseconds.
__global__ __launch_bounds__(256) void k_csr_tail(Ctrl *ctrl, DevOpts o, ColState cs, double *dvec,
                                                  const double *theta, const double *part, int64_t kpc,
                                                  int32_t sweep, int32_t in_par, int32_t out_par,
                                                  const int32_t *row_ptr, const int32_t *col, const double *val,
                                                  const double *zout, int64_t ldz, int64_t k) {
    if (ctrl->error || ctrl->done) return;
    for (int64_t blk = 0; blk < kpc / 64; ++blk)
        finalize_cols(ctrl, o, cs, dvec, theta, part, 1, kpc, sweep, in_par, out_par, nullptr, nullptr, nullptr,
                      nullptr, blk);
    // the column states were written by this block before the finalize's last barrier
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t cc = wv; cc < k; cc += 4) {
        if (cs.state[cc] != COL_ACTIVE) continue;  // the same for the whole wave
        const int32_t i = cs.idx[cc];
        double a2 = 0.0;
        for (int32_t p = row_ptr[i] + lane; p < row_ptr[i + 1]; p += 64) a2 += val[p] * zout[(int64_t)col[p] * ldz + cc];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a2 += __shfl_xor(a2, off);
        if (lane == 0) dvec[cc] = a2;
    }
    if (threadIdx.x == 0) {
        // the finalize's counters were accumulated with device-scope atomics: drop any
        // copy of the control block this compute unit's cache still holds
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        control_step(ctrl, o, sweep);
    }
}

// The active columns in ascending order: the packed column positions of the next
// dense sweep's GEMM (one block of 1024 threads; a block-wide scan per 1024 columns).
__device__ void plan_dense(Ctrl *ctrl, ColState cs, int64_t kp) {
    __shared__ int32_t s_w[16];
    __shared__ int32_t s_base;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < kp; c0 += 1024) {
        const int64_t c = c0 + threadIdx.x;
        const int act = (c < kp && cs.state[c] == COL_ACTIVE) ? 1 : 0;
        int inc = act;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(inc, off);
            if (lane >= off) inc += o;
        }
        if (lane == 63) s_w[wave] = inc;
        __syncthreads();
        int pos = s_base + inc - act;
        for (int w2 = 0; w2 < wave; ++w2) pos += s_w[w2];
        if (act) cs.alist[pos] = (int32_t)c;
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int w2 = 0; w2 < 16; ++w2) tot += s_w[w2];
            s_base += tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) ctrl->kact = s_base;
}

__global__ __launch_bounds__(1024) void k_plan_dense(Ctrl *ctrl, ColState cs, int64_t kp) {
    if (ctrl->error || ctrl->done) return;
    plan_dense(ctrl, cs, kp);
}

// Bookkeeping after sweep t and the precision of sweep t+1 (the ladder): leave the
// low rung when the max step is <= tau_low or stops falling, leave FP32 when it is
// <= tau_32 or stops falling; FP64 is final.

__global__ void k_control(Ctrl *ctrl, DevOpts o, int32_t sweep) {
    if (ctrl->error || ctrl->done) return;
    control_step(ctrl, o, sweep);
}

// Dense sweeps: the plan of the next sweep (packed active columns), then the control.
__global__ __launch_bounds__(1024) void k_control_plan(Ctrl *ctrl, DevOpts o, int32_t sweep, ColState cs,
                                                       int64_t kp) {
    if (ctrl->error || ctrl->done) return;
    // the packed list only changes when a column left the active set in this sweep
    if (ctrl->acc_active != ctrl->active) plan_dense(ctrl, cs, kp);
    __syncthreads();
    if (threadIdx.x == 0) control_step(ctrl, o, sweep);
}

__device__ void control_step(Ctrl *ctrl, const DevOpts &o, int32_t sweep) {
    const double ms = bitsd(ctrl->acc_maxstep);
    const int32_t prec = ctrl->prec;
    if (sweep - 1 < IPT_HIST) {
        ctrl->hist_prec[sweep - 1] = prec;
        ctrl->hist_active[sweep - 1] = ctrl->active;
        ctrl->hist_step[sweep - 1] = ms;
    }
    if (prec != PREC_EXACT_FIRST || o.first_product) ctrl->matvecs += ctrl->active;
    ctrl->active = ctrl->acc_active;
    ctrl->acc_active = 0;
    ctrl->acc_maxstep = 0;
    ctrl->sweeps = sweep;
    if (ctrl->active == 0 || sweep >= o.max_iter) ctrl->done = 1;
    int32_t next = PREC_F64;
    if (o.ladder) {
        // Leave a rung when its step is below the rung's threshold, when it stopped
        // falling (the rung's rounding floor), or when the next exact sweep is
        // predicted to certify: with the observed contraction ratio q = s_t / s_{t-1},
        // the next step is about q s_t.  "Certify" allows IPT_CERTIFY_SLACK: the
        // prediction is for the largest column step, and the few columns left above
        // tol cost one narrow FP64 sweep, far less than another full sweep of a rung.
        // A warm start has observed no ratio after its first sweep (prev_maxstep is
        // still +inf), so the prediction waits for a second step.
        const double slack_tol = IPT_CERTIFY_SLACK * o.tol;
        const bool stalled = !(ms < ctrl->prev_maxstep);
        const bool have_ratio = isfinite(ctrl->prev_maxstep) && ctrl->prev_maxstep > 0.0;
        const double predicted = ms * (ms / ctrl->prev_maxstep);
        const bool certify_next = have_ratio && isfinite(predicted) && predicted <= slack_tol;
        if (prec == PREC_EXACT_FIRST) {
            // From Z = E the first step is the first-order correction |G o Delta e_i|,
            // which also estimates the contraction ratio: q ~ s_1, so the step after
            // one more sweep is ~ s_1^2 and after two ~ s_1^3.  Go straight to FP64
            // when the next sweep should certify, and skip the low rung when an
            // FP32-class sweep followed by the certifying FP64 sweep should do.
            const bool f64_next = ms <= o.tau_32 || ms * ms <= slack_tol;
            const bool f32_next = ms <= o.tau_low || o.low_type == IPT_LOW_NONE || ms * ms * ms <= slack_tol;
            next = f64_next ? PREC_F64 : f32_next ? PREC_F32 : PREC_LOW;
        } else if (prec == PREC_LOW) {
            next = (ms <= o.tau_32) ? PREC_F64 : (ms <= o.tau_low || stalled) ? PREC_F32 : PREC_LOW;
        } else if (prec == PREC_F32) {
            next = (ms <= o.tau_32 || stalled || certify_next) ? PREC_F64 : PREC_F32;
        }
    }
    ctrl->prec = next;
    ctrl->prev_maxstep = ms;
    // continuation: the scale of sweep t + 1 is 1 - alpha^(t+1); it stays at 1 once there
    if (o.cont_alpha > 0.0 && ctrl->escale < 1.0) {
        ctrl->apow *= o.cont_alpha;
        ctrl->escale = 1.0 - ctrl->apow;
    }
    // FP16 shadows (FP16 low rung, three-product rung): scale Z - E by a power of two
    // so that its largest entry (bounded by max_c |W_c - e_i|) lands near 2^13, well
    // inside the FP16 range.
    if (o.ladder && (o.low_type == IPT_LOW_FP16 || o.mid_x3)) {
        const double md = bitsd(ctrl->acc_maxdist);
        ctrl->zscale = (md > 0.0 && isfinite(md)) ? exp2(floor(log2(8192.0 / md))) : 1.0;
    }
    ctrl->acc_maxdist = 0;
}

// The FP16 scale of the Delta shadows from max |Delta_jl| (the nb per-block maxima of
// k_prep_delta, kept in ctrl->dmax_bits): a power of two that brings the largest entry
// near 2^13.  One block.
__global__ __launch_bounds__(256) void k_set_dscale(Ctrl *ctrl, const uint64_t *bmax, int64_t nb) {
    __shared__ uint64_t wm[4];
    uint64_t m = 0;
    for (int64_t i = threadIdx.x; i < nb; i += 256) m = bmax[i] > m ? bmax[i] : m;
    m = wave_max_u64(m);
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x != 0) return;
    m = wm[0];
    for (int w = 1; w < 4; ++w) m = wm[w] > m ? wm[w] : m;
    ctrl->dmax_bits = m;
    const double md = bitsd(m);
    ctrl->dscale = (md > 0.0 && isfinite(md)) ? exp2(floor(log2(8192.0 / md))) : 1.0;
}

// z_out[:, c] <- the buffer holding column c's final value; lambda, status and the
// optional per-column outputs.
// Block: cw columns (a power of two, cw <= 256) x 256 / cw row lanes over 64-row
// chunks, so that narrow solves (few columns) still use every thread of a block.
__global__ __launch_bounds__(256) void k_copyout(const Ctrl *ctrl, ColState cs, const double *buf0,
                                                 const double *buf1, int64_t ldzb, double *z_out, int64_t ldz,
                                                 double *lambda_out, int32_t *status_out, int64_t n, int64_t k,
                                                 int32_t cw, int32_t *ci_sweeps, double *ci_step, double *ci_resid,
                                                 int32_t only_if_done) {
    if (ctrl->error || (only_if_done && !ctrl->done)) return;
    const int rl = threadIdx.x / cw, rstep = 256 / cw;
    const int64_t c = blockIdx.x * (int64_t)cw + (threadIdx.x % cw);
    const int64_t j0 = (int64_t)blockIdx.y * 64;
    if (c >= k) return;
    const int32_t par = cs.par[c];
    const int32_t i = cs.idx[c];
    const double *src = (par == PAR_BUF1) ? buf1 : buf0;
    // an iterate buffer that is z_out itself already holds the column in place
    const bool in_place = par != PAR_UNIT && src == z_out && ldzb == ldz;
    for (int64_t jb = in_place ? n : j0; jb < n; jb += (int64_t)gridDim.y * 64) {
        int64_t j1 = jb + 64;
        if (j1 > n) j1 = n;
        // eight rows per step, their loads issued together
        for (int64_t j = jb + rl; j < j1; j += 8 * rstep) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t jj = j + u * rstep;
                v[u] = jj < j1 ? ((par == PAR_UNIT) ? (jj == i ? 1.0 : 0.0) : src[jj * ldzb + c]) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t jj = j + u * rstep;
                if (jj < j1) z_out[jj * ldz + c] = v[u];
            }
        }
    }
    if (blockIdx.y == 0 && rl == 0) {
        lambda_out[c] = cs.lam[c];
        const int32_t st = cs.state[c];
        status_out[c] = (st == COL_ACTIVE) ? IPT_NOT_CONVERGED : st;
        if (ci_sweeps) ci_sweeps[c] = cs.sweeps[c];
        if (ci_step) ci_step[c] = cs.step[c];
        if (ci_resid) ci_resid[c] = cs.resid[c];
    }
}

// Transposed shadow of the split iterate for a low-precision or FP32 sweep:
// zt[c][j] = lowp(scale * (Z_jc - [j == i])).  Only Z - E goes through low
// precision; Delta E is added back exactly in FP64 by the GEMM epilogue.  The
// element type follows the precision the ladder chose for this sweep (nothing is
// done for an FP64 sweep).  64 x 64 tiles transposed through LDS: 16-byte loads along
// the rows of Z (a thread keeps two columns, whose idx and state it reads once), and
// each thread stores 8 consecutive rows of one column of the shadow at once.
template <typename T>
__device__ __forceinline__ void cast_z_store(double (*tile)[65], T *zt, int64_t ldt, int64_t c0, int64_t j0,
                                             T *zlo) {
    typedef T t8_t __attribute__((ext_vector_type(8)));
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        const int u = threadIdx.x + 256 * w, cc = u >> 3, r0 = 8 * (u & 7);
        t8_t h, l;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const double x = tile[r0 + e][cc];
            h[e] = to_low<T>(x);
            if (zlo) l[e] = to_low<T>(x - (double)h[e]);
        }
        const int64_t o = (c0 + cc) * ldt + j0 + r0;
        *(t8_t *)(zt + o) = h;
        if (zlo) *(t8_t *)(zlo + o) = l;
    }
}

__global__ __launch_bounds__(256) void k_cast_z(const Ctrl *ctrl, const double *zin, int64_t ldzb, ColState cs,
                                                void *zt, int64_t ldt, int64_t kp, int32_t low_type, int32_t mid_x3) {
    if (ctrl->error || ctrl->done) return;
    const int32_t prec = ctrl->prec;
    if (prec != PREC_LOW && prec != PREC_F32) return;
    const bool x3 = prec == PREC_F32 && mid_x3;
    const bool f16 = (prec == PREC_LOW && low_type == LT_F16) || x3;
    const double scale = f16 ? ctrl->zscale : 1.0;
    __shared__ double tile[64][65];
    const int64_t j0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int cp = threadIdx.x & 31, ry = threadIdx.x >> 5;
    const int64_t ca = c0 + 2 * cp;
    const int64_t ia = cs.state[ca] != COL_PAD ? cs.idx[ca] : -1;
    const int64_t ib = cs.state[ca + 1] != COL_PAD ? cs.idx[ca + 1] : -1;
    double2 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = *(const double2 *)(zin + (j0 + ry + 8 * q) * ldzb + ca);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int r = ry + 8 * q;
        const int64_t j = j0 + r;
        tile[r][2 * cp] = (j == ia ? v[q].x - 1.0 : v[q].x) * scale;
        tile[r][2 * cp + 1] = (j == ib ? v[q].y - 1.0 : v[q].y) * scale;
    }
    __syncthreads();
    if (x3) {  // hi/lo FP16 halves (kp x ldt each)
        _Float16 *zh = (_Float16 *)zt;
        cast_z_store<_Float16>(tile, zh, ldt, c0, j0, zh + kp * ldt);
    } else if (prec == PREC_F32) {
        cast_z_store<float>(tile, (float *)zt, ldt, c0, j0, nullptr);
    } else if (f16) {
        cast_z_store<_Float16>(tile, (_Float16 *)zt, ldt, c0, j0, nullptr);
    } else {
        cast_z_store<__bf16>(tile, (__bf16 *)zt, ldt, c0, j0, nullptr);
    }
}

inline int blocks_for(int64_t count, int per) { return (int)((count + per - 1) / per); }

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_init(hipStream_t s, Ctrl *ctrl, ColState cs, const int32_t *idx_user, int64_t n, int64_t k,
                       int64_t kp, uint32_t *bitmap, int32_t start_prec, int32_t ntiles_n, int32_t start_stamp,
                       const double *theta, double cont_alpha) {
    k_ctrl_init<<<1, 256, 0, s>>>(ctrl, start_prec, k, 0, cont_alpha, bitmap, (n + 31) / 32);
    return launch_init_cols(s, ctrl, cs, idx_user, n, k, kp, bitmap, ntiles_n, start_stamp, true, theta);
}

hipError_t launch_init_cols(hipStream_t s, Ctrl *ctrl, ColState cs, const int32_t *idx_user, int64_t n, int64_t k,
                            int64_t kp, uint32_t *bitmap, int32_t ntiles_n, int32_t start_stamp, bool bitmap_zeroed,
                            const double *theta) {
    const int64_t words = (n + 31) / 32;
    if (!bitmap_zeroed)
        k_fill_u32<<<blocks_for(words, 256) < 1024 ? blocks_for(words, 256) : 1024, 256, 0, s>>>(bitmap, words, 0u);
    int64_t m = kp > ntiles_n ? kp : ntiles_n;
    // theta's order check strides over the grid: one element per thread up to n = 2^20
    if (theta && m < n) m = n < (int64_t(1) << 20) ? n : (int64_t(1) << 20);
    k_init_cols<<<blocks_for(m, 256), 256, 0, s>>>(ctrl, cs, idx_user, n, k, kp, bitmap, ntiles_n, start_stamp,
                                                   theta);
    return hipGetLastError();
}

hipError_t launch_plan_dense(hipStream_t s, Ctrl *ctrl, ColState cs, int64_t kp) {
    k_plan_dense<<<1, 1024, 0, s>>>(ctrl, cs, kp);
    return hipGetLastError();
}

hipError_t launch_ctrl_init(hipStream_t s, Ctrl *ctrl, int32_t start_prec, int64_t active, int32_t sym0,
                            double cont_alpha, uint32_t *bitmap, int64_t n_bits) {
    k_ctrl_init<<<1, 256, 0, s>>>(ctrl, start_prec, active, sym0, cont_alpha, bitmap, bitmap ? (n_bits + 31) / 32 : 0);
    return hipGetLastError();
}

hipError_t launch_scan_delta(hipStream_t s, Ctrl *ctrl, const double *delta, int64_t lda, int64_t n, int64_t np,
                             int32_t want_sym, _Float16 *f16, _Float16 *hi) {
    const int64_t nb = np / 64;
    k_scan_delta<<<(unsigned)(nb * (nb + 1) / 2), 256, 0, s>>>(ctrl, delta, lda, n, np, nb, want_sym, f16, hi);
    return hipGetLastError();
}

hipError_t launch_check_theta(hipStream_t s, Ctrl *ctrl, const double *theta, const int32_t *idx, int64_t n,
                              int64_t k, bool order_done) {
    const int ob = blocks_for(n, 256) < 256 ? blocks_for(n, 256) : 256;
    if (!order_done) k_theta_order<<<ob, 256, 0, s>>>(ctrl, theta, n);
    dim3 g(blocks_for(n, 256), blocks_for(k, 256));
    k_check_theta<<<g, 256, 0, s>>>(ctrl, theta, idx, n, k);
    return hipGetLastError();
}

int64_t prep_delta_chunks(int64_t np) { return (np + PREP_ROWS - 1) / PREP_ROWS; }
int64_t prep_delta_blocks(int64_t np) { return ((np + 255) / 256) * prep_delta_chunks(np); }

hipError_t launch_prep_delta(hipStream_t s, Ctrl *ctrl, const double *theta, const double *delta, int64_t lda,
                             int64_t n, int64_t np, double *dpad, __bf16 *dlo, float *d32, double *colpart,
                             uint64_t *bmax) {
    const int64_t chunks = prep_delta_chunks(np);
    dim3 g((unsigned)((np + 255) / 256), (unsigned)chunks);
    k_prep_delta<__bf16><<<g, 256, 0, s>>>(ctrl, theta, delta, lda, n, np, dpad, dlo, d32, colpart, bmax);
    if (colpart) k_norm1_reduce<<<blocks_for(n, 256), 256, 0, s>>>(ctrl, colpart, n, chunks);
    if (bmax) k_set_dscale<<<1, 256, 0, s>>>(ctrl, bmax, prep_delta_blocks(np));
    return hipGetLastError();
}

// Debug-mode guard bands: nb bands of `words` 64-bit words at byte offsets list[b] from
// base.  Fill writes the pattern (and resets the damage word to "none"); check records
// the lowest band index that holds anything else.  One block per band.
constexpr uint64_t GUARD_PATTERN = 0x7ff4a5a55a5aa5a5ull;  // a signalling-NaN bit pattern

__global__ __launch_bounds__(256) void k_guard_fill(char *base, const uint64_t *list, int64_t words,
                                                    int32_t *damage) {
    uint64_t *g = (uint64_t *)(base + list[blockIdx.x]);
    for (int64_t w = threadIdx.x; w < words; w += 256) g[w] = GUARD_PATTERN;
    if (blockIdx.x == 0 && threadIdx.x == 0) *damage = INT32_MAX;
}

__global__ __launch_bounds__(256) void k_guard_check(const char *base, const uint64_t *list, int64_t words,
                                                     int32_t *damage) {
    const uint64_t *g = (const uint64_t *)(base + list[blockIdx.x]);
    bool bad = false;
    for (int64_t w = threadIdx.x; w < words; w += 256) bad |= g[w] != GUARD_PATTERN;
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicMin(damage, (int32_t)blockIdx.x);
}

hipError_t launch_guard_fill(hipStream_t s, char *base, const uint64_t *list, int64_t nb, int64_t words,
                             int32_t *damage) {
    if (nb < 1) return hipSuccess;
    k_guard_fill<<<(unsigned)nb, 256, 0, s>>>(base, list, words, damage);
    return hipGetLastError();
}

hipError_t launch_guard_check(hipStream_t s, const char *base, const uint64_t *list, int64_t nb, int64_t words,
                              int32_t *damage) {
    if (nb < 1) return hipSuccess;
    k_guard_check<<<(unsigned)nb, 256, 0, s>>>(base, list, words, damage);
    return hipGetLastError();
}

hipError_t launch_fill_f32(hipStream_t s, float *p, int64_t count) {
    k_fill_u32<<<blocks_for(count, 256) < 4096 ? blocks_for(count, 256) : 4096, 256, 0, s>>>((uint32_t *)p, count, 0u);
    return hipGetLastError();
}

int64_t norm1_csr_scratch_doubles(int64_t n) { return n + CSR_SUM_BLOCKS + 2; }

hipError_t launch_norm1_csr(hipStream_t s, Ctrl *ctrl, const double *theta, const int32_t *row_ptr,
                            const int32_t *col, const double *val, int64_t n, int64_t nnz, double *scratch,
                            const double *theta_im) {
    const int32_t cplx = theta_im != nullptr;
    uint64_t *acc = (uint64_t *)scratch;
    double *part = scratch + n, *scale = part + CSR_SUM_BLOCKS;
    const int64_t work = nnz > n ? nnz : n;
    int nb = blocks_for(work, 256);
    nb = nb < 1 ? 1 : (nb > CSR_SUM_BLOCKS ? CSR_SUM_BLOCKS : nb);
    k_csr_abs_sum<<<nb, 256, 0, s>>>(ctrl, val, nnz, acc, n, part, cplx);
    k_csr_abs_scale<<<1, 256, 0, s>>>(ctrl, part, nb, scale);
    k_csr_colsum<<<blocks_for(n, 256), 256, 0, s>>>(ctrl, row_ptr, col, val, n, scale, acc, cplx);
    k_norm1_csr_reduce<<<blocks_for(n, 256) < 512 ? blocks_for(n, 256) : 512, 256, 0, s>>>(ctrl, theta, row_ptr, col,
                                                                                         val, acc, scale, n, theta_im);
    return hipGetLastError();
}

hipError_t launch_load_z0(hipStream_t s, Ctrl *ctrl, const double *z0, int64_t ldz0, double *zb, int64_t ldzb,
                          const int32_t *idx, int64_t n, int64_t np, int64_t k, int64_t kp, int32_t set_zscale) {
    int b = blocks_for(np * kp, 256);
    if (b > 8192) b = 8192;
    k_load_z0<<<b, 256, 0, s>>>(ctrl, z0, ldz0, zb, ldzb, idx, n, np, k, kp, set_zscale);
    if (set_zscale) k_set_zscale<<<1, 1, 0, s>>>(ctrl);
    return hipGetLastError();
}

hipError_t launch_zero_pad(hipStream_t s, double *zb, int64_t ldzb, int64_t n, int64_t np, int64_t k, int64_t kp) {
    int b = blocks_for(np * kp, 256);
    if (b > 8192) b = 8192;
    k_zero_pad<<<b, 256, 0, s>>>(zb, ldzb, n, np, k, kp);
    return hipGetLastError();
}

hipError_t launch_sweep1_dense(hipStream_t s, const Ctrl *ctrl, const double *theta, const double *delta, int64_t lda,
                               ColState cs, double *dvec, double *zout, int64_t ldzb, double *part, int64_t n,
                               int64_t np, int64_t kp, double *dnp) {
    dim3 g((unsigned)(kp / 64), (unsigned)(np / TILE_M));
    k_sweep1_dense<<<g, 256, 0, s>>>(ctrl, theta, delta, lda, cs, dvec, zout, ldzb, part, n, kp, dnp);
    return hipGetLastError();
}

hipError_t launch_diag_dense(hipStream_t s, const Ctrl *ctrl, const double *delta, int64_t lda, const double *zin,
                             int64_t ldzb, ColState cs, double *dnp, double *dvec, int64_t n, int64_t kp) {
    const int64_t nrt = (n + TILE_M - 1) / TILE_M;
    dim3 g((unsigned)(kp / 64), (unsigned)nrt);
    k_diag_tiles<<<g, 256, 0, s>>>(ctrl, delta, lda, zin, ldzb, cs, dnp, n, kp);
    k_diag_reduce<<<(unsigned)(kp / 64), 256, 0, s>>>(ctrl, cs, dnp, dvec, nrt, kp);
    return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t s, Ctrl *ctrl, const DevOpts &o, ColState cs, double *dvec,
                           const double *theta, const double *part, int64_t nrt, int64_t kp, int32_t sweep,
                           int32_t in_par, int32_t out_par, const double *dnp, const double *theta_im,
                           const double *dvec_im, double *lam_im) {
    k_finalize<<<(unsigned)(kp / 64), 256, 0, s>>>(ctrl, o, cs, dvec, theta, part, nrt, kp, sweep, in_par, out_par,
                                                     dnp, theta_im, dvec_im, lam_im);
    return hipGetLastError();
}

hipError_t launch_control_plan(hipStream_t s, Ctrl *ctrl, const DevOpts &o, int32_t sweep, ColState cs, int64_t kp) {
    k_control_plan<<<1, 1024, 0, s>>>(ctrl, o, sweep, cs, kp);
    return hipGetLastError();
}

hipError_t launch_csr_tail(hipStream_t s, Ctrl *ctrl, const DevOpts &o, ColState cs, double *dvec,
                           const double *theta, double *part, int64_t nblk, int64_t k, int64_t kpc, int32_t sweep,
                           int32_t in_par, int32_t out_par, const int32_t *row_ptr, const int32_t *col,
                           const double *val, const double *zout, int64_t ldz) {
    if (hipError_t e = launch_reduce_parts(s, ctrl, cs, part, nblk, k, kpc)) return e;
    k_csr_tail<<<1, 256, 0, s>>>(ctrl, o, cs, dvec, theta, part, kpc, sweep, in_par, out_par, row_ptr, col, val, zout,
                                 ldz, k);
    return hipGetLastError();
}

hipError_t launch_control(hipStream_t s, Ctrl *ctrl, const DevOpts &o, int32_t sweep) {
    k_control<<<1, 1, 0, s>>>(ctrl, o, sweep);
    return hipGetLastError();
}

hipError_t launch_copyout(hipStream_t s, const Ctrl *ctrl, ColState cs, const double *buf0, const double *buf1,
                          int64_t ldzb, double *z_out, int64_t ldz, double *lambda_out, int32_t *status_out, int64_t n,
                          int64_t k, const ipt_colinfo *ci, bool only_if_done) {
    const int gy = blocks_for(n, 64) < 65535 ? blocks_for(n, 64) : 65535;
    int32_t cw = 1;
    while (cw < 256 && cw < k) cw <<= 1;
    dim3 g(blocks_for(k, cw), gy);
    k_copyout<<<g, 256, 0, s>>>(ctrl, cs, buf0, buf1, ldzb, z_out, ldz, lambda_out, status_out, n, k, cw,
                                ci ? ci->sweeps : nullptr, ci ? ci->step : nullptr, ci ? ci->resid : nullptr,
                                only_if_done ? 1 : 0);
    return hipGetLastError();
}


// Continuation sweep: W <- E + s (W - E) on this sweep's active columns (packed list
// of the plan that launched it), rows j != i; block = 64 columns x 4 row lanes.
__global__ __launch_bounds__(256) void k_cont_blend(const Ctrl *ctrl, double *w, int64_t ldw, ColState cs,
                                                    int64_t n) {
    if (ctrl->error || ctrl->done) return;
    const double es = ctrl->escale;
    if (!(es < 1.0)) return;
    const int64_t p = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    if (p >= ctrl->kact) return;
    const int32_t c = cs.alist[p];
    const int32_t i = cs.idx[c];
    for (int64_t j = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); j < n; j += (int64_t)gridDim.y * 4)
        if (j != i) w[j * ldw + c] *= es;
}

// The same blend for solves without a packed list (CSR): the columns still active in
// this sweep (their state is not yet updated by the finalize), block = 64 columns x 4
// row lanes.
__global__ __launch_bounds__(256) void k_cont_blend_cols(const Ctrl *ctrl, double *w, int64_t ldw, ColState cs,
                                                         int64_t n, int64_t k) {
    if (ctrl->error || ctrl->done) return;
    const double es = ctrl->escale;
    if (!(es < 1.0)) return;
    const int64_t c = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    if (c >= k || cs.state[c] != COL_ACTIVE) return;
    const int32_t i = cs.idx[c];
    for (int64_t j = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); j < n; j += (int64_t)gridDim.y * 4)
        if (j != i) w[j * ldw + c] *= es;
}

hipError_t launch_cont_blend_cols(hipStream_t s, const Ctrl *ctrl, double *w, int64_t ldw, ColState cs, int64_t n,
                                  int64_t k) {
    const int64_t rows = (n + 3) / 4;
    dim3 g((unsigned)((k + 63) / 64), (unsigned)(rows < 1024 ? rows : 1024));
    k_cont_blend_cols<<<g, 256, 0, s>>>(ctrl, w, ldw, cs, n, k);
    return hipGetLastError();
}

hipError_t launch_cont_blend(hipStream_t s, const Ctrl *ctrl, double *w, int64_t ldw, ColState cs, int64_t n,
                             int64_t kp) {
    const int64_t rows = (n + 3) / 4;
    dim3 g((unsigned)((kp + 63) / 64), (unsigned)(rows < 64 ? rows : 64));
    k_cont_blend<<<g, 256, 0, s>>>(ctrl, w, ldw, cs, n);
    return hipGetLastError();
}

// dst = scale * Delta (n x n, leading dimension n), one product per entry.
__global__ void k_scale_copy(double *dst, const double *src, int64_t lda, int64_t n, double scale) {
    const int64_t total = n * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / n, l = e - j * n;
        dst[e] = scale * src[j * lda + l];
    }
}

hipError_t launch_scale_copy(hipStream_t s, double *dst, const double *src, int64_t lda, int64_t n, double scale) {
    int b = blocks_for(n * n, 256);
    if (b > 8192) b = 8192;
    k_scale_copy<<<b, 256, 0, s>>>(dst, src, lda, n, scale);
    return hipGetLastError();
}

hipError_t launch_cast_z(hipStream_t s, const Ctrl *ctrl, const double *zin, int64_t ldzb, ColState cs, void *zt,
                         int64_t ldt, int64_t np, int64_t kp, int32_t low_type, int32_t mid_x3) {
    dim3 g((unsigned)(kp / 64), (unsigned)(np / 64));
    k_cast_z<<<g, 256, 0, s>>>(ctrl, zin, ldzb, cs, zt, ldt, kp, low_type, mid_x3);
    return hipGetLastError();
}

}  // namespace ipt
