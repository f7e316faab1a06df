// Sparse sweep: Y = Delta Z with Delta in CSR form (few eigenpairs of a sparse
// near-diagonal M), with the IPT update fused into the same kernel:
//   W_jc = (Z_jc d_c - Y_jc) / (theta_j - theta_i)  (j != i),  W_ic = 1      (eq. dyn)
// and the per-column partial sums of |W - Z|^2, |Z|^2, |(theta_j - theta_i)(W - Z)|^2 and
// |W - e_i|^2 over each block of rows.
//
// Layout: Z is row-major n x ldz (ldz = k rounded up to 2), so the k entries of a
// gathered row Z[col[p], :] are contiguous.  kg lanes serve one row (kg = k rounded
// up to a power of two, at most 64); a wave walks 64/kg rows at a time, each lane
// owning one column (columns c, c + 64, ... when k > 64).  The col/val entries of a
// row are broadcast to its kg lanes.
//
// FP32 sweeps of the precision ladder read an FP32 copy of val and the FP32 shadow
// of Z - E; Delta E is added exactly in FP64 (the lane meets entry (j, idx[c]) while
// walking row j).  Every sweep writes the FP32 shadow of W - E for the next one.
//
// The first sweep of a cold start (unit_in) needs no product: Z = E, so Y = Delta E is
// the entries (j, idx[c]) that the lanes meet while walking their rows (no gathers), and
// d_c = Delta_ii comes from row i itself (eq. dyn at Z = I: F(I) = I - G o Delta).
#include <math.h>

#include "ipt_internal.h"

namespace ipt {

namespace {

constexpr int UNIT_UP = 4;   // passes of the product-free sweep whose loads go out together
constexpr int SP_ROWS = 64;  // rows per block (one partial-sum row tile before the block reduction)

struct SpArgs {
    const int32_t *row_ptr;
    const int32_t *col;
    const double *val;
    const float *val32;   // FP32 copy of val (ladder only)
    const double *theta;
    const double *zin;
    double *zout;
    const float *zlo_in;  // FP32 shadow of Z - E (ladder only)
    float *zlo_out;       // FP32 shadow of W - E (ladder only)
    ColState cs;
    double *dvec;         // read (d of this sweep), or written by a unit_in sweep
    double *part;
    int64_t n, k, ldz, kpc;
    int32_t kg;           // lanes per row
    int32_t unit_in;      // Z = E (the product-free first sweep)
};

// Entries of a row whose gathers are issued together.  The kernel is bound by the
// latency of its loads, so its occupancy matters most: four (64 VGPRs, 8 waves per
// SIMD) ran faster than 8 or 16 with the operands staged in LDS (more registers, half
// the waves), and faster than 16 rows per block (fixed latency per block dominated).
constexpr int SP_GATHER = 4;

__global__ __launch_bounds__(256) void k_spmm_sweep(const Ctrl *ctrl, SpArgs a) {
    if (ctrl->error || ctrl->done) return;
    const bool f32 = ctrl->prec == PREC_F32;
    __shared__ double red[4][64][NPART];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int kg = a.kg;
    const int rows_per_pass = 64 / kg;
    const int sub = lane / kg;     // which row of the pass this lane serves
    const int cl = lane % kg;      // column slot
    const int64_t r0 = (int64_t)blockIdx.x * SP_ROWS;
    int64_t r1 = r0 + SP_ROWS;
    if (r1 > a.n) r1 = a.n;
    // columns handled by this lane: cl, cl + 64, ... (kg == 64 when k > 64)
    for (int64_t c0 = 0; c0 < a.k; c0 += 64) {
        const int64_t c = c0 + cl;
        const bool colok = c < a.k && a.cs.state[c] == COL_ACTIVE;
        const int32_t i = colok ? a.cs.idx[c] : 0;
        const double ti = a.theta[i];
        const double d = colok ? a.dvec[c] : 0.0;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        // waves take interleaved passes of rows_per_pass rows
        for (int64_t jb = r0 + (int64_t)wv * rows_per_pass; jb < r1; jb += 4 * rows_per_pass) {
            const int64_t j = jb + sub;
            if (j >= r1 || !colok) continue;
            const int32_t pb = a.row_ptr[j], pe = a.row_ptr[j + 1];
            // the epilogue's loads of row j, issued before the walk so they overlap it
            const double z = a.zin[j * a.ldz + c];
            const double tj = a.theta[j];
            double y = 0.0, ye = 0.0;
            float y32 = 0.f;
            // Entries are taken SP_GATHER at a time so that their gathers of Z rows are in
            // flight together (a lane past the row's end re-reads row j, and its term is
            // skipped); the sum still runs in storage order.
            if (!f32) {
                for (int32_t p = pb; p < pe; p += SP_GATHER) {
                    int32_t cq[SP_GATHER];
                    double vq[SP_GATHER], zq[SP_GATHER];
#pragma unroll
                    for (int u = 0; u < SP_GATHER; ++u) {
                        const bool in = p + u < pe;
                        cq[u] = in ? a.col[p + u] : (int32_t)j;
                        vq[u] = in ? a.val[p + u] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < SP_GATHER; ++u) zq[u] = a.zin[(int64_t)cq[u] * a.ldz + c];
#pragma unroll
                    for (int u = 0; u < SP_GATHER; ++u)
                        if (p + u < pe) y += vq[u] * zq[u];
                }
            } else {
                for (int32_t p = pb; p < pe; p += SP_GATHER) {
                    int32_t cq[SP_GATHER];
                    float vq[SP_GATHER], zq[SP_GATHER];
#pragma unroll
                    for (int u = 0; u < SP_GATHER; ++u) {
                        const bool in = p + u < pe;
                        cq[u] = in ? a.col[p + u] : (int32_t)j;
                        vq[u] = in ? a.val32[p + u] : 0.f;
                    }
#pragma unroll
                    for (int u = 0; u < SP_GATHER; ++u) zq[u] = a.zlo_in[(int64_t)cq[u] * a.ldz + c];
#pragma unroll
                    for (int u = 0; u < SP_GATHER; ++u)
                        if (p + u < pe) {
                            y32 += vq[u] * zq[u];
                            if (cq[u] == i) ye += a.val[p + u];
                        }
                }
                y = ye + (double)y32;
            }
            double w, st, gs, de;
            if (j == i) {
                w = 1.0;
                st = w - z;
                gs = 0.0;
                de = 0.0;
            } else {
                const double gap = tj - ti;
                w = (z * d - y) / gap;
                st = w - z;
                gs = gap * st;
                de = w;
            }
            a.zout[j * a.ldz + c] = w;
            if (a.zlo_out) a.zlo_out[j * a.ldz + c] = (float)(j == i ? 0.0 : w);
            s0 += st * st;
            s1 += z * z;
            s2 += gs * gs;
            s3 += de * de;
        }
        // reduce the rows_per_pass lanes of each column (fixed xor pattern), then the
        // 4 waves in order
        for (int off = kg; off < 64; off <<= 1) {
            s0 += __shfl_xor(s0, off);
            s1 += __shfl_xor(s1, off);
            s2 += __shfl_xor(s2, off);
            s3 += __shfl_xor(s3, off);
        }
        if (lane < kg) {
            red[wv][lane][0] = s0;
            red[wv][lane][1] = s1;
            red[wv][lane][2] = s2;
            red[wv][lane][3] = s3;
        }
        __syncthreads();
        if (threadIdx.x < kg) {
            const int t = threadIdx.x;
            const int64_t cc = c0 + t;
            if (cc < a.k) {  // partial rows of k columns: [block][k][NPART]
#pragma unroll
                for (int q = 0; q < NPART; ++q)
                    a.part[((int64_t)blockIdx.x * a.k + cc) * NPART + q] =
                        ((red[0][t][q] + red[1][t][q]) + red[2][t][q]) + red[3][t][q];
            }
        }
        __syncthreads();
    }
}

// The product-free first sweep of a cold start (Z = E): per row j and column c,
// y = sum of the entries (j, i = idx[c]) in storage order (Delta E, no gathers), W from
// the fused update with z = [j == i], and d_c = Delta_ii written by the lane of row i.
// Same lane layout and partial sums as k_spmm_sweep; a kernel of its own so that the
// product kernel keeps its register budget.
__global__ __launch_bounds__(256) void k_spmm_unit(const Ctrl *ctrl, SpArgs a) {
    if (ctrl->error || ctrl->done) return;
    __shared__ double red[4][64][NPART];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int kg = a.kg;
    const int rows_per_pass = 64 / kg;
    const int sub = lane / kg, cl = lane % kg, g0 = sub * kg;  // g0: first lane of the row's group
    const int64_t r0 = (int64_t)blockIdx.x * SP_ROWS;
    int64_t r1 = r0 + SP_ROWS;
    if (r1 > a.n) r1 = a.n;
    for (int64_t c0 = 0; c0 < a.k; c0 += 64) {
        const int64_t c = c0 + cl;
        const bool colok = c < a.k && a.cs.state[c] == COL_ACTIVE;
        const int32_t i = colok ? a.cs.idx[c] : 0;
        const double ti = a.theta[i];
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        // UNIT_UP passes of the wave at a time: their row pointers, then the first kg
        // entries of each of their rows (lane cl of a row's group loads entry pb + cl), are
        // loaded together, so a wave waits for two rounds of loads per UNIT_UP passes
        // instead of one per pointer and per eight entries; every lane of the group then
        // scans the row's entries in storage order through shuffles within the group.
        const int64_t pstep = 4 * rows_per_pass;
        for (int64_t jb = r0 + (int64_t)wv * rows_per_pass; jb < r1; jb += UNIT_UP * pstep) {
            int64_t jq[UNIT_UP];
            int32_t pb[UNIT_UP], pe[UNIT_UP], ce[UNIT_UP];
            double ve[UNIT_UP], tq[UNIT_UP];
#pragma unroll
            for (int q = 0; q < UNIT_UP; ++q) {
                jq[q] = jb + q * pstep + sub;
                const bool rin = jq[q] < r1;
                pb[q] = rin ? a.row_ptr[jq[q]] : 0;
                pe[q] = rin ? a.row_ptr[jq[q] + 1] : 0;
                tq[q] = rin ? a.theta[jq[q]] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < UNIT_UP; ++q) {
                const bool in = pb[q] + cl < pe[q];
                ce[q] = in ? a.col[pb[q] + cl] : -1;
                ve[q] = in ? a.val[pb[q] + cl] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < UNIT_UP; ++q) {
                // all lanes of the group take part in the shuffles (the group shares the row)
                double y = 0.0;
                for (int32_t p0 = pb[q]; p0 < pe[q]; p0 += kg) {
                    int32_t cv = ce[q];
                    double vv = ve[q];
                    if (p0 != pb[q]) {
                        const bool in = p0 + cl < pe[q];
                        cv = in ? a.col[p0 + cl] : -1;
                        vv = in ? a.val[p0 + cl] : 0.0;
                    }
                    const int nin = pe[q] - p0 < kg ? pe[q] - p0 : kg;
                    for (int u = 0; u < nin; ++u) {
                        const int32_t cu = __shfl(cv, g0 + u);
                        const double vu = __shfl(vv, g0 + u);
                        if (cu == i) y += vu;
                    }
                }
                const int64_t j = jq[q];
                if (j >= r1 || !colok) continue;
                const double tj = tq[q];
                double w, st, gs, de;
                if (j == i) {
                    a.dvec[c] = y;  // d_c = Delta_ii for this sweep's finalize
                    w = 1.0;
                    st = 0.0;
                    gs = 0.0;
                    de = 0.0;
                } else {
                    const double gap = tj - ti;
                    w = -y / gap;  // (z d - y) / gap with z = 0
                    st = w;
                    gs = gap * st;
                    de = w;
                }
                a.zout[j * a.ldz + c] = w;
                if (a.zlo_out) a.zlo_out[j * a.ldz + c] = (float)(j == i ? 0.0 : w);
                s0 += st * st;
                s1 += (j == i) ? 1.0 : 0.0;
                s2 += gs * gs;
                s3 += de * de;
            }
        }
        for (int off = kg; off < 64; off <<= 1) {
            s0 += __shfl_xor(s0, off);
            s1 += __shfl_xor(s1, off);
            s2 += __shfl_xor(s2, off);
            s3 += __shfl_xor(s3, off);
        }
        if (lane < kg) {
            red[wv][lane][0] = s0;
            red[wv][lane][1] = s1;
            red[wv][lane][2] = s2;
            red[wv][lane][3] = s3;
        }
        __syncthreads();
        if (threadIdx.x < kg) {
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
}

// Second level of the per-column reduction: part[0][c][q] <- sum over all row blocks
// of part[blk][c][q].  Block per (column, quantity); thread t adds blocks t, t + 256,
// ... in order, then a fixed tree over the 256 threads.
__global__ __launch_bounds__(256) void k_reduce_parts(const Ctrl *ctrl, const ColState cs, double *part, int64_t nblk,
                                                      int64_t ldp) {
    if (ctrl->error || ctrl->done) return;
    __shared__ double sh[256];
    const int64_t c = blockIdx.x >> 2;
    const int q = blockIdx.x & 3;
    if (cs.state[c] != COL_ACTIVE) return;
    double acc = 0.0;
    for (int64_t b = threadIdx.x; b < nblk; b += 256) acc += part[(b * ldp + c) * NPART + q];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[c * NPART + q] = sh[0];
}

// d_c = (Delta Z)_{i,c} = sum over row i of val[p] Z[col[p], c], FP64, one wave per
// column: lane-strided partial sums then a fixed xor tree.
__global__ void k_diag_csr(const Ctrl *ctrl, const int32_t *row_ptr, const int32_t *col, const double *val,
                           const double *zin, int64_t ldz, ColState cs, double *dvec, int64_t k) {
    if (ctrl->error || ctrl->done) return;
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= k || cs.state[c] != COL_ACTIVE) return;
    const int32_t i = cs.idx[c];
    double acc = 0.0;
    for (int32_t p = row_ptr[i] + lane; p < row_ptr[i + 1]; p += 64) acc += val[p] * zin[(int64_t)col[p] * ldz + c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) dvec[c] = acc;
}

// CSR structure checks: row_ptr[0] == 0, non-decreasing, row_ptr[n] == nnz, and
// every column index in [0, n).  With val32, the FP32 copy of val in the same pass.
__global__ void k_check_csr(Ctrl *ctrl, const int32_t *row_ptr, const int32_t *col, int64_t n, int64_t nnz,
                            const double *val, float *val32) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool bad = false;
    if (t == 0) bad |= row_ptr[0] != 0 || (int64_t)row_ptr[n] != nnz;
    if (t < n) bad |= row_ptr[t + 1] < row_ptr[t];
    for (int64_t p = t; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
        bad |= col[p] < 0 || (int64_t)col[p] >= n;
        if (val32) val32[p] = (float)val[p];
    }
    if (bad) atomicMax(&ctrl->error, (int32_t)IPT_EINVAL);
}

// FP32 shadow of Z0 - E for a warm start (zero elsewhere).
__global__ void k_zlo_init(const double *zb, float *zlo, int64_t ldz, const int32_t *idx, int64_t n, int64_t k) {
    const int64_t total = n * ldz;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / ldz, c = e - j * ldz;
        const double v = (c < k) ? zb[e] - (j == idx[c] ? 1.0 : 0.0) : 0.0;
        zlo[e] = (float)v;
    }
}

inline int blocks_for(int64_t count, int per) { return (int)((count + per - 1) / per); }

}  // namespace

int64_t spmm_row_tiles(int64_t n) { return (n + SP_ROWS - 1) / SP_ROWS; }

hipError_t launch_reduce_parts(hipStream_t s, const Ctrl *ctrl, ColState cs, double *part, int64_t nblk, int64_t ldp,
                               int64_t kpc) {
    k_reduce_parts<<<(unsigned)(kpc * 4), 256, 0, s>>>(ctrl, cs, part, nblk, ldp);
    return hipGetLastError();
}

hipError_t launch_spmm_sweep(hipStream_t s, const Ctrl *ctrl, const int32_t *row_ptr, const int32_t *col,
                             const double *val, const float *val32, const double *theta, const double *zin,
                             double *zout, const float *zlo_in, float *zlo_out, ColState cs, double *dvec,
                             double *part, int64_t n, int64_t k, int64_t ldz, int64_t kpc, int32_t unit_in) {
    int kg = 1;
    while (kg < k && kg < 64) kg <<= 1;
    SpArgs a{row_ptr, col, val, val32, theta, zin, zout, zlo_in, zlo_out, cs, dvec, part, n, k, ldz, kpc, kg, unit_in};
    if (unit_in)
        k_spmm_unit<<<(unsigned)spmm_row_tiles(n), 256, 0, s>>>(ctrl, a);
    else
        k_spmm_sweep<<<(unsigned)spmm_row_tiles(n), 256, 0, s>>>(ctrl, a);
    return hipGetLastError();
}

hipError_t launch_diag_csr(hipStream_t s, const Ctrl *ctrl, const int32_t *row_ptr, const int32_t *col,
                           const double *val, const double *zin, int64_t ldz, ColState cs, double *dvec, int64_t k) {
    k_diag_csr<<<(unsigned)((k + 3) / 4), 256, 0, s>>>(ctrl, row_ptr, col, val, zin, ldz, cs, dvec, k);
    return hipGetLastError();
}

hipError_t launch_check_csr(hipStream_t s, Ctrl *ctrl, const int32_t *row_ptr, const int32_t *col, int64_t n,
                            int64_t nnz, const double *val, float *val32) {
    int b = blocks_for(n + 1 > nnz ? n + 1 : nnz, 256);
    if (b > 4096) b = 4096;
    if (b < blocks_for(n, 256)) b = blocks_for(n, 256);
    k_check_csr<<<b, 256, 0, s>>>(ctrl, row_ptr, col, n, nnz, val, val32);
    return hipGetLastError();
}

hipError_t launch_zlo_init(hipStream_t s, const double *zb, float *zlo, int64_t ldz, const int32_t *idx, int64_t n,
                           int64_t k) {
    int b = blocks_for(n * ldz, 256);
    if (b > 8192) b = 8192;
    k_zlo_init<<<b, 256, 0, s>>>(zb, zlo, ldz, idx, n, k);
    return hipGetLastError();
}

}  // namespace ipt
