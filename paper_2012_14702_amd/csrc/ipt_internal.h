// Internal declarations of the gfx950 IPT library: device control block, column
// states, workspace layout and the host-side launchers of every kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ipt.h"

namespace ipt {

// Column states kept on the device.  ACTIVE columns are iterated; the others are
// frozen and their final value sits in the ping-pong buffer named by col_par.
enum : int32_t { COL_ACTIVE = -1, COL_CONVERGED = IPT_CONVERGED, COL_NOT_CONVERGED = IPT_NOT_CONVERGED,
                 COL_DIVERGED = IPT_DIVERGED, COL_PAD = -2 };

// Where a frozen column's final value lives: buffer 0 or 1, or the unit vector
// e_i (a column certified by the first sweep of a cold start).
enum : int32_t { PAR_BUF0 = 0, PAR_BUF1 = 1, PAR_UNIT = 2 };

// Sweep precisions (same numbering as IPT_SWEEP_*).
enum : int32_t { PREC_EXACT_FIRST = IPT_SWEEP_EXACT_FIRST, PREC_LOW = IPT_SWEEP_LOW, PREC_F32 = IPT_SWEEP_FP32,
                 PREC_F64 = IPT_SWEEP_FP64 };

// Device control block of one solve.  Written by the setup, finalize and control
// kernels; read at the start of every sweep kernel, which returns at once when
// `done` is set or when the sweep's precision is not its own.
struct Ctrl {
    int32_t error;       // IPT_EINVAL / IPT_EDEGENERATE found by the device checks, else 0
    int32_t done;        // 1 once no column is active or max_iter sweeps ran
    int32_t prec;        // precision of the next sweep
    int32_t sweeps;      // sweeps executed
    int32_t active;      // active columns entering the next sweep
    int32_t acc_active;  // finalize accumulator: columns still active after this sweep
    int32_t n_conv, n_notconv, n_div;
    int32_t prec_mask;  // batched: bit PREC_F32 set when a tile of this sweep ran in FP32
    int32_t kact;       // dense: active columns entering the next sweep (length of ColState::alist)
    int32_t sym;        // dense: 1 once Delta is verified exactly symmetric (Delta_ji may stand for Delta_ij)
    int32_t theta_order;  // bit 0: theta not strictly increasing, bit 1: not strictly decreasing
    uint64_t acc_maxstep;  // finalize accumulator: max s_c (bit pattern of a non-negative double)
    uint64_t acc_maxres;   // max normalised eigen-residual over converged columns (bits)
    uint64_t dec_maxstep;  // max deciding step over decided columns (bits)
    uint64_t norm1_bits;   // |M|_1 (bits), set by the norm kernel
    uint64_t acc_maxdist;  // finalize accumulator: max |W_c - e_i| over active columns (bits)
    uint64_t dmax_bits;    // max |Delta_jl| (bits), set when the FP16 rung needs a scale
    double dscale;         // power-of-two scale of the low-precision Delta shadow (1 unless FP16)
    double zscale;         // power-of-two scale of the low-precision (Z - E) shadow (1 unless FP16)
    double apow;           // continuation: alpha^t of the next sweep t (0 without continuation)
    double escale;         // continuation: the next sweep's perturbation scale 1 - alpha^t (1 without)
    int64_t matvecs;
    double prev_maxstep;
    int32_t hist_prec[IPT_HIST];
    int32_t hist_active[IPT_HIST];
    double hist_step[IPT_HIST];
};

// Options as the kernels see them.
struct DevOpts {
    double tol, tau_low, tau_32, div_norm;
    double cont_alpha;      // non-autonomous continuation (0: off)
    int32_t max_iter, div_growth, ladder, low_type;
    int32_t first_product;  // the first sweep of a cold start multiplies by Delta (sparse path)
    int32_t acx;            // IPT-ACX cycles (orders 3, 2, 3, 2, ...)
    int32_t mid_x3;         // dense ladder: FP32-class rung as three FP16 products
};

// IPT-ACX schedule: sweep t (1-based) is application q (0-based) of a cycle of
// order p; the orders alternate 3, 2, so the pattern repeats every 5 sweeps.
// Without ACX every sweep is a cycle of order 1.
__host__ __device__ inline void acx_phase(int32_t acx, int32_t t, int32_t &q, int32_t &p) {
    if (!acx) {
        q = 0;
        p = 1;
        return;
    }
    const int32_t r = (t - 1) % 5;
    q = r < 3 ? r : r - 3;
    p = r < 3 ? 3 : 2;
}

// Per-column state arrays (length kp).
struct ColState {
    int32_t *state;   // COL_*
    int32_t *sweeps;  // deciding sweep
    int32_t *grow;    // consecutive FP64 sweeps with a growing step
    int32_t *par;     // PAR_* of frozen columns
    double *prev;     // previous step
    double *step;     // deciding step
    double *lam;      // lambda of the deciding sweep
    double *resid;    // normalised eigen-residual of the deciding sweep
    int32_t *idx;     // requested indices (padding columns hold 0)
    int32_t *tile_stamp;  // per column tile of width TILE_N: last sweep in which it had an active column
    int32_t *alist;       // dense: the active columns in ascending order (packed positions of the GEMM)
};

constexpr int TILE_M = 128;   // rows of Delta / Y per GEMM tile, and per partial-sum row tile
constexpr int TILE_N = 128;   // columns of Z / Y per GEMM tile
constexpr int NPART = 4;      // partial sums per (row tile, column): step^2, z^2, (gap*step)^2, |w-e|^2

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Element types of the low-precision shadows.
enum : int32_t { LT_BF16 = 0, LT_F16 = 1, LT_F32 = 2 };

// -------------------------------------------------------------- launchers

// Setup and bookkeeping (ipt_setup.hip)
// With theta, the column part also checks theta's order (as launch_init_cols);
// cont_alpha > 0 starts the continuation's scale (as launch_ctrl_init).
hipError_t launch_init(hipStream_t s, Ctrl *ctrl, ColState cs, const int32_t *idx_user, int64_t n, int64_t k,
                       int64_t kp, uint32_t *bitmap, int32_t start_prec, int32_t ntiles_n, int32_t start_stamp,
                       const double *theta = nullptr, double cont_alpha = 0.0);
// The column part of launch_init (after a separate launch_ctrl_init): bitmap_zeroed
// when that launch cleared the bitmap; with theta it also checks theta's order (then
// launch_check_theta(..., order_done = true)).  With cs.alist it writes the packed
// list of the first sweep (all k columns in order; ctrl->kact = k from the reset).
hipError_t launch_init_cols(hipStream_t s, Ctrl *ctrl, ColState cs, const int32_t *idx_user, int64_t n, int64_t k,
                            int64_t kp, uint32_t *bitmap, int32_t ntiles_n, int32_t start_stamp,
                            bool bitmap_zeroed = false, const double *theta = nullptr);
// sym0 = 1 when the symmetry scan runs next (it clears sym on the first asymmetric pair);
// bitmap (n bits) is cleared for launch_init_cols when given.
hipError_t launch_ctrl_init(hipStream_t s, Ctrl *ctrl, int32_t start_prec, int64_t active, int32_t sym0 = 0,
                            double cont_alpha = 0.0, uint32_t *bitmap = nullptr, int64_t n_bits = 0);
// dst = scale * Delta, n x n with leading dimension n (the homotopy restart's stages).
hipError_t launch_scale_copy(hipStream_t s, double *dst, const double *src, int64_t lda, int64_t n, double scale);
// Continuation sweep (scale s = Ctrl::escale < 1): the sweep computed W = F(Z) of the
// unscaled partition; the continuation map is E + s (F(Z) - E), so the off-diagonal
// entries of this sweep's active columns are multiplied by s in place.  Nothing is
// done once s = 1.  launch_cont_blend takes the columns from the packed list (dense
// solves), launch_cont_blend_cols the columns 0 .. k-1 still active (CSR solves).
hipError_t launch_cont_blend(hipStream_t s, const Ctrl *ctrl, double *w, int64_t ldw, ColState cs, int64_t n,
                             int64_t kp);
hipError_t launch_cont_blend_cols(hipStream_t s, const Ctrl *ctrl, double *w, int64_t ldw, ColState cs, int64_t n,
                                  int64_t k);
// Tile pairs of Delta over the padded np x np, after launch_prep_delta: want_sym
// clears ctrl->sym unless Delta equals its transpose bit for bit; f16 (the FP16 low
// rung) and hi (hi/lo of the three-product rung, lo = hi + np^2) receive the FP16
// shadows scaled by ctrl->dscale.
hipError_t launch_scan_delta(hipStream_t s, Ctrl *ctrl, const double *delta, int64_t lda, int64_t n, int64_t np,
                             int32_t want_sym, _Float16 *f16, _Float16 *hi);
// Dense: list the active columns in ascending order (ColState::alist, ctrl->kact).
hipError_t launch_plan_dense(hipStream_t s, Ctrl *ctrl, ColState cs, int64_t kp);
// Dense: the plan of the next sweep followed by the control step, in one launch.
hipError_t launch_control_plan(hipStream_t s, Ctrl *ctrl, const DevOpts &o, int32_t sweep, ColState cs, int64_t kp);
hipError_t launch_check_theta(hipStream_t s, Ctrl *ctrl, const double *theta, const int32_t *idx, int64_t n,
                              int64_t k, bool order_done = false);
// colpart holds prep_delta_chunks(np) x n doubles; bmax (prep_delta_blocks(np) words of
// per-block maxima of |Delta|), when given, also sets ctrl->dscale.
hipError_t launch_prep_delta(hipStream_t s, Ctrl *ctrl, const double *theta, const double *delta, int64_t lda,
                             int64_t n, int64_t np, double *dpad, __bf16 *dlo, float *d32, double *colpart,
                             uint64_t *bmax);
int64_t prep_delta_chunks(int64_t np);
int64_t prep_delta_blocks(int64_t np);
// scratch: norm1_csr_scratch_doubles(n) doubles.  With theta_im, the matrix is complex:
// theta is its real part and val holds nnz (re, im) pairs.
int64_t norm1_csr_scratch_doubles(int64_t n);
hipError_t launch_norm1_csr(hipStream_t s, Ctrl *ctrl, const double *theta, const int32_t *row_ptr,
                            const int32_t *col, const double *val, int64_t n, int64_t nnz, double *scratch,
                            const double *theta_im = nullptr);
// set_zscale: also the power-of-two scale of the FP16 shadow of Z - E from max |Z - E|
// (a warm-started ladder whose first sweep is on an FP16-shadowed rung).
hipError_t launch_load_z0(hipStream_t s, Ctrl *ctrl, const double *z0, int64_t ldz0, double *zb, int64_t ldzb,
                          const int32_t *idx, int64_t n, int64_t np, int64_t k, int64_t kp, int32_t set_zscale = 0);
hipError_t launch_zero_pad(hipStream_t s, double *zb, int64_t ldzb, int64_t n, int64_t np, int64_t k, int64_t kp);
hipError_t launch_sweep1_dense(hipStream_t s, const Ctrl *ctrl, const double *theta, const double *delta,
                               int64_t lda, ColState cs, double *dvec, double *zout, int64_t ldzb, double *part,
                               int64_t n, int64_t np, int64_t kp, double *dnp = nullptr);
// d of the sweep from Delta and its input Z, through the same row-tile partials
// (dnp: ceil(n / TILE_M) x kp) and summation order as the sweep epilogue's d.
hipError_t launch_diag_dense(hipStream_t s, const Ctrl *ctrl, const double *delta, int64_t lda, const double *zin,
                             int64_t ldzb, ColState cs, double *dnp, double *dvec, int64_t n, int64_t kp);
// dnp: NULL, or the nrt x kp partials of the next sweep's d from the sweep's
// epilogue; the finalize then writes dvec[c] = their sum for the columns that stay
// active (after reading this sweep's d).
// theta_im, dvec_im, lam_im: complex solves (theta, dvec the real parts), else NULL.
hipError_t launch_finalize(hipStream_t s, Ctrl *ctrl, const DevOpts &o, ColState cs, double *dvec,
                           const double *theta, const double *part, int64_t nrt, int64_t kp, int32_t sweep,
                           int32_t in_par, int32_t out_par, const double *dnp = nullptr,
                           const double *theta_im = nullptr, const double *dvec_im = nullptr,
                           double *lam_im = nullptr);
hipError_t launch_control(hipStream_t s, Ctrl *ctrl, const DevOpts &o, int32_t sweep);
// CSR sweep tail (plain sweeps, not IPT-ACX): the per-column sums of the SpMM's row-tile
// partials (launch_reduce_parts), then one single-block launch for the finalize of every
// column, d = (Delta W)_ic of the next sweep for the columns still active (W = zout, as
// launch_diag_csr) and the control step.
hipError_t launch_csr_tail(hipStream_t s, Ctrl *ctrl, const DevOpts &o, ColState cs, double *dvec,
                           const double *theta, double *part, int64_t nblk, int64_t k, int64_t kpc, int32_t sweep,
                           int32_t in_par, int32_t out_par, const int32_t *row_ptr, const int32_t *col,
                           const double *val, const double *zout, int64_t ldz);
// only_if_done: the kernel does nothing unless the device has set its done flag (a
// copy-out enqueued where the solve is expected to stop, before the host knows).
hipError_t launch_copyout(hipStream_t s, const Ctrl *ctrl, ColState cs, const double *buf0, const double *buf1,
                          int64_t ldzb, double *z_out, int64_t ldz, double *lambda_out, int32_t *status_out,
                          int64_t n, int64_t k, const ipt_colinfo *ci, bool only_if_done = false);
hipError_t launch_cast_z(hipStream_t s, const Ctrl *ctrl, const double *zin, int64_t ldzb, ColState cs, void *zt,
                         int64_t ldt, int64_t np, int64_t kp, int32_t low_type, int32_t mid_x3 = 0);

hipError_t launch_fill_f32(hipStream_t s, float *p, int64_t count);  // zero fill
// debug-mode workspace guard bands (nb bands of `words` 64-bit words at base + list[b])
hipError_t launch_guard_fill(hipStream_t s, char *base, const uint64_t *list, int64_t nb, int64_t words,
                             int32_t *damage);
hipError_t launch_guard_check(hipStream_t s, const char *base, const uint64_t *list, int64_t nb, int64_t words,
                              int32_t *damage);

// Sparse sweeps (ipt_spmm.hip)
int64_t spmm_row_tiles(int64_t n);
// part: [nblk][ldp][NPART] partials of the sweep; the sums land in part[c][q] (c < kpc)
hipError_t launch_reduce_parts(hipStream_t s, const Ctrl *ctrl, ColState cs, double *part, int64_t nblk, int64_t ldp,
                               int64_t kpc);
hipError_t launch_spmm_sweep(hipStream_t s, const Ctrl *ctrl, const int32_t *row_ptr, const int32_t *col,
                             const double *val, const float *val32, const double *theta, const double *zin,
                             double *zout, const float *zlo_in, float *zlo_out, ColState cs, double *dvec,
                             double *part, int64_t n, int64_t k, int64_t ldz, int64_t kpc, int32_t unit_in);
hipError_t launch_diag_csr(hipStream_t s, const Ctrl *ctrl, const int32_t *row_ptr, const int32_t *col,
                           const double *val, const double *zin, int64_t ldz, ColState cs, double *dvec, int64_t k);
// CSR structure checks; with val32 the same pass writes the FP32 copy of val.
hipError_t launch_check_csr(hipStream_t s, Ctrl *ctrl, const int32_t *row_ptr, const int32_t *col, int64_t n,
                            int64_t nnz, const double *val = nullptr, float *val32 = nullptr);
hipError_t launch_zlo_init(hipStream_t s, const double *zb, float *zlo, int64_t ldz, const int32_t *idx, int64_t n,
                           int64_t k);

// Batched solves (ipt_batched.hip).  Problem b: size n, tile size T (32, 64 or
// 128), padded size np = round_up(n, T); offsets of its Delta and theta (caller
// pools), of its output in z_pool (offo), of its padded np x np blocks in the
// workspace arrays (offz: padded Delta, both iterate buffers and their shadows), of
// its columns, its partial sums (offp, NPART per row tile and column), its
// per-row-tile d and norm partials (offq) and its column-tile flags (offf).
struct BatchMeta {
    int32_t n, T, np, xcd;  // xcd: the accelerator die whose work list holds the problem's tiles
    int64_t offd, offt, offo, offz, offc, offp, offq, offf;
};
struct BatchCols {  // per column of all problems, concatenated
    int32_t *state, *sweeps, *grow, *par, *prob;
    double *prev, *step, *lam, *resid, *d;
    double *dslot;        // IPT-ACX: [4][columns] d of each iterate slot of the running cycle
    int32_t *alist;       // per problem, its active columns in ascending order (packed positions)
    int32_t *cprec;       // precision of the tile that computes the column in the running sweep
    int32_t *want;        // precision the column asks for in the next sweep
    int32_t *kact;        // per problem: active columns (length of its alist)
    int32_t *asym;        // per problem: nonzero when Delta_b is not exactly symmetric
    uint64_t *norm_bits;  // per problem: |M_b|_1 (bits)
};
struct BatchLaunch {
    const BatchMeta *meta;
    const double *theta, *delta;  // caller pools
    double *dpad;                 // padded FP64 Delta
    float *d32;                   // padded FP32 Delta (ladder)
    double *zs[4];                // iterate slots: ping-pong in 0/1; IPT-ACX cycles use 0..3
    float *zlo0, *zlo1;           // FP32 shadows of Z - E (ladder)
    BatchCols col;
    double *part;
    double *dpart;     // [total_q] next sweep's d, one partial per (row tile, column)
    double *normpart;  // [total_q] column sums of |M_b| per row tile (first sweep)
    uint64_t *bpart;   // [finalize blocks][8] per-block batch counters
    uint32_t *tflag;   // [total column tiles] precision of each packed column tile of the next sweep
    int32_t *ncols;    // [problems][16] the columns of a problem's narrow tile (-1 past its end)
    int64_t total_tiles, total_q;
};
// Work lists of (problem, row tile, column tile, 0) items per tile class (T = 32, 64,
// 128) and sweep parity, filled by the finalize of the previous sweep.
// Work lists of the batched GEMM, per tile class and sweep parity.  Each list is cut
// into NXCD segments, one per accelerator die (XCD, with its own L2): the problems
// are dealt to the dies, a block of the persistent GEMM works through the segment
// of the die it runs on (workgroups are dispatched round-robin over the dies) and
// then helps with the others, so the tiles of one problem, which share its Delta
// and Z panels, are mostly computed under one L2.
// Classes 0..2 hold the tiles of size 32, 64 and 128; class CLS_NARROW holds the
// (last) column tiles of at most 16 columns, whatever their size.
constexpr int NXCD = 8;
constexpr int CLS_NARROW = 3, NCLS = 4;
struct BatchLists {
    int4 *l[NCLS][2];
    int32_t segcap[NCLS];  // entries per die segment in the lists of a class (segment x starts at x segcap)
    int32_t *counts;       // [NCLS][2][NXCD] items in each segment
    int32_t *tickets;      // [NCLS][NXCD] next item of the running sweep, per class and segment
};
constexpr int BLIST_COUNTS = NCLS * 2 * NXCD;                 // words of BatchLists::counts
constexpr int BLIST_WORDS = BLIST_COUNTS + NCLS * NXCD;        // counts, then tickets
int bfinalize_blocks(int64_t total_cols);
hipError_t launch_binit(hipStream_t s, Ctrl *ctrl, const BatchLaunch &L, int32_t count, int32_t start_prec);
hipError_t launch_bsweep1(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, const int4 *items, int64_t nitems,
                          int32_t ladder, int32_t acx);
hipError_t launch_bacx(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, const BatchLists &lists,
                       int64_t total_cols);
hipError_t launch_bgemm(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, const BatchLists &lists, int tile,
                        int grid, int32_t acx);
int bnarrow_grid();
hipError_t launch_bnarrow(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, const BatchLists &lists, int grid,
                         int32_t acx);
hipError_t launch_bfinalize(hipStream_t s, Ctrl *ctrl, const DevOpts &o, const BatchLaunch &L, int64_t total_cols,
                            const BatchLists &lists);
hipError_t launch_bcontrol(hipStream_t s, Ctrl *ctrl, const DevOpts &o, const BatchLaunch &L, int64_t total_cols,
                           const BatchLists &lists);
hipError_t launch_bplan(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, const BatchLists &lists, int32_t count);
hipError_t launch_bcopyout(hipStream_t s, const Ctrl *ctrl, const BatchLaunch &L, const int4 *items, int64_t nitems,
                           double *z_pool, double *lambda_pool, int32_t *status_pool, double *max_resid_out,
                           int32_t *ci_sweeps = nullptr, double *ci_step = nullptr, double *ci_resid = nullptr);
int bgemm_grid(int tile);  // persistent grid size (CUs x resident blocks)

// MLP kernels (ipt_mlp.hip).  Every matrix the GEMM reads is BF16, row-major with
// its reduction (K) dimension contiguous, zero-padded to multiples of MLP_TILE in
// both dimensions.  C[M x N] = A[M x K] B[N x K]^T, 128 x 128 tiles, then one of the
// epilogues below.
constexpr int MLP_TILE = 128;
constexpr int MLP_SLAB = 8;   // rows per block of the split-K reduction (its column sums come per slab)
enum : int {
    MLP_EPI_ACT = 0,    // + bias, optional tanh; BF16 C and C^T (zero outside mvalid x nvalid)
    MLP_EPI_MSE = 1,    // + bias; g = scale (y - t) in BF16 as C and C^T, loss and column-sum partials
    MLP_EPI_F32 = 2,    // + bias; FP32 C (valid part, leading dimension ldc32)
    MLP_EPI_GRAD = 3,   // FP32 C (valid part): a weight gradient in the parameter layout
    MLP_EPI_ADAM = 4,   // Adam on the weights from this gradient; BF16 copies W and W^T
    MLP_EPI_SPLIT = 5,  // FP32 partial tile of split-K (partial z at c32 + z M N, leading dimension N)
    MLP_EPI_WARM = 6    // + bias; warm start Z0 = E + sum_l eps^l T_l + eps^(order+1) (mu + sigma y), FP64
};
struct MlpEpi {
    int32_t mvalid, nvalid;        // rows and columns of C that are data (the rest is padding)
    const float *bias;             // [nvalid] or null
    int32_t tanh_act;
    __bf16 *c16;                   // BF16 C, leading dimension ldc16
    int64_t ldc16;
    __bf16 *ct16;                  // BF16 C^T, leading dimension ldct16
    int64_t ldct16;
    float *c32;                    // FP32 C, leading dimension ldc32
    int64_t ldc32;
    const float *tgt;              // MSE targets [mvalid x nvalid], leading dimension ldt
    const float *roww;             // MSE: per-row loss weights (null: 1)
    int64_t ldt;
    float scale;                   // MSE: 2 / (number of outputs)
    double *lossp;                 // MSE: per-block sums of (y - t)^2
    float *colp;                   // column sums of the stored BF16 C: [M/128][ldcolp] (split reduce: [M/MLP_SLAB])
    int64_t ldcolp;
    const __bf16 *h;               // split reduce: the activation H of the layer below (tanh derivative)
    int64_t ldh;
    float *w, *am, *av;            // Adam: FP32 weights and moments, parameter layout (row stride nvalid)
    const int32_t *adam_t;         // Adam: steps taken so far (device)
    float lr;
    double *z0;                    // warm start output: problem p, entry q = j kcols + c at z0 + p pstride + j ldz0 + c
    int64_t ldz0, pstride, kcols;
    const int32_t *idx;
    const float *mu, *sigma;
    const double *eps;             // [mvalid] family parameter of each problem
    const double *terms;           // order x (nvalid) analytic terms T_l (may be null when order = 0)
    int32_t order;
};
// Every hidden layer of a network whose padded widths are at most 256 in one launch
// (mlp_fused_fits): xb is the packed BF16 input (bp x ip), w[l] the BF16 W_l (loutp x
// linp), bias[l] the FP32 b_l; writes H_l (bp x hp) and H_l^T (hp x bp) as the
// bias + tanh epilogue of the GEMM path.
constexpr int MLP_MAX_LAYERS = 16;
struct MlpFused {
    const __bf16 *xb;
    int32_t ip, hp, depth;
    const __bf16 *w[MLP_MAX_LAYERS];
    const float *bias[MLP_MAX_LAYERS];
    __bf16 *hb[MLP_MAX_LAYERS], *ht[MLP_MAX_LAYERS];
    int32_t linp[MLP_MAX_LAYERS], loutp[MLP_MAX_LAYERS], lout[MLP_MAX_LAYERS];
};
bool mlp_fused_fits(int depth, const int *linp, const int *loutp);
// x null: input from the packed f.xb, H_l and H_l^T stored (training); x non-null: the
// BF16 of x [batch x in] (in <= linp[0]) read directly and H_l^T not stored (inference).
hipError_t mlp_hidden_fused(hipStream_t s, const MlpFused &f, int batch, int bp, const float *x = nullptr, int in = 0);
hipError_t mlp_gemm(hipStream_t s, int mode, const __bf16 *A, int64_t lda, const __bf16 *B, int64_t ldb, int M, int N,
                    int K, int splits, const MlpEpi &e);
// Sum of the split-K partials (FP32 [splits][M][N]) in split order, then mode
// MLP_EPI_SPLIT: times the tanh derivative (1 - h^2) of the stored activation e.h;
// MLP_EPI_ACT: + bias, tanh; MLP_EPI_ADAM: Adam on the weights; BF16 C (required), C^T
// and the column sums per MLP_SLAB rows when given.
hipError_t mlp_split_reduce(hipStream_t s, int mode, const float *part, int splits, int M, int N, const MlpEpi &e);
int mlp_split_count(int M, int N, int K);
// Padded BF16 copies W [loutp x linp] and W^T [linp x loutp] of a layer from the FP32 weights.
hipError_t mlp_pack_weights(hipStream_t s, const float *w, int lout, int lin, __bf16 *wb, __bf16 *wbt, int loutp,
                            int linp);
// Padded BF16 copies X [bp x ip] and X^T [ip x bp] of the FP32 input batch x [batch x in].
hipError_t mlp_pack_x(hipStream_t s, const float *x, int batch, int in, __bf16 *xb, __bf16 *xt, int bp, int ip);
struct MlpBiasLayers {
    int32_t count;                 // layers
    int32_t lout[17];              // bias length of each layer
    int64_t boff[17];              // offset of the bias in the parameter layout
    const float *colp[17];         // that layer's column-sum partials [mtiles][ld]
    int64_t ldcolp[17];
    int32_t mtiles[17];
};
// Bias gradients (column sums over the row tiles, in tile order); Adam on the biases
// when adam (else the gradient goes to g).
hipError_t mlp_bias_step(hipStream_t s, const MlpBiasLayers &L, int adam, float *w, float *g, float *am, float *av,
                         const int32_t *adam_t, float lr);
// Loss = sum of the per-block partials / count; with adam, the step counter advances.
hipError_t mlp_loss_step(hipStream_t s, const double *lossp, int nparts, double inv_count, float *loss,
                         int32_t *adam_t, int adam);
hipError_t mlp_targets(hipStream_t s, const double *z, int32_t batch, int64_t n, int64_t k, int64_t ldz,
                       int64_t pstride, const int32_t *idx, const double *eps, int32_t order, const double *terms,
                       const double *weights, float *targets, float *mu, float *sigma);

// Rayleigh-Schroedinger terms of M = D + Delta on requested columns (ipt_rs.hip).
// err: bit 0 = an index outside [0, n), bit 1 = theta_j == theta_i (or not finite) for a
// requested i and j != i.  rs_clear zeroes it.
hipError_t rs_clear(hipStream_t s, int32_t *err);
hipError_t rs_gather(hipStream_t s, const double *delta, int64_t lda, const int32_t *idx, int64_t n, int64_t k,
                     double *y, int32_t *err);
hipError_t rs_product(hipStream_t s, const double *delta, int64_t lda, const double *z, int64_t n, int64_t k,
                      double *y);
hipError_t rs_term(hipStream_t s, const double *theta, const int32_t *idx, const double *y, double *terms, double *d,
                   int32_t l, int64_t n, int64_t k, int32_t *err);
hipError_t rs_start(hipStream_t s, const double *eps, int32_t count, int32_t order, const double *terms, int64_t n,
                    int64_t k, const int32_t *idx, double *z0, int64_t ldz0, int64_t pstride);

// IPT-ACX extrapolation over row-major iterate slots z, f1, f2, f3 (n rows, leading
// dimension ld, kc columns with states `state`) after a cycle of order p
// (ipt_acx.hip): per-column dot and squared norm of the two highest differences in
// row-range partials, sigma, and the in-place update of z for the active columns.
int acx_splits(int64_t n, int64_t kc);  // row splits of the partial sums (workspace: splits x kc x 2)
hipError_t launch_acx(hipStream_t s, const Ctrl *ctrl, const int32_t *state, double *z, const double *f1,
                      const double *f2, const double *f3, int64_t ld, int64_t n, int64_t kc, int32_t p, double *part,
                      double *sigma);

// Near-degenerate pair rotation (ipt_pairs.hip).  launch_pair_rotate: for problems b
// < count (n[b] <= 4096, theta at toff[b], row-major Delta at doff[b]), pairs
// (partner[toff + r]), their rotations (cs[2 (toff + r) + 0/1]) and the rotated
// partition in tp/dp (tp holds a copy of theta on entry; Delta is copied to dp at the
// same offsets as it is searched), then the level shifts moved into theta' (first and
// second order); best,
// rmax and th2 are scratch of the same length as tp.  launch_pair_rows: rows
// of each pair in z (ncols[b] columns, leading dimension ldz[b], at zoff[b]) rotated
// back (z = R z', forward = 0) or forward (z' = R^T z, forward = 1).
hipError_t launch_pair_rotate(hipStream_t s, int32_t count, int32_t max_n, const int32_t *n, const int64_t *toff,
                              const int64_t *doff, const double *theta, const double *delta, double *tp, double *dp,
                              int32_t *best, double *rmax, int32_t *partner, double *cs, double tau, double *th2);
hipError_t launch_pair_rows(hipStream_t s, int32_t count, const int32_t *n, const int64_t *toff, const int64_t *zoff,
                            const int64_t *ldz, const int32_t *ncols, double *z, const int32_t *partner,
                            const double *cs, int32_t forward);

// The product and fused epilogue of one sweep (ipt_gemm.hip), in the precision the
// device-side ladder chose (ctrl->prec).
hipError_t launch_sweep_gemm(hipStream_t s, const Ctrl *ctrl, const double *delta, int64_t lda, const void *dlo,
                             const float *d32, const void *zt, const double *zin, double *zout, const double *theta,
                             ColState cs, const double *dvec, double *part, int64_t n, int64_t np, int64_t kp,
                             int32_t sweep, int32_t low_type, double *ypart, int nblk, double *dnp, int32_t mid_x3);
// Launch bounds of the split-K path of narrow sweeps (grid sizes and the tiles of
// the partial-product workspace, each 128 x 128 FP64); all zero when no packed width
// of this shape is narrow.
struct SplitBounds {
    int64_t split_blocks, epi_blocks, ypart_tiles;
};
SplitBounds split_bounds(int64_t np, int64_t kp, int nblk);



// ---------------------------------------------------------- complex (ipt_complex.hip)
// Dense IPT over C^n; complex arrays are (re, im) pairs of doubles.
hipError_t launch_zsetup(hipStream_t s, Ctrl *ctrl, const double *theta, const double *delta, int64_t lda,
                         double *th_re, double *th_im, double *part2, int64_t n);
int64_t zsetup_part2_doubles(int64_t n);
hipError_t launch_zcheck_gaps(hipStream_t s, Ctrl *ctrl, const double *th_re, const double *th_im, const int32_t *idx,
                              int64_t n, int64_t k);
hipError_t launch_zload(hipStream_t s, const Ctrl *ctrl, const double *z0, int64_t ldz0, double *zb, int64_t kp,
                        const int32_t *idx, int64_t n, int64_t np, int64_t k);
int64_t zdiag_part_doubles(int64_t kp);
hipError_t launch_zdiag(hipStream_t s, const Ctrl *ctrl, const double *delta, int64_t lda, const double *zin,
                        int64_t kp, ColState cs, double *dpart, double *d_re, double *d_im, int64_t n);
int64_t zsweep_tile();
hipError_t launch_zsweep1(hipStream_t s, const Ctrl *ctrl, const double *delta, int64_t lda, const double *th_re,
                          const double *th_im, ColState cs, double *d_re, double *d_im, double *zout, int64_t kp,
                          double *part, int64_t n, int64_t np);
hipError_t launch_zsweep(hipStream_t s, const Ctrl *ctrl, const double *delta, int64_t lda, const double *th_re,
                         const double *th_im, const double *zin, double *zout, ColState cs, const double *d_re,
                         const double *d_im, double *part, int64_t n, int64_t np, int64_t kp);
hipError_t launch_zcopyout(hipStream_t s, const Ctrl *ctrl, ColState cs, const double *buf0, const double *buf1,
                           int64_t kp, double *z_out, int64_t ldz, const double *lam_im, double *lambda_out,
                           int32_t *status_out, int64_t n, int64_t k, const ipt_colinfo *ci);

// ------------------------------------------------------ complex CSR (ipt_zcsr.hip)
// Sparse IPT over C^n: val holds nnz (re, im) pairs; Z buffers are n x ldz complex.
// The sweep writes per-row-block partial sums part[block][k][NPART] (reduced by
// launch_reduce_parts with ldp = k); unit_in: the product-free first sweep of a cold
// start, which also writes d_c = Delta_ii.
int64_t zspmm_row_blocks(int64_t n);
hipError_t launch_zspmm_sweep(hipStream_t s, const Ctrl *ctrl, const int32_t *row_ptr, const int32_t *col,
                              const double *val, const double *th_re, const double *th_im, const double *zin,
                              double *zout, ColState cs, double *d_re, double *d_im, double *part, int64_t n,
                              int64_t k, int64_t ldz, int32_t unit_in);
hipError_t launch_zdiag_csr(hipStream_t s, const Ctrl *ctrl, const int32_t *row_ptr, const int32_t *col,
                            const double *val, const double *zin, int64_t ldz, ColState cs, double *d_re,
                            double *d_im, int64_t k);

}  // namespace ipt
