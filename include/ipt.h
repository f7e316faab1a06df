/*
 * ipt.h -- C ABI of the MI355X (gfx950) Iterative Perturbation Theory eigensolver.
 *
 * The method (Kenmoe, Kriemann, Smerlak, Zadorin, "A fast iterative algorithm for
 * near-diagonal eigenvalue problems"):
 *   M = D + Delta with D diagonal, theta = diag(D) pairwise distinct (Sec. 3, the
 *   partition; any split is allowed and Delta may have a non-zero diagonal).
 *   G_jk = 1/(theta_j - theta_k) for j != k, G_jj = 0 (inverse gaps matrix).
 *   For each requested index i = idx[c], column c of Z is iterated with
 *     f_i(z) = e_i + g_i o (z (Delta z)_i - Delta z)          (eq. single_line_dyn)
 *   i.e. all columns at once Z <- F(Z) = I + G o (Z D(Delta Z) - Delta Z)  (eq. dyn)
 *   from Z = I (Alg. 1 / Alg. 2), until the per-column relative step
 *   s_c = |F(Z)_c - Z_c|_2 / |Z_c|_2 is <= tol.  The returned eigenvector is the
 *   iterate that passed the test (entry i equals 1, intermediate normalisation) and
 *   lambda_c = (M Z)_ic = theta_i + (Delta Z)_ic from that same sweep (Alg. 1/2
 *   return steps).
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer owned by the caller (allocated with
 *     hipMalloc or by PyTorch on the GPU), except where a parameter says "host".
 *     The library never frees or retains caller memory past the call.
 *   - Matrices are row-major: element (j, c) of an n x k matrix X with leading
 *     dimension ldx is X[j*ldx + c].
 *   - Work is ordered on the handle's stream.  A solve call returns when its
 *     outputs are written (it waits on the stream for the stop decision), so the
 *     outputs are ready on return.  One handle per stream; a handle is not
 *     thread-safe.  Handles may be created on any device; a handle uses the device
 *     that was current at ipt_create.
 *   - Errors are returned as ipt_status, never by aborting.  ipt_last_error gives
 *     a human-readable message for the last failing call on a handle.  On
 *     IPT_EINVAL, IPT_EDEGENERATE, IPT_ENOMEM and IPT_EHIP the output arrays are
 *     unspecified.  IPT_ENOTCONV means every output is written and some column's
 *     status is not IPT_CONVERGED.
 *   - Logging: with IPT_LOG set (to anything but "0") in the environment, every
 *     solve prints to stderr, after its outputs are written, one summary line (the
 *     ipt_info fields) and one line per sweep (precision, active columns, max step
 *     s_c and, with IPT_FLAG_TIME_KERNELS, the product kernel's time).  The lines
 *     come from the history the device keeps, so logging adds no synchronisation
 *     inside a solve.
 *   - Debug mode: with IPT_GUARD set (to anything but "0") when a handle is created,
 *     every slice a solve carves out of the handle's workspace is followed by a
 *     4 KiB guard band of a known pattern, written before the solve's first kernel
 *     and checked after its last; a changed band fails the solve with IPT_EGUARD and
 *     ipt_last_error names the band.  IPT_GUARD=selftest also overwrites 8 bytes of
 *     the second band from the host before each solve, so that the check must fire.
 *     The no-allocation solve and the network calls carve no bands.
 */
#ifndef IPT_H
#define IPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ipt_status {
    IPT_OK = 0,
    IPT_EINVAL = 1,      /* bad sizes, pointers, indices or options; non-finite theta */
    IPT_EDEGENERATE = 2, /* theta_j == theta_idx[c] for some j != idx[c]: G undefined (Sec. 3) */
    IPT_ENOTCONV = 3,    /* outputs written, some column NOT_CONVERGED or DIVERGED */
    IPT_EHIP = 4,        /* a HIP runtime call failed */
    IPT_ENOMEM = 5,      /* workspace allocation failed */
    IPT_EGUARD = 6       /* debug mode only (IPT_GUARD): a kernel wrote into a workspace guard band */
} ipt_status;

/* Per-column status written to col_status[c]. */
enum { IPT_CONVERGED = 0, IPT_NOT_CONVERGED = 1, IPT_DIVERGED = 2 };

/* Arithmetic of the product Delta x Z in a sweep. */
enum {
    IPT_PREC_FP64 = 0,   /* every product in FP64 (plain IPT) */
    IPT_PREC_LADDER = 1  /* low precision -> FP32 class -> FP64; only FP64 sweeps may certify */
};
/* Low rung of the ladder. */
enum { IPT_LOW_BF16 = 0, IPT_LOW_FP16 = 1, IPT_LOW_NONE = 2 /* start the ladder at FP32 */ };

/* Precision tags recorded per sweep in ipt_info.sweep_prec. */
enum { IPT_SWEEP_EXACT_FIRST = 0, IPT_SWEEP_LOW = 1, IPT_SWEEP_FP32 = 2, IPT_SWEEP_FP64 = 3 };

typedef struct ipt_opts {
    double tol;         /* eta of the stopping test (per-column relative step); default 1e-10 */
    int32_t max_iter;   /* maximum sweeps; default 100; 1 <= max_iter <= 100000 */
    int32_t precision;  /* IPT_PREC_FP64 (default) or IPT_PREC_LADDER */
    int32_t low_type;   /* IPT_LOW_BF16 (default), IPT_LOW_FP16 or IPT_LOW_NONE */
    int32_t sync_every; /* sweeps launched between host checks of the device stop flag; 0 = auto */
    double tau_low;     /* ladder: leave the low rung once max step <= tau_low; default 1e-5 */
    double tau_32;      /* ladder: leave FP32 once max step <= tau_32; default 1e-9.  A rung
                         * is also left early once the next sweeps are predicted to certify
                         * (IPT_CERTIFY_SLACK) */
    double div_norm;    /* DIVERGED when |f_i(z) - e_i|_2 > div_norm; default 1e3 */
    int32_t div_growth; /* DIVERGED when s grew on this many consecutive FP64 sweeps; default 8 */
    int32_t flags;      /* IPT_FLAG_* bits */
    double cont_alpha;  /* 0 (default): the autonomous map.  0 < cont_alpha < 1: the
                         * non-autonomous continuation of the concluding discussion (its
                         * 3 x 3 example): sweep t applies the map of the partition
                         * D + (1 - cont_alpha^t) Delta, cont_alpha^t formed by repeated
                         * multiplication in FP64, so the scale reaches exactly 1 once
                         * cont_alpha^t drops below half an ulp of 1 (t = 54 for 1/2).  A
                         * column certifies only on a sweep of scale 1; before that only
                         * the non-finite and div_norm rules (on the scaled iterate) end a
                         * column, and the growth rule restarts.  It moves the start e_i
                         * (or z0) along with the fixed point as the perturbation grows.
                         * Real dense and CSR solves with precision = IPT_PREC_FP64 and
                         * without IPT_FLAG_ACX only; elsewhere IPT_EINVAL */
    int32_t homotopy_q; /* 0 or 1 (default): one solve.  Q > 1 (at most 1000): the homotopy
                         * restart of the concluding section, dense solves only: stages
                         * q = 1..Q solve the partition D + (q/Q) Delta (each entry times the
                         * FP64 number q/Q), each started from the previous stage's vectors
                         * (the first from z0, or cold); the last stage is the problem
                         * itself and gives the outputs and statuses.  info sums sweeps,
                         * matvecs and time over the stages.  Not with cont_alpha */
} ipt_opts;

/* Skip |M|_1 (one extra pass over Delta) and report resid unnormalised. */
#define IPT_FLAG_NO_NORM 1
/* Bracket every product kernel launch with HIP events on the handle's stream and
 * report the device time per sweep precision in ipt_info.prec_ms. */
#define IPT_FLAG_TIME_KERNELS 2
/* Batched solves: launch every sweep from the host instead of replaying the captured
 * hipGraph of a chunk of sweeps (the results are the same, bit for bit). */
#define IPT_FLAG_NO_GRAPH 4
/* IPT-ACX (Sec. 5, Alg. 3): replace the plain update by alternating cyclic
 * extrapolation with orders 3, 2, 3, 2, ...: a cycle of order p applies F p times
 * (F(z), ..., F^p(z)) and moves each active column to
 *   z + sum_{q=1..p} binom(p, q) sigma^q D^q,  sigma = |<D^p, D^(p-1)>| / |D^p|^2,
 * D^q the q-th forward difference of the iterates (sigma = 1 when D^p = 0).  The
 * stopping and divergence tests run on the first application of each cycle; a
 * test whose cycle could not be followed by another test within max_iter ends the
 * column NOT_CONVERGED.  Sweeps then count applications of F.  Requires
 * precision = IPT_PREC_FP64 (every application is an FP64 sweep). */
#define IPT_FLAG_ACX 8
/* Dense ladder: compute the FP32-class rung's correction product Delta (Z - E) on
 * the FP32 matrix cores.  By default it is formed from three FP16 products: A =
 * s_d Delta and B = s_z (Z - E), scaled by powers of two into the FP16 range, are
 * split into hi + lo halves and A B ~ Ah Bh + Ah Bl + Al Bh accumulated in FP32,
 * about 2^-22 relative against FP32's 2^-24, at FP16 matrix-core speed.  Either way
 * only FP64 sweeps certify a column.  (The sparse and batched ladders always use FP32.) */
#define IPT_FLAG_MID_FP32 16
/* A choice of D (the concluding section's use of the freedom in choosing D to widen
 * the convergence domain), for batched solves and for full-spectrum dense solves
 * (ipt_solve_dense with k = n, idx and z0 NULL, lda = ldz = n <= 4096, no continuation
 * or homotopy: run as a batch of one problem, so a ladder runs the batched FP32 and FP64
 * sweeps and opts.low_type is ignored).  Before solving, each problem is
 * re-partitioned, M unchanged:
 *  1. Near-degenerate pairs: i, j that are each other's strongest coupling relative
 *     to the gap, r_ij = |Delta_ij| / |theta_i - theta_j| > IPT_PAIR_TAU, with
 *     Delta_ij == Delta_ji, are rotated out: M' = R^T M R with the 2x2 Jacobi rotation
 *     [[c, s], [-s, c]] that diagonalizes the pair's block of M = diag(theta) + Delta;
 *     the pair takes the rotated block's diagonal as theta and loses its coupling.
 *  2. Level shifts: theta' = theta + Delta_ii + s_i with the second-order shift
 *     s_i = sum_{k != i} Delta_ik Delta_ki / ((theta + Delta_ii)_i - (theta + Delta_kk)_k),
 *     Delta'_ii = -s_i.
 * IPT runs on (theta', Delta') (same eigenvalues) and z = R z' is returned, so a paired
 * column c is normalized by (R^T z)_c = 1 instead of z_c = 1.  Residuals are normalised
 * by |M'|_1 of the re-partitioned matrix (reported as info.norm1 by a dense solve).  The
 * re-partitioned copies of the pools take a second workspace of their size. */
#define IPT_FLAG_CHOOSE_D 32
#define IPT_PAIR_TAU 0.05
/* Ladder rule (dense and sparse): the precision of the next sweep follows the steps
 * seen so far.  After sweep t the largest column step s_t and the ratio q = s_t /
 * s_(t-1) predict the next step q s_t; after the exact first sweep of a cold start
 * q ~ s_1 (the first-order correction), so s_1^2 and s_1^3 are the steps one and two
 * sweeps on.  A rung moves to FP64 (or a cold start skips the low rung) when that
 * prediction is <= IPT_CERTIFY_SLACK * tol: only the prediction is relaxed, a column
 * still certifies only on an FP64 step <= tol. */
#define IPT_CERTIFY_SLACK 2.0
#define IPT_HIST 128

/* Host struct filled by a solve (may be NULL). */
typedef struct ipt_info {
    int32_t sweeps;        /* sweeps executed (applications of F) */
    int32_t converged;     /* columns CONVERGED */
    int32_t not_converged; /* columns NOT_CONVERGED */
    int32_t diverged;      /* columns DIVERGED */
    int64_t matvecs;       /* sum over sweeps of the columns multiplied by Delta */
    double max_step;       /* max over columns of the deciding step s_c */
    double norm1;          /* |M|_1 = max column sum of |D + Delta| (0 if IPT_FLAG_NO_NORM) */
    double max_resid;      /* max over CONVERGED columns of |M z - lambda z|_2 / (|M|_1 |z|_2) */
    float time_ms;         /* device time of the solve, from the first kernel to the outputs */
    int32_t hist_len;      /* entries used in the per-sweep arrays below (min(sweeps, IPT_HIST)) */
    int32_t sweep_prec[IPT_HIST];     /* IPT_SWEEP_* of each sweep */
    int32_t sweep_active[IPT_HIST];   /* active columns entering each sweep */
    double sweep_max_step[IPT_HIST];  /* max s_c over the active columns of each sweep */
    /* With IPT_FLAG_TIME_KERNELS, indexed by IPT_SWEEP_*: summed device time of the
     * kernel that computed each sweep's product (the product-free first sweep, the
     * low-precision, FP32 or FP64 GEMM / SpMM) and the number of such sweeps. */
    float prec_ms[4];
    int32_t prec_sweeps[4];
    /* With IPT_FLAG_TIME_KERNELS: device time of each sweep's product kernel(s). */
    float sweep_ms[IPT_HIST];
} ipt_info;

/* Optional per-column device outputs (any member may be NULL). */
typedef struct ipt_colinfo {
    int32_t *sweeps; /* [k] sweep at which the column's status was decided */
    double *step;    /* [k] s_c of the deciding sweep */
    double *resid;   /* [k] |M z_c - lambda_c z_c|_2 / (|M|_1 |z_c|_2), from F(Z) - Z = -G o (MZ - Z Lambda) */
} ipt_colinfo;

typedef struct ipt_context *ipt_handle;

/* Fill *o with the defaults listed in ipt_opts. */
void ipt_opts_default(ipt_opts *o);

/* Create a handle bound to the current device and to `stream` (a hipStream_t; NULL
 * is the null stream).  The handle owns a workspace that grows on demand and is
 * released by ipt_destroy.  Errors: IPT_EINVAL (h NULL), IPT_EHIP, IPT_ENOMEM. */
ipt_status ipt_create(ipt_handle *h, void *stream);
ipt_status ipt_destroy(ipt_handle h);
/* Rebind the handle to another stream on the same device. */
ipt_status ipt_set_stream(ipt_handle h, void *stream);

/*
 * Dense solve (Alg. 1 on the requested columns; Alg. 2 when idx covers 0..n-1).
 *   n          problem size, 1 <= n <= 2^20
 *   theta      [n] FP64, the diagonal of D; must be finite
 *   delta      n x n FP64 row-major, leading dimension lda >= n
 *   k          number of requested columns, 1 <= k <= n
 *   idx        [k] int32 distinct indices in [0, n); NULL means idx[c] = c (then any k <= n)
 *   z0         optional n x k FP64 warm start (leading dimension ldz0 >= k); NULL = cold start
 *              from Z = I (the first sweep is then computed without a product, since
 *              F(I) = I - G o Delta restricted to the requested columns).  Entry idx[c]
 *              of column c is taken as 1 whatever z0 holds there (chart z_i = 1, Sec. 2).
 *   opts       host struct, NULL for defaults
 *   z_out      n x k FP64 row-major output (leading dimension ldz >= k); may not alias inputs
 *   lambda_out [k] FP64 eigenvalues; col_status [k] int32 IPT_CONVERGED/NOT_CONVERGED/DIVERGED
 *   info       optional host struct; ci optional per-column device outputs
 * A CONVERGED column holds the certified iterate and lambda from the same sweep.
 * NOT_CONVERGED / DIVERGED columns hold the last computed iterate and the lambda
 * estimate of the last sweep.  Returns IPT_OK, IPT_ENOTCONV, IPT_EINVAL,
 * IPT_EDEGENERATE, IPT_ENOMEM or IPT_EHIP.
 */
ipt_status ipt_solve_dense(ipt_handle h, int64_t n, const double *theta, const double *delta, int64_t lda,
                           int64_t k, const int32_t *idx, const double *z0, int64_t ldz0, const ipt_opts *opts,
                           double *z_out, int64_t ldz, double *lambda_out, int32_t *col_status, ipt_info *info,
                           const ipt_colinfo *ci);

/*
 * Dense solve that allocates nothing, for callers that cannot allocate device or
 * pinned memory during a solve (tight serving loops, harnesses that forbid it).
 * Arguments, results and errors as for ipt_solve_dense, on the same kernels; the
 * workspace is a fixed device array of IPT_NOALLOC_SCRATCH_BYTES that the library
 * holds on each device it runs on until the process ends (its device address is
 * taken once per device by ipt_create, which also allocates the handle's pinned
 * poll buffers).  A solve whose workspace exceeds it (full spectra beyond about
 * n = 1024, fewer columns of larger n) is refused with IPT_EINVAL, as are
 * opts.homotopy_q > 1 and IPT_FLAG_TIME_KERNELS.  Every call on a device shares that
 * device's array, which keeps the last call's contents (each solve initialises what
 * it reads): calls that overlap on one device, from any handle or thread, race and
 * must be serialised by the caller.
 */
#define IPT_NOALLOC_SCRATCH_BYTES (128u << 20)
ipt_status ipt_solve_dense_noalloc(ipt_handle h, int64_t n, const double *theta, const double *delta, int64_t lda,
                                   int64_t k, const int32_t *idx, const double *z0, int64_t ldz0,
                                   const ipt_opts *opts, double *z_out, int64_t ldz, double *lambda_out,
                                   int32_t *col_status, ipt_info *info, const ipt_colinfo *ci);

/*
 * Dense solve over C^n (Sec. 2 states IPT for complex M: the same map, the stopping
 * test on the Euclidean norm of C^n, lambda = theta_i + (Delta z)_i).
 *   theta      [n] complex, finite; delta n x n complex row-major (lda >= n complex elements)
 *   z0         optional n x k complex warm start (ldz0 >= k); entry idx[c] of column c is
 *              taken as 1 + 0i
 *   z_out      n x k complex (ldz >= k); lambda_out [k] complex
 * A complex number is a (re, im) pair of doubles (the layout of C99 double complex,
 * std::complex<double> and torch.complex128); theta, delta, z0, z_out and lambda_out
 * must be 16-byte aligned.  n, k, idx, col_status, info and ci as for ipt_solve_dense;
 * |M|_1 and the eigen-residual use the modulus.  Sweeps are FP64 (four real
 * matrix-core products per complex product; the first sweep of a cold start needs no
 * product, as in the real solve): opts.precision must be IPT_PREC_FP64, and IPT_FLAG_ACX,
 * IPT_FLAG_CHOOSE_D, opts.cont_alpha and opts.homotopy_q > 1 are rejected with IPT_EINVAL.
 * IPT_EDEGENERATE when theta_j == theta_i (both parts) for a requested i and j != i.
 */
ipt_status ipt_solve_dense_z(ipt_handle h, int64_t n, const double *theta, const double *delta, int64_t lda,
                             int64_t k, const int32_t *idx, const double *z0, int64_t ldz0, const ipt_opts *opts,
                             double *z_out, int64_t ldz, double *lambda_out, int32_t *col_status, ipt_info *info,
                             const ipt_colinfo *ci);

/*
 * Sparse solve with Delta in CSR form (few eigenpairs of a sparse near-diagonal M,
 * Sec. 6.1): row_ptr [n+1] int32 (row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz),
 * col [nnz] int32 in [0, n), val [nnz] FP64.  Duplicate entries are summed.  Other
 * arguments as for ipt_solve_dense.  The precision ladder uses FP32 then FP64.
 */
ipt_status ipt_solve_csr(ipt_handle h, int64_t n, const double *theta, const int32_t *row_ptr, const int32_t *col,
                         const double *val, int64_t nnz, int64_t k, const int32_t *idx, const double *z0,
                         int64_t ldz0, const ipt_opts *opts, double *z_out, int64_t ldz, double *lambda_out,
                         int32_t *col_status, ipt_info *info, const ipt_colinfo *ci);

/*
 * Sparse solve over C^n (Sec. 2 states IPT for complex M; Sec. 6.1 is the use case of
 * a few eigenpairs of a large sparse near-diagonal M): Delta in CSR form with complex
 * entries, the same map, stopping test and lambda = theta_i + (Delta z)_i as
 * ipt_solve_dense_z.
 *   theta      [n] complex, finite
 *   row_ptr, col, nnz   as for ipt_solve_csr (duplicate entries are summed)
 *   val        [nnz] complex
 *   z0, z_out, lambda_out, ldz0, ldz   complex, as for ipt_solve_dense_z
 * Complex numbers are (re, im) pairs of doubles; theta, val, z0, z_out and lambda_out
 * must be 16-byte aligned.  |M|_1 (unless IPT_FLAG_NO_NORM) and the eigen-residual use
 * the modulus.  Sweeps are FP64 (the first sweep of a cold start needs no product):
 * opts.precision must be IPT_PREC_FP64, and IPT_FLAG_ACX, IPT_FLAG_CHOOSE_D,
 * opts.cont_alpha and opts.homotopy_q > 1 are rejected with IPT_EINVAL.
 * IPT_EDEGENERATE when theta_j == theta_i (both parts) for a requested i and j != i.
 */
ipt_status ipt_solve_csr_z(ipt_handle h, int64_t n, const double *theta, const int32_t *row_ptr, const int32_t *col,
                           const double *val, int64_t nnz, int64_t k, const int32_t *idx, const double *z0,
                           int64_t ldz0, const ipt_opts *opts, double *z_out, int64_t ldz, double *lambda_out,
                           int32_t *col_status, ipt_info *info, const ipt_colinfo *ci);

/*
 * Batched full-spectrum solve of `count` independent dense problems of uneven size
 * (Alg. 2 applied to each M_b = D_b + Delta_b; the columns of all problems are
 * independent, so one sweep advances every active column of the batch).
 *   ns, theta_off, delta_off, z_off   HOST arrays [count]: size n_b (1 <= n_b <= 4096) and the
 *                                     element offsets of problem b in the pools
 *   theta_pool   FP64 device pool; theta of problem b at theta_pool + theta_off[b] ([n_b])
 *   delta_pool   FP64 device pool; row-major n_b x n_b Delta at delta_pool + delta_off[b]
 *   z_pool       FP64 device pool; row-major n_b x n_b output at z_pool + z_off[b].  It is
 *                also one of the two iterate buffers of the solve, so the problems'
 *                regions must not overlap each other or the input pools
 *   lambda_pool, status_pool   outputs at + theta_off[b] ([n_b] each)
 * Every problem is solved for its full spectrum with the same options; info
 * aggregates over the whole batch.  The first sweep is product-free and also yields
 * |M_b|_1, by which each column's resid is normalised (IPT_FLAG_NO_NORM is ignored).
 * The ladder runs FP32 split-form sweeps, then FP64 sweeps, chosen per column tile;
 * opts.low_type is ignored.  Sweeps after the first are replayed as a captured
 * hipGraph of opts.sync_every sweeps (4 when 0) unless IPT_FLAG_NO_GRAPH or
 * IPT_FLAG_TIME_KERNELS is set.  Problems use the tile size of their size bucket
 * (ipt_batched_tune / ipt_batched_set_tiles).
 * Errors: IPT_EINVAL, IPT_EDEGENERATE (theta_j equal within a problem), IPT_ENOTCONV,
 * IPT_EHIP, IPT_ENOMEM.
 */
ipt_status ipt_solve_batched(ipt_handle h, int32_t count, const int32_t *ns, const int64_t *theta_off,
                             const int64_t *delta_off, const int64_t *z_off, const double *theta_pool,
                             const double *delta_pool, const ipt_opts *opts, double *z_pool, double *lambda_pool,
                             int32_t *status_pool, ipt_info *info);

/* Size buckets of the batched tile table: bucket q holds the problems with
 * 64 q < n_b <= 64 (q + 1). */
#define IPT_TILE_BUCKETS 64

/*
 * Autotune the batched tile table of handle h on a batch laid out as for
 * ipt_solve_batched: for every size bucket present (up to 512 of its problems), time
 * two FP32 and two FP64 sweeps with 32 x 32, 64 x 64 and 128 x 128 tiles and keep the
 * fastest.  z_pool, lambda_pool and status_pool serve as scratch (their contents are
 * undefined afterwards).  tiles_out [IPT_TILE_BUCKETS] (host, may be NULL) receives
 * the table.  Buckets with no problem keep their previous entry.
 */
ipt_status ipt_batched_tune(ipt_handle h, int32_t count, const int32_t *ns, const int64_t *theta_off,
                            const int64_t *delta_off, const int64_t *z_off, const double *theta_pool,
                            const double *delta_pool, double *z_pool, double *lambda_pool, int32_t *status_pool,
                            int32_t *tiles_out);
/* Read or replace the handle's tile table (host arrays of IPT_TILE_BUCKETS entries,
 * each 32, 64 or 128), e.g. to reuse a table tuned earlier.  IPT_EINVAL otherwise. */
ipt_status ipt_batched_get_tiles(ipt_handle h, int32_t *tiles);
ipt_status ipt_batched_set_tiles(ipt_handle h, const int32_t *tiles);

/*
 * Learned warm start: a small MLP x -> [Linear -> tanh] x depth -> Linear -> y, trained
 * and evaluated with the library's own kernels (BF16 MFMA GEMMs with FP32
 * accumulation, MSE loss, Adam on FP32 master weights with BF16 compute copies).  It
 * predicts Z0 for a parametrised family M(eps) = D + eps R (initial guesses, Sec. 7) on
 * top of the family's Rayleigh-Schroedinger series (ipt_rs_terms); the solve it
 * warm-starts still certifies every column with FP64 sweeps, so the network can change
 * the cost of a solve but not its answer.
 * Parameters are stored layer by layer as W_l (out_l x in_l, row-major) then b_l.
 * The kernels round to BF16 (from FP32, to nearest even): the input x, the weights,
 * each hidden activation, the output gradient 2 (y - t) / (batch out) and each hidden
 * gradient; products accumulate in FP32.
 * All arrays are device pointers; x is batch x in_dim and y / targets batch x out_dim,
 * row-major FP32.  The MLP runs on its handle's stream; destroy it before the handle.
 */
typedef struct ipt_mlp_context *ipt_mlp;

/* hidden >= 1, 1 <= depth <= 16 hidden layers, in_dim/out_dim >= 1; weights drawn from
 * Glorot-uniform with a 64-bit seed, biases zero.  Errors: IPT_EINVAL, IPT_ENOMEM, IPT_EHIP. */
ipt_status ipt_mlp_create(ipt_handle h, int32_t in_dim, int32_t hidden, int32_t depth, int32_t out_dim, uint64_t seed,
                          ipt_mlp *out);
ipt_status ipt_mlp_destroy(ipt_mlp m);
/* Number of FP32 parameters (the length of the get/set/grad buffers); -1 for NULL. */
int64_t ipt_mlp_num_params(ipt_mlp m);
ipt_status ipt_mlp_get_params(ipt_mlp m, float *dst);
ipt_status ipt_mlp_set_params(ipt_mlp m, const float *src);
/* y = network(x). */
ipt_status ipt_mlp_forward(ipt_mlp m, const float *x, int32_t batch, float *y);
/* Mean squared error sum_b w_b^2 sum_q (y_bq - t_bq)^2 / (batch out_dim) of network(x)
 * against targets, with per-example weights w (FP32 [batch]; NULL: all 1), and its
 * gradient with respect to every parameter (no update).  loss: host float. */
ipt_status ipt_mlp_loss_grad(ipt_mlp m, const float *x, const float *targets, const float *weights, int32_t batch,
                             float *loss, float *grad);
/* `steps` full-batch Adam steps (beta 0.9/0.999, eps 1e-8) at learning rate lr on the
 * weighted loss of ipt_mlp_loss_grad, each replayed from one captured graph; *loss
 * (host) receives the loss before the last update. */
ipt_status ipt_mlp_train(ipt_mlp m, const float *x, const float *targets, const float *weights, int32_t batch,
                         int32_t steps, float lr, float *loss);
/* Warm starts for `batch` family members with parameters eps[p]: y = network(x), then
 *   Z0_p[j, c] = 1 if j == idx[c], else
 *                sum_{l=1..order} eps_p^l T_l[j, c] + eps_p^(order+1) (mu[q] + sigma[q] y[p, q]),
 * q = j k + c (out_dim must equal n k), T_l the terms of ipt_rs_terms (order x n x k,
 * NULL when order = 0).  z0 of problem p starts at z0 + p * pstride (leading dimension
 * ldz0 >= k).  0 <= order <= 16. */
ipt_status ipt_mlp_predict_z0(ipt_mlp m, const float *x, int32_t batch, const float *mu, const float *sigma,
                              const double *eps, int32_t order, const double *terms, int64_t n, int64_t k,
                              const int32_t *idx, double *z0, int64_t ldz0, int64_t pstride);

/* Standardised training targets for the warm-start network.  For problem p and output
 * q = j k + c: r_pq = (Z_p[j, c] - [j == idx[c]] - sum_{l=1..order} eps_p^l T_l[j, c]) /
 * eps_p^(order+1); mu_q and sigma_q are the mean and standard deviation of r_.q over the
 * batch, weighted by weights[p]^2 (FP64 [batch]; NULL: uniform) and summed in problem
 * order (sigma_q = 1 where it would be below 1e-300); targets[p, q] = (r_pq - mu_q) /
 * sigma_q.  Z_p starts at z + p * pstride with leading dimension ldz; targets is
 * batch x (n k) FP32; mu and sigma are (n k) FP32; eps[p] must be non-zero.  Runs on the
 * handle's stream and returns when done. */
ipt_status ipt_mlp_targets(ipt_handle h, const double *z, int32_t batch, int64_t n, int64_t k, int64_t ldz,
                           int64_t pstride, const int32_t *idx, const double *eps, int32_t order, const double *terms,
                           const double *weights, float *targets, float *mu, float *sigma);

/* Rayleigh-Schroedinger terms of M = D + Delta on the requested columns (App. B, eq.
 * ARS-alpha; the series IPT contains, App. C): with Z^[0] = E and d^[s]_c = (Delta Z^[s])_{idx[c] c},
 *   Z^[l] = G o (sum_{s=0}^{l-1} Z^[l-1-s] diag(d^[s]) - Delta Z^[l-1]),  l = 1..order,
 * so that sum_l eps^l Z^[l] is the perturbation series of D + eps Delta.  theta [n],
 * delta n x n row-major (lda >= n), idx [k]; terms receives order x n x k FP64 (term l
 * row-major n x k at terms + (l-1) n k).  FP64 throughout.  Errors: IPT_EINVAL (sizes,
 * NULL pointers, an index outside [0, n), 1 <= order <= 16), IPT_EDEGENERATE
 * (theta_j == theta_idx[c] for j != idx[c], or theta not finite). */
ipt_status ipt_rs_terms(ipt_handle h, int64_t n, const double *theta, const double *delta, int64_t lda, int64_t k,
                        const int32_t *idx, int32_t order, double *terms);

/* Series warm starts Z0_p = E + sum_{l=1..order} eps[p]^l T_l (the Rayleigh-Schroedinger
 * partial sum of the family member D + eps[p] Delta, App. B) for p < count, from the terms
 * of ipt_rs_terms (order x n x k; NULL when order = 0); entry idx[c] of column c is 1.
 * z0 of problem p starts at z0 + p * pstride (leading dimension ldz0 >= k). */
ipt_status ipt_rs_start(ipt_handle h, const double *eps, int32_t count, int32_t order, const double *terms, int64_t n,
                        int64_t k, const int32_t *idx, double *z0, int64_t ldz0, int64_t pstride);

/* Static description of a status code. */
const char *ipt_status_string(ipt_status s);
/* Message of the last failing call on h ("" if none); valid until the next call on h. */
const char *ipt_last_error(ipt_handle h);

#ifdef __cplusplus
}
#endif
#endif /* IPT_H */
