/*
 * hprlp.h - C interface of the MI355X (gfx950) LP solver.
 *
 * Solves the linear program of the paper's eq.(lp), generalised to two-sided rows,
 *
 *     minimise  c^T x + obj_offset
 *     subject to row_lo <= A x <= row_hi,   col_lo <= x <= col_hi,
 *
 * with the restarted Halpern-Peaceman-Rachford iteration of eq.(hpr) (Section III):
 * diagonal scaling and vector normalisation (Section III-A), lambda = lambda_max(A A^T)
 * by the power method, a primal projection step and a dual projection step per
 * iteration, reflection and Halpern averaging, and periodic FP64 checks of the KKT
 * residual map of Theorem 1 that decide termination, restarts and the penalty sigma.
 * A row with row_hi = +inf is the paper's a_i^T x >= theta_i.
 *
 * Conventions shared by every call:
 *   - Every function returns an HPR_* status (0 = HPR_OK, negative = error) and never
 *     aborts or throws. hpr_last_error() gives a message for the calling thread's
 *     most recent error.
 *   - Input arrays are read during the call only; the library keeps its own copies.
 *     Unless a call says otherwise, pointers are host pointers.
 *   - Output arrays are owned by the caller and must hold the stated number of doubles.
 *   - A handle is used by one thread at a time. All device work of a handle runs on
 *     the stream given in hpr_opts.stream (a hipStream_t), or on a stream the library
 *     creates when it is NULL.
 *   - Results are returned in the original (unscaled) space of the problem.
 */
#ifndef HPRLP_H
#define HPRLP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* call status */
enum {
    HPR_OK = 0,
    HPR_ERR_INVALID = -1,   /* bad argument or problem data (NaN, lo > hi, bad CSR, ...) */
    HPR_ERR_NOMEM = -2,     /* device or host allocation failed */
    HPR_ERR_HIP = -3,       /* a HIP runtime call failed */
    HPR_ERR_STATE = -4      /* call not valid in the handle's state (e.g. no solve yet) */
};

/* termination of a solve (hpr_info.term) */
enum {
    HPR_SOLVED = 1,         /* rel_kkt <= tol, verified in FP64 */
    HPR_ITER_LIMIT = 2,
    HPR_TIME_LIMIT = 3,
    HPR_NUMERIC_FAIL = 4,   /* NaN or Inf appeared in a check */
    HPR_PRIMAL_INFEASIBLE = 5,  /* at a check, the dual bar point ybar certifies that no x
                                   satisfies the rows and bounds: with dz = -A^T ybar (scaled
                                   problem), h = sum lo_i ybar_i+ - hi_i ybar_i- + sum l_j dz_j+
                                   - u_j dz_j- exceeds 1e-6 times the sum of its terms'
                                   magnitudes (h <= 0 for every sign-feasible y of a feasible
                                   LP), and the sign violations of dz on infinite column bounds
                                   sum to at most 1e-6 sum |ybar_i|; FP64-evaluated. */
    HPR_DUAL_INFEASIBLE = 6,    /* at a check, the step's primal move d = xbar - x (scaled
                                   problem) is a ray: c~^T d < 0, and the distances of A~ d to
                                   the rows' recession cone ((A~d)_i = 0 for two finite sides,
                                   >= 0 with only lo_i finite, <= 0 with only hi_i finite) and of
                                   d to the columns' cone (same rule for l_j, u_j) sum to at most
                                   1e-6 (-c~^T d) / ||c~||: the dual has no feasible point, so the
                                   LP has no finite optimum (unbounded when it is feasible).
                                   Tested after the two above; FP64-evaluated. With FP32 storage
                                   the margin is 1e-3 instead of 1e-6: the iterates grow along
                                   the ray and d carries their FP32 rounding. */
    HPR_STALLED = 7             /* FP32 storage only (hpr_opts.stall_iters): the check rel_kkt
                                   did not fall to half its value at the last such halving while
                                   the iteration count since then grew to the count at that
                                   halving and to at least stall_iters. FP32 rounding of the
                                   scaled matrix and of the iterates puts a floor under the
                                   residuals (of the order of 2^-24 ||A~^T|y~| || / ||c~|| for
                                   the dual one) and can hold the iteration on a plateau above
                                   the tolerance, so such an LP is to be continued with FP64
                                   storage from the returned point (hpr_set_start on an
                                   HPR_FP64 handle of the same LP). */
};

/* storage precision of A and of the iterates (hpr_opts.precision) */
enum {
    HPR_FP64 = 0,           /* everything FP64 */
    HPR_FP32 = 1            /* A, iterates and matrix-vector sums in FP32; norms, inner
                               products, sigma, restart tests and KKT residuals in FP64 */
};

/* scaling steps (hpr_opts.scaling, bit mask), applied in this order */
enum {
    HPR_SCALE_RUIZ = 2,     /* hpr_opts.ruiz_iters passes of max-norm equilibration */
    HPR_SCALE_PC = 1,       /* Pock-Chambolle diagonal scaling with alpha = 1 */
    HPR_SCALE_BC = 4        /* divide bounds by 1 + ||b|| and the cost by 1 + ||c|| */
};

/* One LP in CSR form. Host pointers, or device pointers of the current HIP device (e.g. torch
 * tensors' data) when on_device = 1: the library then reads them on hpr_opts.stream (the
 * caller's work that writes them must be ordered before the call on that stream) into host
 * memory for the scaling and the layouts, and never keeps them. col_idx entries lie in [0, n)
 * with no column repeated inside a row; val and c are finite; bounds may be +-INFINITY but not
 * NaN, row_lo <= row_hi, col_lo <= col_hi, a lower bound is never +inf and an upper bound
 * never -inf. m may be 0 (row_ptr may then be NULL); n must be >= 1. */
typedef struct {
    int32_t m, n;
    int64_t nnz;
    const int64_t *row_ptr;     /* [m + 1], row_ptr[0] = 0, row_ptr[m] = nnz, nondecreasing */
    const int32_t *col_idx;     /* [nnz] */
    const double *val;          /* [nnz] */
    const double *row_lo;       /* [m] */
    const double *row_hi;       /* [m] */
    const double *col_lo;       /* [n] */
    const double *col_hi;       /* [n] */
    const double *c;            /* [n] */
    double obj_offset;
    int32_t on_device;          /* 0: the arrays above are host memory; 1: device memory */
} hpr_lp;

typedef struct {
    double tol;                 /* stop when rel_kkt <= tol (default 1e-4; 0 = run to max_iter) */
    int64_t max_iter;           /* iteration limit, >= 1 (default 1e6) */
    double time_limit_s;        /* wall-clock limit of hpr_solve, <= 0 = none (default 0) */
    int32_t precision;          /* HPR_FP64 (default) or HPR_FP32 */
    int32_t scaling;            /* mask of HPR_SCALE_* (default PC | BC) */
    int32_t ruiz_iters;         /* passes when HPR_SCALE_RUIZ is set (default 10) */
    int32_t check_every;        /* iterations between checks (default 64); iteration 0 and the
                                   last allowed iteration are checks too */
    double sigma0;              /* initial penalty sigma (default 1) */
    double lambda;              /* > 0: use as lambda and skip the power method (default 0) */
    uint64_t seed;              /* power-method start vector (SplitMix64 stream, default 0) */
    int32_t restart;            /* restart rule on (default 1) */
    int32_t sigma_update;       /* sigma adaptation at restarts on (default 1) */
    double sigma_smoothing;     /* weight w in (0, 1] of the target in the log-space update
                                   log sigma <- (1 - w) log sigma + w log sigma* at restarts;
                                   default 1 (sigma <- sigma*); 0.5 = geometric mean */
    double sigma_smoothing_warm;/* w for an LP whose solve starts from the point given by
                                   hpr_set_start / hpr_batch_set_start (default 0.5: near the
                                   solution the anchor move that sigma* is built from is small
                                   and noisy, so it is followed halfway) */
    int32_t power_max_iter;     /* default 200 */
    double power_tol;           /* relative change that stops the power method (default 1e-6) */
    int32_t profile;            /* 1: time one primal and one dual kernel per block of
                                   iterations with HIP events (hpr_get_kernel_stats) */
    int32_t unroll;             /* quads (4 entries) per lane and pass in the matrix products:
                                   1, 2, 4 or 8; 0 (default) = pick per matrix by timing at
                                   hpr_create (U = 1, 2, 4; ordinary or non-temporal loads),
                                   or reuse the pick made earlier in the process for a matrix of
                                   the same coarse signature (size and row-length profile).
                                   The choice fixes the summation order. */
    int32_t lds_windows;        /* LDS windows of the gathered vector in the matrix products:
                                   0 = none; 1 = "full" windows only (a block whose rows use at
                                   most 16 KB of vector entries copies them into LDS first; a
                                   block of rows with 8 or more lanes each whose window spans at
                                   least 8 KB takes up to 4 rounds of rows while that copy is
                                   more than a quarter of its stored entries, in matrices where
                                   such blocks hold at least a quarter of the entries);
                                   2 = full and "split" windows (the two aligned 8 KB tiles
                                   holding most of a block's entries, the rest read from global
                                   memory); 3 = full, split and "sliced" windows (a block walks
                                   up to 8 consecutive 16 KB windows one at a time, entries
                                   outside them read from global memory); 4, 5 = as 3, with the
                                   rows of sliced blocks regrouped to 16 (4) or 8 (5) lanes per
                                   row, so that each window copy serves more rows; 6, 7 = as 3,
                                   with every row given at most 16 (6) or 8 (7) lanes; -1
                                   (default) = the mode 1 to 7 picked per matrix by timing at
                                   hpr_create
                                   (2 when unroll is given). Results agree to rounding across
                                   modes; modes 0, 1 and 2 sum in the same order. */
    int32_t use_graph;          /* 1 (default): replay each block of check_every iterations,
                                   its check and its control step as one captured HIP graph;
                                   0: launch every kernel directly */
    int32_t warm_fallback;      /* guard of a solve from a caller's start point (hpr_info.warm_start
                                   tells which start each LP used): 0 = none; 1 = compare the
                                   first check (one iteration) from that point with the one from
                                   zero and start from zero when the point's rel_kkt is not finite
                                   or above warm_fallback_ratio times the zero start's; 2 (default)
                                   = run both starts to the second check (1 + check_every
                                   iterations) and keep the point when it stopped there as solved
                                   or its rel_kkt is finite and no higher than the zero start's
                                   (which did not stop as solved); when every LP keeps its point
                                   the solve continues from that run, otherwise all LPs start
                                   again from the chosen points. The probe iterations are not
                                   counted in hpr_info.iters; their time is in solve_s. */
    double warm_fallback_ratio; /* mode 1's ratio, default 1000 (a guard against broken
                                   predictions: an early check does not predict the iteration
                                   count) */
    int64_t stall_iters;        /* FP32 storage: smallest iteration span of the stall test that
                                   ends a solve as HPR_STALLED (default 0 = no test: the solve
                                   runs to its limits; a plateau of the method itself can pass
                                   the test too, so it is for callers that continue such LPs
                                   with FP64 storage) */
    void *stream;               /* hipStream_t or NULL */
} hpr_opts;

typedef struct {
    int32_t term;               /* HPR_SOLVED, ... */
    int64_t iters;              /* iterations performed */
    int64_t restarts;
    double pobj, dobj;          /* primal and dual objective (original space) */
    double rel_p, rel_d, rel_gap, rel_kkt;   /* relative KKT residuals, FP64 */
    double lambda, sigma;       /* step constant used and final sigma */
    double setup_s;             /* hpr_create: scaling, transfer, power method */
    double solve_s;             /* hpr_solve wall time; for a member of a batch, the time from the
                                   start of hpr_batch_solve to the check at which that LP stopped
                                   (the whole call for members still running at its end) */
    int32_t warm_start;         /* 1: started from the point of hpr_set_start, 0: from zero */
} hpr_info;

/* Kernel timings of the last hpr_solve with hpr_opts.profile = 1: average duration of
 * the fused primal step (A^T product, box projection, Halpern averaging) and of the
 * fused dual step (A product, row projection, Halpern averaging) in sampled non-check
 * iterations (every fourth block), from HIP events that the launch stamps at each sampled
 * kernel's own start and end (hipExtLaunchKernelGGL) on the solve's stream. */
typedef struct {
    double primal_ms;
    double dual_ms;
    int64_t samples;
    int32_t unroll_a;           /* schedule used for A (dual step) */
    int32_t unroll_at;          /* schedule used for A^T (primal step) */
    int32_t nontemporal_a;      /* 1: A streamed with non-temporal loads */
    int32_t nontemporal_at;
    int32_t full_blocks_a;      /* thread blocks of A's schedule with a full LDS window */
    int32_t split_blocks_a;     /* ... with a split window */
    int32_t full_blocks_at;     /* the same for A^T */
    int32_t split_blocks_at;
    int32_t blocks_a;           /* all thread blocks of A's schedule */
    int32_t blocks_at;
    int32_t sliced_blocks_a;    /* thread blocks of A's schedule with sliced windows */
    int32_t sliced_blocks_at;
    double setup_prep_s;        /* hpr_create phases: validation, scaling, layouts, schedules (host) */
    double setup_upload_s;      /* ... transfers, FP32 casts, allocation of the iterates */
    double setup_tune_s;        /* ... schedule tuner */
    double setup_power_s;       /* ... power method */
    int64_t narrow_quads_a;     /* stored quads (4 entries) of A's rows with 16-bit column offsets */
    int64_t packed_quads_a;     /* ... of which packed into one 32-bit word (13-bit offset of the
                                   first entry, three 6-bit gaps to the next ones) */
    int64_t narrow_quads_at;    /* the same for A^T */
    int64_t packed_quads_at;
    int32_t packed_a;           /* 1: A's products read the packed words (from 90% packed quads
                                   on; otherwise the 16-bit offsets only) */
    int32_t packed_at;
    int32_t win_mode_a;         /* LDS window mode of A's schedule (hpr_opts.lds_windows, 0 to 7;
                                   the tuner's pick under -1) */
    int32_t win_mode_at;
    int32_t round_blocks_a;     /* thread blocks of A's schedule with a full window that take their
                                   rows in more than one round (up to 4 x 256/G rows, G >= 8 lanes
                                   per row, share one window copy) */
    int32_t round_blocks_at;
} hpr_kernel_stats;

typedef struct hpr_handle hpr_handle;

/* Fills *opts with the defaults listed above. */
void hpr_default_opts(hpr_opts *opts);

/* Validates and copies the LP, scales it, uploads it to the current HIP device and
 * computes lambda. *out receives a handle to free with hpr_destroy. */
int hpr_create(const hpr_lp *lp, const hpr_opts *opts, hpr_handle **out);

/* Replaces the column bounds (original space), e.g. to fix binaries as the paper's
 * Fix operator does; A, rows and scaling are kept. NULL keeps that side. */
int hpr_set_bounds(hpr_handle *h, const double *col_lo, const double *col_hi);

/* Sets the start point (original space) of the next hpr_solve: x0 [n], y0 [m]; NULL for
 * either means zero. The point is projected onto the bounds (x) and onto the sign
 * pattern of the rows (y: >= 0 needs a finite lower side, <= 0 a finite upper side). */
int hpr_set_start(hpr_handle *h, const double *x0, const double *y0);

/* Runs the iteration from the start point until tol, max_iter or the time limit. */
int hpr_solve(hpr_handle *h, hpr_info *info);

/* Copies the last check's point (xbar [n], ybar [m], zbar [n]) in the original space
 * to caller-owned host arrays; any may be NULL. HPR_ERR_STATE before a solve. */
int hpr_get_solution(hpr_handle *h, double *x, double *y, double *z);

/* Round and the Fixing-Strategy of Algorithm 1 (Section IV-A) on the device, for G units
 * and T hours of binaries (u, v, w). cols [G][T][3] (host) gives the column of u (k = 0), v (1),
 * w (2) of unit g at hour t; a negative entry means the column was removed by a presolve and
 * its value is fixval[same index] (host, may be NULL when every entry names a column). The
 * values are read from x [n] (host, original space) or, when x is NULL, from the bar point of
 * the handle's last solve (unscaled on the device, the point hpr_get_solution returns). Each
 * value is rounded with threshold tau in [0, 0.5): 1 if s >= 1 - tau, 0 if 0 <= s <= tau, -1
 * otherwise, into rounded [G][T][3] (host int8). Then for each unit, from its second hour on,
 * an hour is fixed while the rounded u_t, u_{t-1}, v_t, w_t are all confident and satisfy
 * u_t - u_{t-1} = v_t - w_t and v_t + w_t <= 1; the first hour that fails ends that unit's loop
 * (the first hour is never fixed). fixed [G][T] (host int8) receives 1 for the fixed hours.
 * Applying the fixings (the paper's Fix operator) is the caller's: equal column bounds through
 * hpr_set_bounds, or a presolved LP. HPR_ERR_INVALID for bad sizes, columns, values or tau;
 * HPR_ERR_STATE when x is NULL before a solve. */
int hpr_fix_binaries(hpr_handle *h, const double *x, int32_t G, int32_t T, const int32_t *cols,
                     const double *fixval, double tau, int8_t *fixed, int8_t *rounded);

/* Kernel timings of the last solve (zeros unless it ran with hpr_opts.profile = 1). */
int hpr_get_kernel_stats(hpr_handle *h, hpr_kernel_stats *out);

/* Frees the handle and its device memory. NULL is accepted. */
int hpr_destroy(hpr_handle *h);

/* ---- batches: many LPs solved together (the reduced LPs of successive-fixing rounds,
 * Algorithm 2, or of several scenarios). The LPs are pooled into one block-diagonal
 * problem: every kernel launch covers all of them, each LP keeps its own scaling, lambda,
 * sigma, restarts, checks and termination (decided on the device), and an LP that has
 * finished costs nothing in later launches. Each LP follows exactly the schedule and rules
 * of a single solve with the same options. */
typedef struct hpr_batch hpr_batch;

/* lps: array of `count` LPs (1 <= count <= 1024), same rules as hpr_create. */
int hpr_batch_create(const hpr_lp *lps, int32_t count, const hpr_opts *opts, hpr_batch **out);
int hpr_batch_size(hpr_batch *b, int32_t *count);
/* As hpr_set_bounds / hpr_set_start for LP i (0-based). */
int hpr_batch_set_bounds(hpr_batch *b, int32_t i, const double *col_lo, const double *col_hi);
int hpr_batch_set_start(hpr_batch *b, int32_t i, const double *x0, const double *y0);
/* Solves every LP; infos has `count` entries (solve_s: each LP's time to its stop, at the
 * granularity of the checks). */
int hpr_batch_solve(hpr_batch *b, hpr_info *infos);
/* As hpr_get_solution for LP i. */
int hpr_batch_get_solution(hpr_batch *b, int32_t i, double *x, double *y, double *z);
int hpr_batch_get_kernel_stats(hpr_batch *b, hpr_kernel_stats *out);
/* Frees the batch. NULL is accepted. */
int hpr_batch_destroy(hpr_batch *b);

/* ---- warm-start network: a multilayer perceptron whose forward pass, gradients and
 * Adam step run on the GPU (BF16 weights and activations on the matrix cores with FP32
 * accumulation, FP32 master weights and moments). Layer i: z_i = h_i W_i + b_i with
 * h_{i+1} = max(z_i, 0) except after the last layer; loss 0.5 * mean (out - target)^2.
 * Parameters are one FP32 array: for each layer, W_i (sizes[i] x sizes[i+1], row-major)
 * then b_i (sizes[i+1]). Inputs, targets and outputs are host arrays, row-major. Errors
 * of these calls are reported by hpr_mlp_last_error(). */
typedef struct hpr_mlp hpr_mlp;

/* nlayers in [1, 8]; sizes[0..nlayers] in [1, 4096]; params may be NULL (all zero). */
int hpr_mlp_create(int32_t nlayers, const int32_t *sizes, const float *params, void *stream, hpr_mlp **out);
int hpr_mlp_num_params(hpr_mlp *q, int64_t *n);
/* Replaces the parameters and resets the Adam moments and step count. */
int hpr_mlp_set_params(hpr_mlp *q, const float *params);
int hpr_mlp_get_params(hpr_mlp *q, float *params);
/* Y [n][sizes[nlayers]] = network(X [n][sizes[0]]). */
int hpr_mlp_forward(hpr_mlp *q, const float *X, int64_t n, float *Y);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): hpr_mlp_forward on device arrays, with
 * no allocation of any kind. X [n][sizes[0]] and Y [n][sizes[nlayers]] are FP32 device
 * pointers on the handle's device, row-major, owned by the caller; Y may not overlap X.
 * The work is enqueued on the handle's stream and the call returns without waiting (order
 * the caller's work with that stream, e.g. by creating the handle on it). Results equal
 * hpr_mlp_forward's bit for bit. The BF16 activations live in a fixed 32 MiB device array
 * of the library, one per GPU for the life of the process (its address is resolved at
 * hpr_mlp_create); rows are processed in chunks that fit it (a multiple of 16 rows; each
 * chunk's activations are written before they are read, so nothing needs clearing). Every
 * call on one GPU shares that array: calls that overlap in time on one GPU (two streams,
 * or two threads) race and give wrong results. HPR_ERR_INVALID when 16 rows of the input
 * and of two hidden layers of the widest width do not fit the array (never for widths up
 * to 4096 with up to 8 layers), or for NULL pointers with n > 0. */
int hpr_mlp_forward_device(hpr_mlp *q, const float *X, int64_t n, float *Y);
/* Loss and gradients (same layout as the parameters; grads may be NULL) for targets T. */
int hpr_mlp_gradients(hpr_mlp *q, const float *X, const float *T, int64_t n, float *grads, float *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, rate lr) on the mini-batch (X, T). */
int hpr_mlp_train_step(hpr_mlp *q, const float *X, const float *T, int64_t n, float lr, float *loss);
int hpr_mlp_destroy(hpr_mlp *q);
const char *hpr_mlp_last_error(void);

/* Message of the calling thread's last error ("" if none). */
const char *hpr_last_error(void);

/* Measurement aid: streams a device buffer of `bytes` (>= 1 MiB) `reps` times with a plain
 * read-only kernel and a plain copy kernel on the current device and reports the bandwidth
 * of each in GB/s (copy counts bytes read plus bytes written). Allocates and frees
 * 2 * bytes of device memory; runs on the null stream. */
int hpr_probe_stream(int64_t bytes, int32_t reps, double *read_gbs, double *copy_gbs);

#ifdef __cplusplus
}
#endif

#endif /* HPRLP_H */
