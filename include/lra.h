/*
 * lra.h -- C ABI of the MI355X (gfx950) Cross-Approximation / CUR library.
 *
 * The method (Pan, Luan, Svadlenka, Zhao, "Superfast Low-Rank Approximation
 * and Least Squares Regression", arXiv:1611.01391):
 *   - the LRA problem: an m x n matrix M and a target rank (Section 5.1);
 *   - CUR LRA from a row set I and a column set J, generator M_{I,J} and
 *     nucleus U (Section 6.5, "Primitive, Cynical, and Cross-Approximation
 *     Algorithms and CUR LRA"); U = M_{I,J}^{-1} for k = l = r as in the C-A
 *     experiments (Section 12.2, eq. (eqtsts1));
 *   - C-A iterations alternating vertical and horizontal steps, here in the
 *     dual order that starts with a vertical (column) step (Remark
 *     rec-atnsr); each step picks a k x k submatrix of locally maximal volume
 *     in the strip (Section 6.5, footnote defining the volume; Remark
 *     "re vlmmx" for the cost model);
 *   - FAILURE when the sketch is rank deficient, and the remedy of raising
 *     the rank (Algorithm 5.1, its footnotes);
 *   - a posteriori estimation on a random q x s submatrix of the error
 *     matrix (Appendix F).
 *
 * Conventions for every entry point:
 *   - indices are 0-based int64;
 *   - "device" pointers are HIP device memory on the context's device (a
 *     PyTorch CUDA/HIP tensor's data_ptr() qualifies); "host" pointers are
 *     ordinary host memory;
 *   - all device work is enqueued on the context's stream; the blocking
 *     calls (lra_ca_cur, lra_ca_cur_batched, lra_maxvol, lra_wait) return
 *     after the results are on the host;
 *   - input matrices / point sets are owned by the caller and must stay valid
 *     and unmodified until the call returns (or the ticket completes);
 *   - outputs are caller-owned; the library never frees caller memory;
 *   - one context per host thread; contexts are independent;
 *   - every call returns an lra_status: 0 = OK, > 0 = result valid with a
 *     warning, < 0 = error and the result is invalid.
 */
#ifndef LRA_H
#define LRA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LRA_OK = 0,
    LRA_TOL_NOT_MET = 1,    /* tol not reached at k_max (best result returned)       */
    LRA_MAXVOL_CAP = 2,     /* a maxvol call hit max_swaps                            */
    LRA_NUMERICAL_RANK = 3, /* an LU pivot fell below 64 u max|strip| (or was zero):
                               k reduced to the pivots above it                       */
    LRA_PENDING = 4,        /* lra_poll: the ticket has not completed yet             */
    LRA_EINVAL = -1,        /* invalid argument                                       */
    LRA_ERANK = -2,         /* zero strip (no nonzero pivot) or exactly singular
                               generator (paper: FAILURE)                             */
    LRA_ENOMEM = -3,        /* device allocation failed                               */
    LRA_EBUDGET = -4,       /* request exceeds the context's HBM budget               */
    LRA_EDEVICE = -5,       /* HIP runtime error or device-side time-out              */
    LRA_ENONFINITE = -6,    /* NaN or Inf met in a strip                              */
    LRA_ESCRATCH = -7       /* lra_ca_cur_noalloc: the problem's workspace exceeds the
                               fixed per-device scratch (LRA_NOALLOC_SCRATCH_BYTES)   */
} lra_status;

typedef enum { LRA_SRC_DENSE = 0, LRA_SRC_CAUCHY = 1, LRA_SRC_INVDIST = 2, LRA_SRC_PREPROCESSED = 3 } lra_src_kind;
typedef enum { LRA_F32 = 0, LRA_F64 = 1 } lra_dtype;
/* Strip precision.  FP64: strips, basis and swaps in binary64.  MIXED:
 * strips, basis and swaps in binary32.  BF16SEL: binary32 strips; each
 * swap's candidates are shortlisted (8 rows per wavefront) from a bfloat16
 * MFMA product C C[X,:]^{-1} with binary32 accumulation and rechecked in
 * binary32 before the pivot is chosen (k <= 32, at most 256 strip rows per
 * workgroup in LDS; other steps use the MIXED selection).  The nucleus and
 * the residual estimate are binary64 on binary64 entries in every mode. */
typedef enum { LRA_PREC_FP64 = 0, LRA_PREC_MIXED = 1, LRA_PREC_BF16SEL = 2 } lra_prec;

/* Where the entries a(i,j) come from; the matrix is only ever touched entry
 * by entry (Section 1.1: superfast methods read a tiny fraction of it).
 *   DENSE  : a = device matrix of `dtype`; element (i,j) at a[i*lda + j]
 *            (col_major = 0) or a[j*lda + i] (col_major = 1).
 *   CAUCHY : x (m) and y (n) device vectors of `dtype`; a(i,j) = 1/(x_i - y_j).
 *   INVDIST: x (m), y (n) points; a(i,j) = 1/|x_i - y_j|, 0 where they coincide.
 *   PREPROCESSED: the dense m x n device matrix a (as DENSE) seen through
 *            d-abridged Hadamard multipliers with random sign scaling on both
 *            sides (Section 8.3, family (i); d = pre_depth, 1..8, 2^d must
 *            divide m and n): the source is F A H with
 *            F = D_F H_{m,d} / 2^{d/2}, H = H_{n,d} D_H / 2^{d/2},
 *            H_{n,d} = H_{2^d} (Sylvester, entry (a,b) = (-1)^popcount(a & b))
 *            Kronecker I_{n/2^d}, D_F = diag(+-1) from the top bits of
 *            SplitMix64 stream pre_seed (value i), D_H from stream pre_seed + 1.
 *            F and H are orthogonal, so a CUR C U R of F A H gives the LRA
 *            F^T C U R H^T of A with the same error (Section 6.6), and the
 *            sampled estimate of F A H estimates it.  Each entry sums 4^d
 *            entries of A in binary64 (t outer, u inner).
 * Differences of point coordinates are always formed in binary64. */
typedef struct lra_source {
    int32_t kind;        /* lra_src_kind */
    int32_t dtype;       /* lra_dtype    */
    const void* a;       /* DENSE / PREPROCESSED: device pointer */
    int64_t lda;
    int32_t col_major;
    int32_t pre_depth;   /* PREPROCESSED: recursion depth d */
    const void* x;       /* CAUCHY / INVDIST: device pointers */
    const void* y;
    uint64_t pre_seed;   /* PREPROCESSED: sign streams pre_seed, pre_seed + 1 */
} lra_source;

/* Options; lra_default_options() fills the defaults shown. */
typedef struct lra_options {
    double tau;                  /* maxvol tolerance: swap while max|C C_I^{-1}| > 1 + tau (0.01) */
    int32_t k_max;               /* adaptive rank cap; <= k disables growth (0)             */
    int32_t k_step;              /* rank increment (8)                                      */
    int32_t max_swaps;           /* swaps per maxvol call; <= 0 means 4k + 64 (0)           */
    int32_t warm_start;          /* 1: each step starts from the previous index set (1)     */
    int32_t precision;           /* lra_prec: FP64, MIXED or BF16SEL (FP64)                 */
    int32_t sample_q, sample_s;  /* residual sample shape, each 1..64 (64, 64; capped at m, n) */
    int32_t team_wgs;            /* workgroups per problem; 0 = autotuned (0)               */
    int32_t reserved;
    uint64_t seed;               /* SplitMix64 stream for the default draws below (0)       */
    const int64_t* init_cols;    /* host, optional: candidate columns in draw order;
                                    J0 = first k, rank growth takes the rest, skipping
                                    columns already in J. NULL: draw min(n, 2 k_cap)
                                    distinct columns from stream `seed`.                   */
    int64_t n_init_cols;
    const int64_t* sample_rows;  /* host, optional: Q (sample_q distinct rows); NULL: draw
                                    from stream seed+1 and sort                             */
    const int64_t* sample_cols;  /* host, optional: S (sample_s distinct cols); NULL: draw
                                    from stream seed+2 and sort                             */
    /* The fixed-rank CUR algorithms compared by the C-A tests (Section 12.2)
     * and the Primitive algorithm (Section 6.5); all need tol <= 0.          */
    int32_t cur_rank;            /* Cynical step (Tests 3, 4): after the sweeps, an r x r
                                    generator of locally maximal volume inside the k x k
                                    one, by C-A sweeps on that block; 0 or k: none (0)     */
    int32_t inner_sweeps;        /* sweeps of the Cynical step inside the block, stopping
                                    once one changes nothing (4)                           */
    int32_t nucleus_rank;        /* Primitive nucleus U = (A[I,J])_r^+, the rank-r
                                    truncated pseudo-inverse; 0 or k: A[I,J]^{-1} (0)      */
    int32_t reserved2;
    const int64_t* init_rows;    /* host, optional, sweeps = 0 only: the k random rows I
                                    (distinct); NULL: drawn from stream seed+3              */
} lra_options;

/* Results.  I, J, G, U are caller-owned HOST arrays with capacity
 * k_cap = max(k, k_max) (G, U: k_cap^2, row-major k x k for the final k).
 * C_out / R_out are optional caller-owned DEVICE buffers receiving the CUR
 * factors C = A[:,J] (m x k, column-major) and R = A[I,:] (k x n, row-major)
 * in the strip precision (binary64 for LRA_PREC_FP64, else binary32). */
typedef struct lra_result {
    int64_t* I;
    int64_t* J;
    double* G;                   /* generator A[I,J] (binary64)                    */
    double* U;                   /* nucleus A[I,J]^{-1} (binary64)                 */
    void* C_out;
    void* R_out;
    int32_t k;                   /* final rank                                     */
    int32_t status;              /* lra_status of this problem                     */
    int32_t sweeps_done;
    int32_t swaps_total;
    int64_t entries_read;        /* entries touched: strips, generator, sample     */
    double err_est_rel;          /* ||E_QS||_F / ||A_QS||_F                        */
    double err_est_abs;          /* sqrt(mn/(qs)) ||E_QS||_F                       */
    double err_mean, err_var;    /* sample mean / variance of the E_QS entries     */
    double nucleus_cond1;        /* ||G||_1 ||U||_1                                */
    double t_submit_us, t_start_us, t_end_us;  /* serving time stamps (host clock) */
} lra_result;

typedef struct lra_ctx lra_ctx;

/* One far-field block of a hierarchical partition (Section 9: generators of
 * neutered block columns are low-rank approximations of such blocks). */
typedef struct lra_block {
    lra_source src;              /* the block itself as a source (e.g. pointer offsets) */
    int64_t m, n;
    int32_t k, sweeps;
    double tol;
} lra_block;

/* One request of the serving stream. */
typedef struct lra_request {
    lra_source src;
    int64_t m, n;
    int32_t k, sweeps;
    double tol;
    lra_options opts;
    lra_result* result;          /* where lra_poll / lra_wait deliver the result */
} lra_request;

void lra_default_options(lra_options* opts);

/* Create a context on the current HIP device.  stream: a hipStream_t (NULL =
 * the null stream).  hbm_budget_bytes bounds the device workspace the
 * context may hold (0 = no bound): the workspace of the blocking calls, the
 * serving arena and its control images together.  The workspace grows on
 * demand (by the first call of a larger size; later calls no larger than an
 * earlier one allocate nothing); lra_ca_cur_noalloc never allocates.
 * Errors: LRA_EDEVICE, LRA_ENOMEM. */
lra_status lra_create(lra_ctx** ctx, void* stream, size_t hbm_budget_bytes);
void lra_destroy(lra_ctx* ctx);

/* C-A / CUR of one m x n matrix (Section 6.5): `sweeps` sweeps of one column
 * step (maxvol on A[:,J] -> I) and one row step (maxvol on A[I,:]^T -> J)
 * from J0, then the nucleus U = A[I,J]^{-1} and the sampled residual
 * (Appendix F).  sweeps = 0 (tol <= 0): no C-A step, I = opts->init_rows
 * and J = J0 at random (Section 12.2, Tests 1; with cur_rank the random
 * p x q submatrix of Tests 3; with nucleus_rank the Primitive algorithm).
 * opts->cur_rank and opts->nucleus_rank select the Cynical step and the
 * truncated nucleus (see lra_options; the result then has rank cur_rank,
 * resp. k with a rank-nucleus_rank nucleus).  tol <= 0: exactly `sweeps`
 * sweeps at rank k.  tol > 0:
 * per rank level up to `sweeps` sweeps (stopping once a sweep leaves (I, J)
 * unchanged); if the estimate exceeds tol and k < k_max, k_step new
 * candidate columns are appended and the level restarts from a fresh LU.
 * Requires 1 <= k <= min(m, n, 64), k_max <= 64, sweeps >= 0 (0 only with
 * tol <= 0).
 * Errors: LRA_EINVAL, LRA_ERANK, LRA_ENONFINITE, LRA_ENOMEM, LRA_EBUDGET,
 * LRA_EDEVICE. */
lra_status lra_ca_cur(lra_ctx* ctx, const lra_source* src, int64_t m, int64_t n, int k,
                      int sweeps, double tol, const lra_options* opts, lra_result* result);

/* Allocation-free variant of lra_ca_cur, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results as lra_ca_cur (bit for
 * bit), but it calls no hipMalloc / hipHostMalloc / hipFree or other
 * allocating device routine: the device workspace is a fixed array of
 * LRA_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs on
 * until the process ends (its address is looked up once per device by
 * lra_create), and the upload / read-back image is staged through a fixed
 * host array of 1 MiB.  The context's hbm_budget_bytes does not apply.
 * A problem whose workspace (control image, team control blocks, per-problem
 * scratch, and a global strip of max(m, n) x max(k, k_max) elements when the
 * strip rows do not fit the workgroups' LDS) exceeds the array is rejected
 * with LRA_ESCRATCH before anything is launched.  The array keeps the last
 * call's contents; every call clears the parts that must start at zero with
 * a fill kernel.  Calls in one process are serialised by an internal lock
 * (they share the array and the host staging; calls that overlapped on one
 * GPU would race).  Errors: those of lra_ca_cur except LRA_ENOMEM and
 * LRA_EBUDGET, plus LRA_ESCRATCH. */
#define LRA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
lra_status lra_ca_cur_noalloc(lra_ctx* ctx, const lra_source* src, int64_t m, int64_t n, int k,
                              int sweeps, double tol, const lra_options* opts, lra_result* result);

/* The CUR factors of given row and column sets (Section 6.5: C = M_{:,J},
 * R = M_{I,:}): C = A[:,J] (m x k, column-major, m k elements) and
 * R = A[I,:] (k x n, row-major, k n elements) written into caller-owned
 * device buffers (either may be NULL) in out_dtype (LRA_F32 or LRA_F64),
 * by one kernel over the whole device.  I, J: host arrays of k indices
 * (0 <= I[c] < m, 0 <= J[c] < n; repeats allowed).  Generated sources give
 * the generated entries.  Returns after the factors are written.  With
 * timing enabled (lra_set_timing) the kernel is timed like an engine launch.
 * Errors: LRA_EINVAL (also when m k or k n reaches 2^31), LRA_ENOMEM,
 * LRA_EBUDGET, LRA_EDEVICE. */
lra_status lra_cur_factors(lra_ctx* ctx, const lra_source* src, int64_t m, int64_t n, int k,
                           const int64_t* I, const int64_t* J, int32_t out_dtype, void* C_out, void* R_out);

/* The top SVD of an LRA (Appendix D, Algorithm D.1): given M ~ C W R with
 * C (m x k, column-major, ldc >= m) and R (k x n, row-major, ldr >= n) in
 * device memory (both of dtype LRA_F32 or LRA_F64, e.g. from
 * lra_cur_factors) and W (k x k, row-major, binary64) in host memory (the
 * nucleus of an lra_result), and a target rank 1 <= r <= k <= 64 with
 * k <= m, n: the column-pivoted QR factors C P_C = Q_C R_C and
 * R^T P_R = Q_R R_R are truncated to their first r columns and the r x r
 * middle factor R_C[:r,:] P_C^T W P_R R_R[:r,:]^T is split by its SVD
 * S_bar Sigma T_bar^T, so that S diag(sigma) T^T = Pi_C C W R Pi_R
 * (Pi: the orthogonal projectors on the kept columns of Q_C and Q_R) with
 * S = Q_C[:, :r] S_bar and T^T = T_bar^T Q_R[:, :r]^T.  Outputs, binary64:
 * S (m x r, column-major, lds >= m, device), sigma (r, host, descending) and
 * T^T (r x n, row-major, ldt >= n, device); piv_c and piv_r (host, k each,
 * may be NULL) receive the column pivots of C and of R^T (rows of R).
 * Every step runs on the device in binary64 (C and R are read once for the
 * QR and once for the output); the call returns after the outputs are
 * written.  Errors: LRA_EINVAL (bad sizes or pointers), LRA_ENONFINITE (W, C or
 * R not finite; no output written), LRA_ERANK (a kept diagonal entry of R_C or R_R at most
 * max(m, n) u |R[0,0]|, the rounding level of the QR: the factors have
 * numerical rank below r; S, sigma and T^T untouched,
 * the pivots still written), LRA_ENOMEM, LRA_EBUDGET, LRA_EDEVICE. */
lra_status lra_top_svd(lra_ctx* ctx, int64_t m, int64_t n, int k, int r, int32_t dtype, const void* C,
                       int64_t ldc, const double* W, const void* R, int64_t ldr, double* S, int64_t lds,
                       double* sigma, double* Tt, int64_t ldt, int64_t* piv_c, int64_t* piv_r);

/* The maxvol sub-algorithm alone on a tall device strip (m x k, column-major,
 * leading dimension ld >= m, element type `dtype`): locally maximal-volume
 * k x k row subset I (host, capacity k) such that every entry of
 * strip * strip[I,:]^{-1} is at most 1 + tau in modulus.  init: optional host
 * array of k distinct rows to start from (NULL: partial-pivot LU start).
 * *swaps receives the number of swaps, *k_eff the rank used.  The strip is
 * not modified.  Errors: LRA_EINVAL, LRA_ERANK, LRA_ENONFINITE, LRA_EDEVICE. */
lra_status lra_maxvol(lra_ctx* ctx, const void* strip, int32_t dtype, int64_t m, int64_t ld,
                      int k, double tau, int max_swaps, const int64_t* init, int64_t* I,
                      int* swaps, int* k_eff);

/* Many independent C-A / CUR problems (e.g. all admissible blocks of a
 * hierarchical partition, Section 9) in one persistent launch.  Each block
 * uses its own k, sweeps, tol; `opts` applies to all (init_cols /
 * sample_rows / sample_cols must be NULL: each block draws from stream
 * opts->seed + block index).  results[b] as for lra_ca_cur; the call returns
 * the most severe per-block status. */
lra_status lra_ca_cur_batched(lra_ctx* ctx, const lra_block* blocks, int nblocks,
                              const lra_options* opts, lra_result* results);

/* Serving (continuous batching; the paper has no serving layer, this is the
 * runtime around its C-A / CUR kernels).  Admitted requests own a region of a
 * device arena (inputs, resumable state, results, a global strip); a tick
 * launches the engine once per (precision, rank bucket) over every admitted
 * request with a budget of a few phases each (a phase = one C-A step, or the
 * nucleus + estimate), so requests of any size advance together and a new
 * request joins at the next tick.  Waiting requests are admitted first come
 * first served once their region fits.
 *
 * lra_submit: validates and copies the request (its source arrays and
 *   `result` arrays must stay valid until it completes) and returns a ticket;
 *   it may launch a tick but never waits for the device.  Errors: LRA_EINVAL,
 *   LRA_EBUDGET (the request is larger than the whole arena), LRA_ENOMEM,
 *   LRA_EDEVICE.
 * lra_poll: finishes the in-flight tick if the device is done with it
 *   (delivering completed requests into their lra_result, with host-clock
 *   time stamps) and launches the next; never waits.  Returns LRA_PENDING,
 *   or the completed request's status (every later call returns the same).
 *   LRA_EINVAL for an unknown ticket.
 * lra_wait: like lra_poll, but waits for ticks until the ticket completes.
 * A device error fails every admitted and waiting request with LRA_EDEVICE. */
lra_status lra_submit(lra_ctx* ctx, const lra_request* req, uint64_t* ticket);
lra_status lra_poll(lra_ctx* ctx, uint64_t ticket);
lra_status lra_wait(lra_ctx* ctx, uint64_t ticket);

/* Serving configuration; 0 keeps a value.  arena_bytes: device arena for
 * admitted requests (default min(4 GiB, budget / 2)); max_active: admitted
 * requests at most (default 1024); both only before the first submit.
 * phases_per_tick: phase budget of each request per tick (default 4).
 * Errors: LRA_EINVAL. */
lra_status lra_serve_config(lra_ctx* ctx, size_t arena_bytes, int phases_per_tick, int max_active);

/* Autotuning (a search of this library, not a step of the method): each
 * call times its candidates on the context's stream (HIP events around the
 * engine launches, one warm-up, median of the rest), keeps the fastest in
 * the context for later calls, and returns it.
 *
 * lra_autotune_team: workgroups per problem for single problems of this
 *   size class (precision, rank bucket, bit length of max(m, n)); the
 *   candidates are the automatic choice a and a/4, a/2, 3a/2, 2a, 4a within
 *   the co-resident grid.  Results of the timed runs are discarded.
 * lra_autotune_batched: the planning floor of shared launches (batched calls
 *   and serving ticks: a problem keeps at least ceil(rows / floor) workgroups,
 *   at most 32; 0 = none), over 0, 2048, ..., 65536 rows, on a
 *   representative batch.
 * lra_tuning_save / lra_tuning_load: the context's tuned values as a text
 *   file ("team <class> <workgroups>", "floor <rows>").
 * Errors: LRA_EINVAL, and those of lra_ca_cur / lra_ca_cur_batched. */
lra_status lra_autotune_team(lra_ctx* ctx, const lra_source* src, int64_t m, int64_t n, int k, int sweeps,
                             double tol, const lra_options* opts, int* best_team, double* best_ms);
lra_status lra_autotune_batched(lra_ctx* ctx, const lra_block* blocks, int nblocks, const lra_options* opts,
                                int64_t* best_floor_rows, double* best_ms);
lra_status lra_tuning_save(lra_ctx* ctx, const char* path);
lra_status lra_tuning_load(lra_ctx* ctx, const char* path);

/* Kernel timing of a context.  With timing enabled, HIP events on the
 * context's stream bracket every engine launch; engine_ms_total accumulates
 * their elapsed times and last_engine_ms holds the latest one. */
typedef struct lra_stats {
    int64_t launches;            /* engine launches since creation or reset */
    double engine_ms_total;      /* summed event time (timing enabled only)  */
    double last_engine_ms;
    int32_t last_grid;           /* workgroups of the latest launch          */
    int32_t last_teams;          /* teams of the latest launch               */
    int64_t ticks;               /* serving ticks                            */
    int64_t device_allocs;       /* device allocations since creation (never
                                    reset; a call no larger than an earlier
                                    one makes none)                          */
    int64_t device_bytes;        /* device bytes the context holds now (never
                                    above hbm_budget_bytes when one is set)  */
} lra_stats;
/* enable: 1 on, 0 off; reset: zero the counters. */
lra_status lra_set_timing(lra_ctx* ctx, int enable, int reset);
lra_status lra_get_stats(lra_ctx* ctx, lra_stats* out);

const char* lra_status_str(lra_status s);
/* Library version string. */
const char* lra_version(void);

#ifdef __cplusplus
}
#endif
#endif
