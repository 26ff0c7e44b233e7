/*
 * oracle.h -- plain, slow, obviously-correct CPU reference for the
 * Cross-Approximation (C-A) / CUR low-rank approximation of Pan, Luan,
 * Svadlenka and Zhao, "Superfast Low-Rank Approximation and Least Squares
 * Regression" (arXiv:1611.01391).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this library; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no source, header, table
 * or helper with the GPU library.
 *
 * What it computes (paper references):
 *   - submatrix notation M_{I,:}, M_{:,J}, M_{I,J}: Section 2.1, eq. (eq111);
 *   - C-A iterations: Section 6.5 ("Primitive, Cynical, and
 *     Cross-Approximation Algorithms and CUR LRA"), dual form starting with
 *     a vertical step (Remark rec-atnsr);
 *   - the per-step generator choice by volume maximisation (Section 6.5,
 *     footnote on the volume; Remark "re vlmmx" for the maxvol cost model);
 *     the maxvol sub-algorithm itself is not printed in the paper (it is
 *     delegated to the cited volume-maximisation literature), so the oracle
 *     takes the standard reading: partial-pivot LU start, basis
 *     B = C * C[I,:]^{-1}, swap while max|B| > 1 + tau;
 *   - nucleus U = M_{I,J}^{-1} for k = l = r (Section 12.2, eq. (eqtsts1));
 *   - a posteriori estimate on a random q x s submatrix of the error matrix
 *     (Appendix F), with the sample mean/variance of its entries.
 *
 * Precision: everything in IEEE binary64 unless a function name ends in
 * _f32, in which case the strip / basis / swap arithmetic is binary32 (the
 * "mixed" path's selection precision); nucleus and residual are always
 * binary64.
 *
 * Parity status per function is listed in the test-suite header
 * (tests/test_oracle_pins.py): every function below is pinned.
 */
#ifndef LRA_ORACLE_H
#define LRA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Entry source (host pointers). kind: 0 dense, 1 Cauchy 1/(x_i - y_j),
 * 2 inverse distance 1/|x_i - y_j| (0 where x_i == y_j), 3 the dense matrix
 * pre-processed by abridged scaled Hadamard multipliers (see
 * oracle_entry_f64).
 * dtype: 0 = float32, 1 = float64 (element type of a, or of x and y).
 * Dense: element (i,j) at a[i*lda + j] (row-major) or a[j*lda + i].
 * Kind 3 also uses depth d (1 <= d, 2^d dividing pm and pn), the sign seed
 * and the dimensions pm x pn of a. */
typedef struct {
    int32_t kind;
    int32_t dtype;
    const void* a;
    int64_t lda;
    int32_t col_major;
    int32_t pad_;
    const void* x;
    const void* y;
    int32_t depth;
    int32_t pad2_;
    uint64_t seed;
    int64_t pm, pn;
} oracle_source;

/* Smallest recorded decision margins of one run (relative). */
typedef struct {
    double min_pivot_gap;   /* partial-pivot LU: (|1st| - |2nd|) / |1st|   */
    double min_swap_gap;    /* swap argmax: (|1st| - |2nd|) / |1st|         */
    double min_stop_margin; /* | max|B| - (1+tau) | / (1+tau) at every test */
    double min_rank_margin; /* | |pivot| - thresh | / thresh, strip LU and
                               warm-start elimination (fallback test)        */
    double min_tol_margin;  /* | est_rel - tol | / tol at every rank level   */
} oracle_trace;

typedef struct {
    double tau;          /* maxvol tolerance, >= 0                          */
    int32_t k_max;       /* adaptive rank cap (<= k disables growth)        */
    int32_t k_step;      /* rank increment                                  */
    int32_t max_swaps;   /* per maxvol call; <= 0 means 4k + 64             */
    int32_t warm_start;  /* 1: warm-start each step from the previous set   */
    const int64_t* cand_cols; int64_t n_cand;  /* J0 = cand[0..k), growth from the rest */
    const int64_t* sample_rows; int32_t q;     /* residual sample rows Q   */
    const int64_t* sample_cols; int32_t s;     /* residual sample cols S   */
} oracle_options;

typedef struct {
    int32_t k;            /* final rank                                     */
    int32_t status;       /* 0 ok, 1 tol not met, 2 swap cap, 3 numerical rank, -2 exact rank loss, -6 non-finite */
    int32_t sweeps_done;  /* total sweeps over all rank levels              */
    int32_t swaps_total;
    int64_t entries_read;
    double err_est_rel, err_est_abs, err_mean, err_var, nucleus_cond1;
    oracle_trace trace;
} oracle_result;

/* entry a(i,j) in binary64 (nucleus and residual precision).
 * Kind 3 (Section 8.3, family (i): d-abridged Hadamard multipliers with
 * random diagonal scaling, applied on both sides as in Section 6.6):
 * a(i,j) = (F A H)_ij with F = D_F H_{pm,d} / 2^{d/2}, H = H_{pn,d} D_H / 2^{d/2},
 * H_{n,d} = H_{2^d} (Sylvester, entry (a,b) = (-1)^{popcount(a & b)})
 * Kronecker I_{n/2^d}, D_F = diag(+-1) from SplitMix64 stream seed (top bit of
 * value i), D_H from stream seed + 1.  F and H are orthogonal.  The sum runs
 * over the 2^d x 2^d entries A[i mod s + t s, j mod s' + u s'] (s = pm/2^d,
 * s' = pn/2^d), t outer, u inner, in binary64, then times the signs and 2^-d
 * (exact). */
double oracle_entry_f64(const oracle_source* src, int64_t i, int64_t j);
/* entry a(i,j) as it enters a binary32 strip. */
float oracle_entry_f32(const oracle_source* src, int64_t i, int64_t j);

/* Partial-pivot LU on the m x k column-major strip C (overwritten by the
 * basis B = C C[I,:]^{-1}).  I receives the k pivot rows in pivot order.
 * Returns the effective rank (k on success, t < k if the pivot of column t
 * fell below 64 u max|C|), or -1 if the first pivot that fails is exactly 0. */
int oracle_gepp_basis_f64(double* C, int64_t m, int k, int64_t* I, oracle_trace* tr);
int oracle_gepp_basis_f32(float* C, int64_t m, int k, int64_t* I, oracle_trace* tr);

/* maxvol on the m x k column-major strip C (overwritten by the final basis).
 * If have_init, I holds k distinct rows to warm-start from; else the start is
 * the partial-pivot LU.  Returns the number of swaps (>= 0), or a negative
 * status; *k_eff receives the rank actually used. */
int oracle_maxvol_f64(double* C, int64_t m, int k, int64_t* I, int have_init,
                      double tau, int max_swaps, int* k_eff, int* capped, oracle_trace* tr);
int oracle_maxvol_f32(float* C, int64_t m, int k, int64_t* I, int have_init,
                      double tau, int max_swaps, int* k_eff, int* capped, oracle_trace* tr);

/* Nucleus: G = A[I,J] (binary64), U = G^{-1} via partial-pivot LU.
 * G, U: k x k row-major.  Returns 0, or -2 if G is exactly singular. */
int oracle_nucleus(const oracle_source* src, const int64_t* I, const int64_t* J, int k,
                   double* G, double* U, double* cond1);

/* Sampled residual E_QS = A[Q,S] - A[Q,J] G^{-1} A[I,S] of the CUR factors
 * (G = A[I,J], applied through its partial-pivot LU) on the q x s
 * submatrix Q x S.
 * out[0] = ||E_QS||_F, out[1] = ||A_QS||_F, out[2] = mean, out[3] = variance,
 * out[4] = sqrt(mn/(qs)) ||E_QS||_F, out[5] = ||E_QS||_F / ||A_QS||_F. */
void oracle_residual(const oracle_source* src, int64_t m, int64_t n, int k,
                     const int64_t* I, const int64_t* J,
                     const int64_t* Q, int q, const int64_t* S, int s, double* out);

/* Full C-A / CUR run.  I, J: capacity kcap = max(k, k_max); G, U: kcap^2.
 * precision: 0 = binary64 strips, 1 = binary32 strips.
 * One sweep = column step (maxvol on A[:,J] -> I) then row step (maxvol on
 * A[I,:]^T -> J).  tol <= 0: exactly `sweeps` sweeps at rank k.
 * tol > 0: at each rank level run up to `sweeps` sweeps, stopping early once
 * a sweep after the first makes no swap; then estimate the error on Q x S;
 * if est_rel > tol and k < k_max, append the next k_step candidate columns
 * not already in J, forget I, and start the next level with a fresh LU. */
int oracle_ca_cur(const oracle_source* src, int64_t m, int64_t n, int k, int sweeps,
                  double tol, int precision, const oracle_options* opt,
                  int64_t* I, int64_t* J, double* G, double* U, oracle_result* res);

/* The fixed-rank CUR algorithms that the C-A tests of Section 12.2 compare
 * (tol is not used; every run is at fixed ranks):
 *   sweeps >= 1: k x k generator from `sweeps` C-A sweeps at width k from
 *     J0 = cand_cols[0..k) (Tests 2; sweeps = 1 with cur_rank: Tests 4);
 *   sweeps == 0: I = init_rows[0..k), J = J0 at random (Tests 1, the random
 *     p x q submatrix of Tests 3, the Primitive algorithm's random sets);
 *   cur_rank in [1, k): Cynical reduction to an r x r submatrix of locally
 *     maximal volume in the k x k generator, by up to inner_sweeps C-A
 *     sweeps on that block (J0 = its first r columns); 0: none;
 *   nucleus_rank in [1, k): nucleus U = (A[I,J])_r^+ (Primitive algorithm);
 *     0 or k: U = A[I,J]^{-1}.
 * The residual estimate as in oracle_ca_cur (explicit U when truncated).
 * Returns the status (0 ok, 2 swap cap, 3 numerical rank, -2 singular
 * generator or truncation, -6 non-finite entry, -1 invalid arguments). */
int oracle_cur_variant(const oracle_source* src, int64_t m, int64_t n, int k, int sweeps, int cur_rank,
                       int inner_sweeps, int nucleus_rank, int precision, const oracle_options* opt,
                       const int64_t* init_rows, int64_t* I, int64_t* J, double* G, double* U,
                       oracle_result* res);

/* One-sided Jacobi SVD of the k x k row-major G: W = G V with orthogonal
 * columns, V orthogonal, sv[j] = ||W[:,j]||.  Returns the sweeps taken. */
int oracle_svd_jacobi(const double* G, int k, double* W, double* V, double* sv);
/* G = A[I,J] and U = (G)_r^+ (rank-r truncated pseudo-inverse), k x k
 * row-major; cond1 = ||G||_1 ||U||_1.  Returns 0, or -2 if sigma_r = 0. */
int oracle_nucleus_trunc(const oracle_source* src, const int64_t* I, const int64_t* J, int k, int r,
                         double* G, double* U, double* cond1);
/* The sampled residual of oracle_residual with an explicit nucleus U. */
void oracle_residual_explicit(const oracle_source* src, int64_t m, int64_t n, int k,
                              const int64_t* I, const int64_t* J, const double* U,
                              const int64_t* Q, int q, const int64_t* S, int s, double* out);

/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the counter-based generator
 * used for default draws; value number `ctr` of stream `seed`. */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t ctr);
/* `cnt` distinct indices in [0, n), in draw order: value v of the stream is
 * mapped to floor(v * n / 2^64) and kept if not seen before. */
void oracle_draw_distinct(uint64_t seed, int64_t n, int64_t cnt, int64_t* out);

#ifdef __cplusplus
}
#endif
#endif
