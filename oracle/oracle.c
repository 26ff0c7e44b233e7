/*
 * oracle.c -- plain CPU reference for C-A / CUR (see oracle.h).
 *
 * TEST INFRASTRUCTURE ONLY: linked by no product code.  Compiled with plain
 * gcc, -O2, no -ffast-math, no BLAS.  Every loop runs in index order so a
 * reader can check it against the paper by eye.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- entry sources (Section 2.1 notation; Cauchy-like kernels as in the
 * HSS experiments of Section 12.8; 1/|x - y| as the multipole kernel of
 * Section 9) ---------------------------------------------------------------- */

static double load_dense(const oracle_source* s, int64_t i, int64_t j)
{
    int64_t off = s->col_major ? j * s->lda + i : i * s->lda + j;
    return s->dtype == 0 ? (double)((const float*)s->a)[off] : ((const double*)s->a)[off];
}

static double load_pt(const void* p, int dtype, int64_t i)
{
    return dtype == 0 ? (double)((const float*)p)[i] : ((const double*)p)[i];
}

/* +-1 of value number idx of SplitMix64 stream `seed` (its top bit). */
static double pre_sign(uint64_t seed, int64_t idx)
{
    return (oracle_splitmix64(seed, (uint64_t)idx) >> 63) ? -1.0 : 1.0;
}

/* (F A H)_ij of the abridged scaled Hadamard pre-processing (oracle.h). */
static double preprocessed(const oracle_source* s, int64_t i, int64_t j)
{
    const int d = s->depth;
    const int64_t bm = s->pm >> d, bn = s->pn >> d;
    const int64_t ib = i / bm, ir = i % bm, jb = j / bn, jr = j % bn;
    double acc = 0.0;
    for (int64_t t = 0; t < ((int64_t)1 << d); ++t)
        for (int64_t u = 0; u < ((int64_t)1 << d); ++u) {
            const double v = load_dense(s, ir + t * bm, jr + u * bn);
            const int neg = (__builtin_popcountll((unsigned long long)(ib & t)) +
                             __builtin_popcountll((unsigned long long)(u & jb))) & 1;
            acc += neg ? -v : v;
        }
    return acc * pre_sign(s->seed, i) * pre_sign(s->seed + 1, j) * ldexp(1.0, -d);
}

double oracle_entry_f64(const oracle_source* s, int64_t i, int64_t j)
{
    if (s->kind == 0) return load_dense(s, i, j);
    if (s->kind == 3) return preprocessed(s, i, j);
    double d = load_pt(s->x, s->dtype, i) - load_pt(s->y, s->dtype, j);
    if (s->kind == 1) return 1.0 / d;
    d = fabs(d);
    return d == 0.0 ? 0.0 : 1.0 / d;
}

float oracle_entry_f32(const oracle_source* s, int64_t i, int64_t j)
{
    if (s->kind == 3) return (float)preprocessed(s, i, j);
    if (s->kind == 0) {
        int64_t off = s->col_major ? j * s->lda + i : i * s->lda + j;
        return s->dtype == 0 ? ((const float*)s->a)[off] : (float)((const double*)s->a)[off];
    }
    /* difference in binary64, then a binary32 reciprocal */
    double d = load_pt(s->x, s->dtype, i) - load_pt(s->y, s->dtype, j);
    if (s->kind == 1) return 1.0f / (float)d;
    d = fabs(d);
    return d == 0.0 ? 0.0f : 1.0f / (float)d;
}

/* ---- maxvol in both strip precisions -------------------------------------- */

#define REAL double
#define SFX _f64
#define UNIT_ROUNDOFF 0x1p-53
#define strip_entry_f64 oracle_entry_f64
#include "oracle_core.inc"
#undef REAL
#undef SFX
#undef UNIT_ROUNDOFF

#define REAL float
#define SFX _f32
#define UNIT_ROUNDOFF 0x1p-24
#define strip_entry_f32 oracle_entry_f32
#include "oracle_core.inc"
#undef REAL
#undef SFX
#undef UNIT_ROUNDOFF

/* ---- nucleus U = A[I,J]^{-1} (Section 12.2, eq. (eqtsts1)) ---------------- */

int oracle_nucleus(const oracle_source* src, const int64_t* I, const int64_t* J, int k,
                   double* G, double* U, double* cond1)
{
    double* LU = (double*)malloc(sizeof(double) * (size_t)k * (size_t)k);
    int* perm = (int*)malloc(sizeof(int) * (size_t)k);
    for (int s = 0; s < k; ++s)
        for (int t = 0; t < k; ++t) G[s * k + t] = oracle_entry_f64(src, I[s], J[t]);
    memcpy(LU, G, sizeof(double) * (size_t)k * (size_t)k);
    for (int s = 0; s < k; ++s) perm[s] = s;
    int rc = 0;
    for (int t = 0; t < k; ++t) {
        int best = t;
        for (int s = t + 1; s < k; ++s)
            if (fabs(LU[s * k + t]) > fabs(LU[best * k + t])) best = s;
        if (LU[best * k + t] == 0.0) { rc = -2; break; }
        if (best != t) {
            for (int c = 0; c < k; ++c) { double tmp = LU[t * k + c]; LU[t * k + c] = LU[best * k + c]; LU[best * k + c] = tmp; }
            int tp = perm[t]; perm[t] = perm[best]; perm[best] = tp;
        }
        for (int s = t + 1; s < k; ++s) {
            double l = LU[s * k + t] / LU[t * k + t];
            LU[s * k + t] = l;
            for (int c = t + 1; c < k; ++c) LU[s * k + c] -= l * LU[t * k + c];
        }
    }
    if (rc == 0) {
        /* column t of U solves G u = e_t: P G = L U_f, so L y = P e_t, U_f u = y */
        double* y = (double*)malloc(sizeof(double) * (size_t)k);
        for (int t = 0; t < k; ++t) {
            for (int s = 0; s < k; ++s) y[s] = perm[s] == t ? 1.0 : 0.0;
            for (int s = 0; s < k; ++s)
                for (int c = 0; c < s; ++c) y[s] -= LU[s * k + c] * y[c];
            for (int s = k - 1; s >= 0; --s) {
                for (int c = s + 1; c < k; ++c) y[s] -= LU[s * k + c] * y[c];
                y[s] /= LU[s * k + s];
            }
            for (int s = 0; s < k; ++s) U[s * k + t] = y[s];
        }
        free(y);
        /* exact 1-norm condition number ||G||_1 ||U||_1 */
        double ng = 0.0, nu = 0.0;
        for (int t = 0; t < k; ++t) {
            double cg = 0.0, cu = 0.0;
            for (int s = 0; s < k; ++s) { cg += fabs(G[s * k + t]); cu += fabs(U[s * k + t]); }
            if (cg > ng) ng = cg;
            if (cu > nu) nu = cu;
        }
        *cond1 = ng * nu;
    }
    free(LU); free(perm);
    return rc;
}

/* ---- a posteriori estimate on a q x s submatrix of E = A - C U R
 * (Appendix F; sample mean and variance of the entries as in its
 * hypothesis test).  U R[:,S] = G^{-1} R[:,S] is applied through the
 * partial-pivot LU of G = A[I,J] (forward and back substitution), which is
 * the same matrix as U times R[:,S] but keeps the residual accurate when G is
 * ill-conditioned. ---------------------------------------------------------- */

void oracle_residual(const oracle_source* src, int64_t m, int64_t n, int k,
                     const int64_t* I, const int64_t* J,
                     const int64_t* Q, int q, const int64_t* S, int s, double* out)
{
    double* LU = (double*)malloc(sizeof(double) * (size_t)k * (size_t)k);
    int* perm = (int*)malloc(sizeof(int) * (size_t)k);
    for (int a = 0; a < k; ++a) {
        perm[a] = a;
        for (int t = 0; t < k; ++t) LU[a * k + t] = oracle_entry_f64(src, I[a], J[t]);
    }
    for (int t = 0; t < k; ++t) {
        int best = t;
        for (int a = t + 1; a < k; ++a)
            if (fabs(LU[a * k + t]) > fabs(LU[best * k + t])) best = a;
        if (best != t) {
            for (int c = 0; c < k; ++c) { double tmp = LU[t * k + c]; LU[t * k + c] = LU[best * k + c]; LU[best * k + c] = tmp; }
            int tp = perm[t]; perm[t] = perm[best]; perm[best] = tp;
        }
        for (int a = t + 1; a < k; ++a) {
            double l = LU[a * k + t] / LU[t * k + t];
            LU[a * k + t] = l;
            for (int c = t + 1; c < k; ++c) LU[a * k + c] -= l * LU[t * k + c];
        }
    }
    /* W = G^{-1} R[:,S], one column b at a time: L y = P r_b, U_f w = y */
    double* W = (double*)malloc(sizeof(double) * (size_t)k * (size_t)s);
    double* y = (double*)malloc(sizeof(double) * (size_t)k);
    for (int b = 0; b < s; ++b) {
        for (int a = 0; a < k; ++a) y[a] = oracle_entry_f64(src, I[perm[a]], S[b]);
        for (int a = 0; a < k; ++a)
            for (int c = 0; c < a; ++c) y[a] -= LU[a * k + c] * y[c];
        for (int a = k - 1; a >= 0; --a) {
            for (int c = a + 1; c < k; ++c) y[a] -= LU[a * k + c] * y[c];
            y[a] /= LU[a * k + a];
        }
        for (int a = 0; a < k; ++a) W[a * s + b] = y[a];
    }
    double se = 0.0, sa = 0.0, sum = 0.0;
    double* E = (double*)malloc(sizeof(double) * (size_t)q * (size_t)s);
    for (int a = 0; a < q; ++a)
        for (int b = 0; b < s; ++b) {
            double cur = 0.0;
            for (int t = 0; t < k; ++t) cur += oracle_entry_f64(src, Q[a], J[t]) * W[t * s + b];
            double av = oracle_entry_f64(src, Q[a], S[b]);
            double e = av - cur;
            E[a * s + b] = e;
            se += e * e;
            sa += av * av;
            sum += e;
        }
    const double cnt = (double)q * (double)s;
    const double mean = sum / cnt;
    double var = 0.0;
    for (int e = 0; e < q * s; ++e) var += (E[e] - mean) * (E[e] - mean);
    var /= cnt;
    out[0] = sqrt(se);
    out[1] = sqrt(sa);
    out[2] = mean;
    out[3] = var;
    out[4] = sqrt((double)m * (double)n / cnt) * out[0];
    out[5] = out[1] > 0.0 ? out[0] / out[1] : (out[0] > 0.0 ? INFINITY : 0.0);
    free(LU); free(perm); free(W); free(y); free(E);
}

/* ---- driver ----------------------------------------------------------------- */

int oracle_ca_cur(const oracle_source* src, int64_t m, int64_t n, int k, int sweeps,
                  double tol, int precision, const oracle_options* opt,
                  int64_t* I, int64_t* J, double* G, double* U, oracle_result* res)
{
    memset(res, 0, sizeof(*res));
    res->trace.min_pivot_gap = res->trace.min_swap_gap = INFINITY;
    res->trace.min_stop_margin = res->trace.min_rank_margin = INFINITY;
    res->trace.min_tol_margin = INFINITY;
    if (k < 1 || k > m || k > n || sweeps < 1 || opt->n_cand < k || opt->q < 1 || opt->s < 1 ||
        opt->tau < 0.0) {
        res->status = -1;
        return -1;
    }
    if (precision == 1) return ca_cur_f32(src, m, n, k, sweeps, tol, opt, I, J, G, U, res);
    return ca_cur_f64(src, m, n, k, sweeps, tol, opt, I, J, G, U, res);
}

/* ---- the fixed-rank CUR algorithms of Section 12.2 (see oracle.h) ---------- */

int oracle_cur_variant(const oracle_source* src, int64_t m, int64_t n, int k, int sweeps, int cur_rank,
                       int inner_sweeps, int nucleus_rank, int precision, const oracle_options* opt,
                       const int64_t* init_rows, int64_t* I, int64_t* J, double* G, double* U,
                       oracle_result* res)
{
    memset(res, 0, sizeof(*res));
    res->trace.min_pivot_gap = res->trace.min_swap_gap = INFINITY;
    res->trace.min_stop_margin = res->trace.min_rank_margin = INFINITY;
    res->trace.min_tol_margin = INFINITY;
    if (k < 1 || k > m || k > n || sweeps < 0 || opt->n_cand < k || opt->q < 1 || opt->s < 1 ||
        opt->tau < 0.0 || cur_rank < 0 || cur_rank > k || nucleus_rank < 0 ||
        nucleus_rank > k || inner_sweeps < 1 || (sweeps == 0 && !init_rows)) {
        res->status = -1;
        return -1;
    }
    if (precision == 1)
        return cur_variant_f32(src, m, n, k, sweeps, cur_rank, inner_sweeps, nucleus_rank, opt, init_rows,
                               I, J, G, U, res);
    return cur_variant_f64(src, m, n, k, sweeps, cur_rank, inner_sweeps, nucleus_rank, opt, init_rows,
                           I, J, G, U, res);
}

/* ---- the Primitive algorithm's nucleus (Section 6.5): U = (M_{k,l})_r^+,
 * the pseudo-inverse of the rank-r truncation of the generator.  The SVD is
 * the one-sided Jacobi method (Hestenes 1958; Golub and Van Loan, Matrix
 * Computations, Section 8.6.3): W = G V, rotating column pairs (p, q) of W
 * and of V = I until every pair is orthogonal to working precision; then the
 * singular values are the column norms of W, u_j = W[:,j] / sigma_j, and
 * U = sum over the r largest sigma_j of v_j u_j^T / sigma_j.  Rows of U are
 * indexed like the columns of G (J) and its columns like the rows (I). ------ */

int oracle_svd_jacobi(const double* G, int k, double* W, double* V, double* sv)
{
    memcpy(W, G, sizeof(double) * (size_t)k * (size_t)k);
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) V[a * k + b] = a == b ? 1.0 : 0.0;
    const double eps = (double)k * 0x1p-53;
    int sweeps = 0;
    for (; sweeps < 100; ++sweeps) {
        int rotated = 0;
        for (int p = 0; p < k - 1; ++p)
            for (int q = p + 1; q < k; ++q) {
                double alpha = 0.0, beta = 0.0, gamma = 0.0;
                for (int i = 0; i < k; ++i) {
                    alpha += W[i * k + p] * W[i * k + p];
                    beta += W[i * k + q] * W[i * k + q];
                    gamma += W[i * k + p] * W[i * k + q];
                }
                if (!(fabs(gamma) > eps * sqrt(alpha * beta))) continue;
                rotated = 1;
                /* the rotation that zeroes the (p, q) entry of W^T W */
                const double zeta = (beta - alpha) / (2.0 * gamma);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double sn = c * t;
                for (int i = 0; i < k; ++i) {
                    const double wp = W[i * k + p], wq = W[i * k + q];
                    W[i * k + p] = c * wp - sn * wq;
                    W[i * k + q] = sn * wp + c * wq;
                    const double vp = V[i * k + p], vq = V[i * k + q];
                    V[i * k + p] = c * vp - sn * vq;
                    V[i * k + q] = sn * vp + c * vq;
                }
            }
        if (!rotated) break;
    }
    for (int j = 0; j < k; ++j) {
        double s2 = 0.0;
        for (int i = 0; i < k; ++i) s2 += W[i * k + j] * W[i * k + j];
        sv[j] = sqrt(s2);
    }
    return sweeps;
}

int oracle_nucleus_trunc(const oracle_source* src, const int64_t* I, const int64_t* J, int k, int r,
                         double* G, double* U, double* cond1)
{
    if (r < 1 || r > k) return -1;
    for (int s = 0; s < k; ++s)
        for (int t = 0; t < k; ++t) G[s * k + t] = oracle_entry_f64(src, I[s], J[t]);
    double* W = (double*)malloc(sizeof(double) * (size_t)k * (size_t)k);
    double* V = (double*)malloc(sizeof(double) * (size_t)k * (size_t)k);
    double* sv = (double*)malloc(sizeof(double) * (size_t)k);
    int* order = (int*)malloc(sizeof(int) * (size_t)k);
    oracle_svd_jacobi(G, k, W, V, sv);
    /* column indices by decreasing singular value (ties: smaller index) */
    for (int j = 0; j < k; ++j) order[j] = j;
    for (int a = 1; a < k; ++a) {
        const int v = order[a];
        int b = a - 1;
        while (b >= 0 && sv[order[b]] < sv[v]) { order[b + 1] = order[b]; --b; }
        order[b + 1] = v;
    }
    int rc = 0;
    if (!(sv[order[r - 1]] > 0.0)) rc = -2;  /* the rank-r truncation is singular */
    if (rc == 0) {
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) {
                double u = 0.0;
                for (int t = 0; t < r; ++t) {
                    const int j = order[t];
                    u += V[a * k + j] * (W[b * k + j] / (sv[j] * sv[j]));
                }
                U[a * k + b] = u;
            }
        double ng = 0.0, nu = 0.0;
        for (int t = 0; t < k; ++t) {
            double cg = 0.0, cu = 0.0;
            for (int s = 0; s < k; ++s) { cg += fabs(G[s * k + t]); cu += fabs(U[s * k + t]); }
            if (cg > ng) ng = cg;
            if (cu > nu) nu = cu;
        }
        *cond1 = ng * nu;
    }
    free(W); free(V); free(sv); free(order);
    return rc;
}

/* The a posteriori estimate of Appendix F for an explicit nucleus U (k x k,
 * rows indexed by J, columns by I): E_QS = A[Q,S] - A[Q,J] (U A[I,S]),
 * out[] as in oracle_residual. */
void oracle_residual_explicit(const oracle_source* src, int64_t m, int64_t n, int k,
                              const int64_t* I, const int64_t* J, const double* U,
                              const int64_t* Q, int q, const int64_t* S, int s, double* out)
{
    double* W = (double*)malloc(sizeof(double) * (size_t)k * (size_t)s);
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < s; ++b) {
            double w = 0.0;
            for (int c = 0; c < k; ++c) w += U[a * k + c] * oracle_entry_f64(src, I[c], S[b]);
            W[a * s + b] = w;
        }
    double se = 0.0, sa = 0.0, sum = 0.0;
    double* E = (double*)malloc(sizeof(double) * (size_t)q * (size_t)s);
    for (int a = 0; a < q; ++a)
        for (int b = 0; b < s; ++b) {
            double cur = 0.0;
            for (int t = 0; t < k; ++t) cur += oracle_entry_f64(src, Q[a], J[t]) * W[t * s + b];
            double av = oracle_entry_f64(src, Q[a], S[b]);
            double e = av - cur;
            E[a * s + b] = e;
            se += e * e;
            sa += av * av;
            sum += e;
        }
    const double cnt = (double)q * (double)s;
    const double mean = sum / cnt;
    double var = 0.0;
    for (int e = 0; e < q * s; ++e) var += (E[e] - mean) * (E[e] - mean);
    var /= cnt;
    out[0] = sqrt(se);
    out[1] = sqrt(sa);
    out[2] = mean;
    out[3] = var;
    out[4] = sqrt((double)m * (double)n / cnt) * out[0];
    out[5] = out[1] > 0.0 ? out[0] / out[1] : (out[0] > 0.0 ? INFINITY : 0.0);
    free(W); free(E);
}

/* ---- SplitMix64 ------------------------------------------------------------- */

uint64_t oracle_splitmix64(uint64_t seed, uint64_t ctr)
{
    uint64_t z = seed + (ctr + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void oracle_draw_distinct(uint64_t seed, int64_t n, int64_t cnt, int64_t* out)
{
    int64_t got = 0;
    for (uint64_t ctr = 0; got < cnt; ++ctr) {
        uint64_t v = oracle_splitmix64(seed, ctr);
        int64_t idx = (int64_t)(((unsigned __int128)v * (unsigned __int128)(uint64_t)n) >> 64);
        int dup = 0;
        for (int64_t e = 0; e < got; ++e) if (out[e] == idx) { dup = 1; break; }
        if (!dup) out[got++] = idx;
    }
}
