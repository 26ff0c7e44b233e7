// lra_topsvd.hip -- the transition from an LRA C W R to its top SVD
// (Appendix D, Algorithm D.1) on gfx950, binary64 throughout.
//
//   1. rank-revealing QR of C (m x k) and of R^T (n x k): each tall factor is
//      reduced to a k x k triangle by a tree of Householder QRs of 256-row
//      blocks held in LDS (TSQR: the triangle of a stack of triangles is the
//      triangle of the stacked rows, up to the signs of its rows), then one
//      workgroup takes the column-pivoted Householder QR of each triangle,
//      X P = Q_2 R_2.  The column norms a pivoted QR compares are invariant
//      under the orthogonal factor, so the pivots are those of the pivoted QR
//      of the tall factor itself;
//   2. the same workgroup forms the r x r middle factor
//      R_C[:r,:] P_C^T W P_R R_R[:r,:]^T, takes its SVD S_bar Sigma T_bar^T by
//      one-sided Jacobi rotations (parallel round-robin order, Rutishauser's
//      rotation) and sorts it;
//   3. the orthonormal factors follow without forming Q: the first r columns
//      of (C P_C) equal Q[:, :r] R_C[:r,:r], so S = (C P_C)[:, :r] M_S with
//      M_S = R_C[:r,:r]^{-1} S_bar, and likewise
//      T^T = N^T (P_R^T R)[:r, :] with N = R_R[:r,:r]^{-1} T_bar: one pass
//      over r columns of C and r rows of R, HBM-bound.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#define DI __device__ __forceinline__

namespace lra {

constexpr int TS_ROWS = 256;          // rows of a TSQR block (one per thread)
constexpr int TS_LD = TS_ROWS + 1;    // odd stride: column-parallel LDS reads spread over banks
constexpr int TS_KMAX = 64;
constexpr int CORE_LD = TS_KMAX + 1;

// A tall column-major factor of one TSQR level and the triangles it yields.
struct TallLevel {
    const void* x;    // rows x k, element (i, c) at x[c * ld + i]
    int64_t rows, ld;
    int32_t dtype;    // 0 float32, 1 float64 (levels after the first: 1)
    int32_t nblk;     // ceil(rows / TS_ROWS)
    double* out;      // (nblk k) x k column-major, ld = nblk k
};

// Outputs of the core kernel (device workspace).
struct CoreOut {
    int32_t status;       // 0, or -2 (a kept pivot of C or R^T is at rounding level)
    int32_t sweeps;       // Jacobi sweeps
    int32_t pc[TS_KMAX];  // column pivots of C
    int32_t pr[TS_KMAX];  // column pivots of R^T
    double sigma[TS_KMAX];
    double ms[TS_KMAX * TS_KMAX];  // M_S, r x r row-major
    double nt[TS_KMAX * TS_KMAX];  // N, r x r row-major (T^T = N^T (P_R^T R)[:r, :])
};

DI double load_f(const void* p, int dtype, int64_t off)
{
    return dtype == 0 ? (double)((const float*)p)[off] : ((const double*)p)[off];
}

DI double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Householder QR (no pivoting) of 256-row blocks; block b of level L writes
// its k x k triangle to rows b k .. b k + k - 1 of the next level.  Two tall
// factors share a launch: blocks [0, a.nblk) take a, the rest take b.
__global__ __launch_bounds__(256) void tsqr_kernel(TallLevel a, TallLevel b, int k)
{
    extern __shared__ __align__(16) unsigned char ts_smem[];
    double* X = (double*)ts_smem;                 // k columns of TS_LD
    double* part = X + TS_KMAX * TS_LD;           // 4 x 64 partial dot products
    double* wv = part + 4 * 64;                   // 64 reduced dot products
    double* red = wv + 64;                        // 4 wave sums
    const bool first = (int)blockIdx.x < a.nblk;
    const TallLevel L = first ? a : b;
    const int blk = first ? (int)blockIdx.x : (int)blockIdx.x - a.nblk;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t r0 = (int64_t)blk * TS_ROWS;
    const int nr = (int)(L.rows - r0 < TS_ROWS ? L.rows - r0 : TS_ROWS);
    for (int c = 0; c < k; ++c)
        X[c * TS_LD + t] = t < nr ? load_f(L.x, L.dtype, c * L.ld + r0 + t) : 0.0;
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        // norm of column j over rows j..
        const double xj = X[j * TS_LD + t];
        double sq = wave_sum(t >= j ? xj * xj : 0.0);
        if (lane == 0) red[wave] = sq;
        __syncthreads();
        const double nn = red[0] + red[1] + red[2] + red[3];
        const double x0 = X[j * TS_LD + j];
        const double nrm = sqrt(nn);
        if (nrm == 0.0) {  // nothing to annihilate: R[j,j] = 0, no reflection
            __syncthreads();
            continue;
        }
        const double alpha = x0 >= 0.0 ? -nrm : nrm;
        const double v0 = x0 - alpha;
        const double beta = 1.0 / (nrm * (nrm + fabs(x0)));  // 2 / (v^T v)
        // w_c = v^T X[j.., c] for c > j: 64 columns x 4 row segments
        {
            const int c = j + 1 + lane;
            double p = 0.0;
            if (c < k) {
                const int lo = wave * 64 > j ? wave * 64 : j;
                for (int i = lo; i < wave * 64 + 64; ++i) {
                    const double vi = i == j ? v0 : X[j * TS_LD + i];
                    p = fma(vi, X[c * TS_LD + i], p);
                }
            }
            part[wave * 64 + lane] = p;
        }
        __syncthreads();
        if (t < 64) wv[t] = part[t] + part[64 + t] + part[128 + t] + part[192 + t];
        __syncthreads();
        if (t >= j) {
            const double vi = t == j ? v0 : xj;
            const double bv = beta * vi;
            for (int c = j + 1; c < k; ++c) X[c * TS_LD + t] -= bv * wv[c - j - 1];
            X[j * TS_LD + t] = t == j ? alpha : 0.0;
        }
        __syncthreads();
    }
    // the k x k triangle (rows past the block's height are zero rows)
    const int64_t ld_out = (int64_t)L.nblk * k;
    for (int e = t; e < k * k; e += 256) {
        const int c = e / k, i = e - c * k;
        L.out[c * ld_out + (int64_t)blk * k + i] = i <= c ? X[c * TS_LD + i] : 0.0;
    }
}

// Column-pivoted Householder QR of the k x k matrix A (column-major, ld
// CORE_LD) in LDS, in place: A P = Q R with R left in A's upper triangle.
// At step j the remaining column of largest norm over rows j.. moves to
// position j (lowest index among equals), the norms recomputed each step.
DI void core_qrp(double* A, int32_t* piv, double* nrm2, double* w, int k)
{
    const int t = threadIdx.x;
    if (t < k) piv[t] = t;
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        if (t >= j && t < k) {
            double s = 0.0;
            for (int i = j; i < k; ++i) s = fma(A[t * CORE_LD + i], A[t * CORE_LD + i], s);
            nrm2[t] = s;
        }
        __syncthreads();
        if (t < 64) {  // wavefront 0: argmax, lowest index among equals
            double v = (t >= j && t < k) ? nrm2[t] : -1.0;
            int ix = t;
            for (int o = 32; o > 0; o >>= 1) {
                const double ov = __shfl_xor(v, o);
                const int oi = __shfl_xor(ix, o);
                if (ov > v || (ov == v && oi < ix)) {
                    v = ov;
                    ix = oi;
                }
            }
            if (t == 0) w[64] = (double)ix;
        }
        __syncthreads();
        const int p = (int)w[64];
        if (p != j) {
            if (t < k) {
                const double s = A[j * CORE_LD + t];
                A[j * CORE_LD + t] = A[p * CORE_LD + t];
                A[p * CORE_LD + t] = s;
            }
            if (t == 0) {
                const int32_t s = piv[j];
                piv[j] = piv[p];
                piv[p] = s;
                const double q = nrm2[j];
                nrm2[j] = nrm2[p];
                nrm2[p] = q;
            }
        }
        __syncthreads();
        const double nrm = sqrt(nrm2[j]);
        const double x0 = A[j * CORE_LD + j];
        if (nrm != 0.0) {
            const double alpha = x0 >= 0.0 ? -nrm : nrm;
            const double v0 = x0 - alpha;
            const double beta = 1.0 / (nrm * (nrm + fabs(x0)));
            if (t > j && t < k) {
                double s = v0 * A[t * CORE_LD + j];
                for (int i = j + 1; i < k; ++i) s = fma(A[j * CORE_LD + i], A[t * CORE_LD + i], s);
                w[t] = s;
            }
            __syncthreads();
            // 256 threads: column c = j + 1 + (t & 63), rows j + (t >> 6) + 4 q
            const int c = j + 1 + (t & 63);
            if (c < k)
                for (int i = j + (t >> 6); i < k; i += 4) {
                    const double vi = i == j ? v0 : A[j * CORE_LD + i];
                    A[c * CORE_LD + i] -= beta * vi * w[c];
                }
            __syncthreads();
            if (t >= j && t < k) A[j * CORE_LD + t] = t == j ? alpha : 0.0;
        }
        __syncthreads();
    }
}

// x := U^{-1} x for the r x r upper triangle U of A (ld CORE_LD), columns of
// B (ld CORE_LD, r columns) in place: one thread per column.
DI void core_backsolve(const double* A, double* B, int r)
{
    const int c = threadIdx.x;
    if (c < r)
        for (int i = r - 1; i >= 0; --i) {
            double s = B[c * CORE_LD + i];
            for (int l = i + 1; l < r; ++l) s = fma(-A[l * CORE_LD + i], B[c * CORE_LD + l], s);
            B[c * CORE_LD + i] = s / A[i * CORE_LD + i];
        }
    __syncthreads();
}

// One workgroup: pivoted QR of both triangles, the middle factor, its SVD and
// the small factors of the output.
__global__ __launch_bounds__(256) void topsvd_core_kernel(const double* RC, const double* RR, const double* W, int k,
                                                          int r, double rank_lim, CoreOut* out)
{
    extern __shared__ __align__(16) unsigned char cs_smem[];
    double* A1 = (double*)cs_smem;           // R_C, then its pivoted triangle
    double* A2 = A1 + TS_KMAX * CORE_LD;     // R_R, likewise
    double* B = A2 + TS_KMAX * CORE_LD;      // R_C[:r,:] P_C^T W P_R (r x k), then the rotations V
    double* Y = B + TS_KMAX * CORE_LD;       // middle factor, Jacobi iterate (r x r)
    double* nrm2 = Y + TS_KMAX * CORE_LD;    // 64
    double* w = nrm2 + 64;                   // 72
    int32_t* pc = (int32_t*)(w + 72);        // 64
    int32_t* pr = pc + 64;                   // 64
    int32_t* flag = pr + 64;                 // 68: rotations in the sweep; sort ranks
    const int t = threadIdx.x;
    for (int e = t; e < k * k; e += 256) {
        const int c = e / k, i = e - c * k;
        A1[c * CORE_LD + i] = RC[c * k + i];
        A2[c * CORE_LD + i] = RR[c * k + i];
    }
    __syncthreads();
    core_qrp(A1, pc, nrm2, w, k);
    core_qrp(A2, pr, nrm2, w, k);
    if (t < k) {
        out->pc[t] = pc[t];
        out->pr[t] = pr[t];
    }
    // a kept pivot at the rounding level of the QR (rank_lim = max(m, n) u):
    // the requested rank exceeds the factors' numerical rank
    const double tc = rank_lim * fabs(A1[0]), tr = rank_lim * fabs(A2[0]);
    bool bad = false;
    for (int j = 0; j < r; ++j)
        bad = bad || !(fabs(A1[j * CORE_LD + j]) > tc) || !(fabs(A2[j * CORE_LD + j]) > tr);
    if (bad) {
        if (t == 0) out->status = -2;
        return;
    }
    // B = R_C[:r,:] W~ with W~[a][b] = W[pc[a]][pr[b]] (R_C upper triangular)
    for (int e = t; e < r * k; e += 256) {
        const int b = e / r, a = e - b * r;
        double s = 0.0;
        for (int c = a; c < k; ++c) s = fma(A1[c * CORE_LD + a], W[pc[c] * k + pr[b]], s);
        B[b * CORE_LD + a] = s;
    }
    __syncthreads();
    // middle Y = B R_R[:r,:]^T: Y[a][b] = sum_{c >= b} B[a][c] R_R[b][c]
    for (int e = t; e < r * r; e += 256) {
        const int b = e / r, a = e - b * r;
        double s = 0.0;
        for (int c = b; c < k; ++c) s = fma(B[c * CORE_LD + a], A2[c * CORE_LD + b], s);
        Y[b * CORE_LD + a] = s;
    }
    __syncthreads();
    double* V = B;
    for (int e = t; e < r * r; e += 256) {
        const int b = e / r, a = e - b * r;
        V[b * CORE_LD + a] = a == b ? 1.0 : 0.0;
    }
    __syncthreads();
    // one-sided Jacobi on the columns of Y: Y V = S_bar Sigma.  Round-robin
    // order over rp = r rounded up to even players (a bye when r is odd);
    // pair g of a round is handled by the 8 threads 8 g .. 8 g + 7.
    const int rp = (r + 1) & ~1;
    const int g = t >> 3, sub = t & 7;
    int sweep = 0;
    for (; sweep < 40; ++sweep) {
        if (t == 0) flag[0] = 0;
        __syncthreads();
        for (int round = 0; round < rp - 1; ++round) {
            int p = -1, q = -1;
            if (g < rp / 2) {
                // player 0 fixed, the others rotate
                auto pos = [&](int s) { return s == 0 ? 0 : 1 + (s - 1 + round) % (rp - 1); };
                p = pos(g);
                q = pos(rp - 1 - g);
                if (p > q) {
                    const int s = p;
                    p = q;
                    q = s;
                }
            }
            if (p >= 0 && q < r) {
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = sub; i < r; i += 8) {
                    const double yp = Y[p * CORE_LD + i], yq = Y[q * CORE_LD + i];
                    al = fma(yp, yp, al);
                    be = fma(yq, yq, be);
                    ga = fma(yp, yq, ga);
                }
                for (int o = 4; o > 0; o >>= 1) {
                    al += __shfl_xor(al, o);
                    be += __shfl_xor(be, o);
                    ga += __shfl_xor(ga, o);
                }
                if (fabs(ga) > r * 2.220446049250313e-16 * sqrt(al * be) && ga != 0.0) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double tn = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double cs = 1.0 / sqrt(1.0 + tn * tn), sn = cs * tn;
                    for (int i = sub; i < r; i += 8) {
                        const double yp = Y[p * CORE_LD + i], yq = Y[q * CORE_LD + i];
                        Y[p * CORE_LD + i] = cs * yp - sn * yq;
                        Y[q * CORE_LD + i] = sn * yp + cs * yq;
                        const double vp = V[p * CORE_LD + i], vq = V[q * CORE_LD + i];
                        V[p * CORE_LD + i] = cs * vp - sn * vq;
                        V[q * CORE_LD + i] = sn * vp + cs * vq;
                    }
                    if (sub == 0) flag[0] = 1;
                }
            }
            __syncthreads();
        }
        const int any = flag[0];
        __syncthreads();
        if (!any) break;
    }
    // singular values, descending (ties: lower index first)
    if (t < r) {
        double s = 0.0;
        for (int i = 0; i < r; ++i) s = fma(Y[t * CORE_LD + i], Y[t * CORE_LD + i], s);
        nrm2[t] = sqrt(s);
    }
    __syncthreads();
    if (t < r) {
        int rank = 0;
        for (int j = 0; j < r; ++j) rank += nrm2[j] > nrm2[t] || (nrm2[j] == nrm2[t] && j < t);
        flag[1 + t] = rank;
    }
    __syncthreads();
    // S_bar = Y Sigma^{-1}; M_S = R_C[:r,:r]^{-1} S_bar and N = R_R[:r,:r]^{-1} V
    // in place, column by column; the sort permutes columns on the way out
    for (int e = t; e < r * r; e += 256) {
        const int c = e / r, i = e - c * r;
        const double s = nrm2[c];
        Y[c * CORE_LD + i] = s > 0.0 ? Y[c * CORE_LD + i] / s : 0.0;
    }
    if (t < r) out->sigma[flag[1 + t]] = nrm2[t];
    __syncthreads();
    core_backsolve(A1, Y, r);
    core_backsolve(A2, V, r);
    for (int e = t; e < r * r; e += 256) {
        const int c = e / r, i = e - c * r;
        out->ms[i * r + flag[1 + c]] = Y[c * CORE_LD + i];
        out->nt[i * r + flag[1 + c]] = V[c * CORE_LD + i];
    }
    if (t == 0) {
        out->status = 0;
        out->sweeps = sweep;
    }
}

// S (m x r, column-major) = (C P_C)[:, :r] M_S and
// T^T (r x n, row-major) = N^T (P_R^T R)[:r, :]: thread per row of S or column
// of T^T; blocks [0, bs) cover S, the rest T^T.
__global__ __launch_bounds__(256) void topsvd_apply_kernel(const void* C, int64_t ldc, const void* R, int64_t ldr,
                                                           int dtype, int64_t m, int64_t n, int r,
                                                           const CoreOut* co, int bs, double* S, int64_t lds,
                                                           double* Tt, int64_t ldt)
{
    __shared__ double M[TS_KMAX * TS_KMAX];
    __shared__ int32_t P[TS_KMAX];
    if (co->status != 0) return;  // rank loss: outputs untouched
    const bool isS = (int)blockIdx.x < bs;
    const double* src = isS ? co->ms : co->nt;
    for (int e = threadIdx.x; e < r * r; e += 256) M[e] = src[e];
    if ((int)threadIdx.x < r) P[threadIdx.x] = isS ? co->pc[threadIdx.x] : co->pr[threadIdx.x];
    __syncthreads();
    const int64_t i = (int64_t)(isS ? blockIdx.x : blockIdx.x - bs) * 256 + threadIdx.x;
    if (isS ? i >= m : i >= n) return;
    double v[TS_KMAX];
#pragma unroll
    for (int b = 0; b < TS_KMAX; ++b)
        if (b < r) v[b] = isS ? load_f(C, dtype, P[b] * ldc + i) : load_f(R, dtype, P[b] * ldr + i);
    for (int a = 0; a < r; ++a) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < TS_KMAX; ++b)
            if (b < r) s = fma(v[b], M[b * r + a], s);
        if (isS)
            S[a * lds + i] = s;
        else
            Tt[a * ldt + i] = s;
    }
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------

size_t tsqr_lds_bytes() { return (size_t)(TS_KMAX * TS_LD + 4 * 64 + 64 + 8) * sizeof(double); }
size_t core_lds_bytes() { return (size_t)(4 * TS_KMAX * CORE_LD + 64 + 72) * sizeof(double) + (64 + 64 + 68) * 4; }
size_t core_out_bytes() { return sizeof(CoreOut); }

hipError_t topsvd_set_attributes()
{
    hipError_t e = hipFuncSetAttribute((const void*)tsqr_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)tsqr_lds_bytes());
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)topsvd_core_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)core_lds_bytes());
}

// One TSQR level of each of the two factors (a factor with nblk 0 is skipped).
hipError_t launch_tsqr(const void* xa, int64_t rows_a, int64_t lda, int dta, int nblk_a, double* out_a,
                       const void* xb, int64_t rows_b, int64_t ldb, int dtb, int nblk_b, double* out_b, int k,
                       hipStream_t stream)
{
    TallLevel a{xa, rows_a, lda, dta, nblk_a, out_a};
    TallLevel b{xb, rows_b, ldb, dtb, nblk_b, out_b};
    hipLaunchKernelGGL(tsqr_kernel, dim3((unsigned)(nblk_a + nblk_b)), dim3(256), tsqr_lds_bytes(), stream, a, b, k);
    return hipGetLastError();
}

hipError_t launch_topsvd_core(const double* RC, const double* RR, const double* W, int k, int r, double rank_lim,
                              void* out, hipStream_t stream)
{
    hipLaunchKernelGGL(topsvd_core_kernel, dim3(1), dim3(256), core_lds_bytes(), stream, RC, RR, W, k, r, rank_lim,
                       (CoreOut*)out);
    return hipGetLastError();
}

hipError_t launch_topsvd_apply(const void* C, int64_t ldc, const void* R, int64_t ldr, int dtype, int64_t m,
                               int64_t n, int r, const void* core, double* S, int64_t lds, double* Tt, int64_t ldt,
                               hipStream_t stream)
{
    const int bs = (int)((m + 255) / 256), bt = (int)((n + 255) / 256);
    hipLaunchKernelGGL(topsvd_apply_kernel, dim3((unsigned)(bs + bt)), dim3(256), 0, stream, C, ldc, R, ldr, dtype, m,
                       n, r, (const CoreOut*)core, bs, S, lds, Tt, ldt);
    return hipGetLastError();
}

// Host view of the core kernel's output block.
void topsvd_core_fields(const void* host_copy, int32_t* status, int32_t* sweeps, const int32_t** pc,
                        const int32_t** pr, const double** sigma)
{
    const CoreOut* c = (const CoreOut*)host_copy;
    *status = c->status;
    *sweeps = c->sweeps;
    *pc = c->pc;
    *pr = c->pr;
    *sigma = c->sigma;
}

}  // namespace lra
