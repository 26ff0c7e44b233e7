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
//      rotation, until no pair's cosine exceeds 16 r u) and sorts it;
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

constexpr int TS_ROWS = 256;          // rows of a TSQR block
constexpr int TS_THREADS = 512;       // 8 wavefronts of TS_RPW rows each
constexpr int TS_RPW = TS_ROWS / (TS_THREADS / 64);
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
    int32_t status;       // 0, -2 (a kept pivot of C or R^T at rounding level) or -6 (NaN / Inf)
    int32_t sweeps;       // Jacobi sweeps
    int64_t tick[6];      // wall clock at the core's stage boundaries (diagnostics)
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

DI int64_t wall_clock64() { return (int64_t)__builtin_amdgcn_s_memrealtime(); }

// Lane l's value of v (l uniform): two scalar reads, no LDS round trip.
DI double readlane_d(double v, int l)
{
    const int64_t b = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double((int64_t)(((uint64_t)hi << 32) | lo));
}

template <int CTRL>
DI double dpp_d(double v)
{
    const int64_t b = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((int64_t)(((uint64_t)hi << 32) | lo));
}

// Sum over each aligned group of 8 lanes, the same bits in all 8: lane i
// first adds lane 7 - i (row_half_mirror), then the partner in its quad at
// distance 2 and 1; every lane ends with the same two partial sums, added in
// either order.
DI double sum8(double v)
{
    v += dpp_d<0x141>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0xB1>(v);
    return v;
}

// Orders a wavefront's LDS accesses: its lanes run in lockstep and LDS
// serves one wavefront's requests in order, so program order suffices.
DI void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Householder QR (no pivoting) of 256-row blocks; block b of level L writes
// its k x k triangle to rows b k .. b k + k - 1 of the next level.  Two tall
// factors share a launch: blocks [0, a.nblk) take a, the rest take b.  The
// block is staged through LDS (coalesced loads), then lane c of wavefront w
// (8 wavefronts) keeps rows 32 w .. 32 w + 31 of column c in registers.
// Step j: lane j of each wavefront lays its rows of column j (zero above row
// j) out in LDS and every lane reads them back (broadcast reads); each
// wavefront forms its part of d_c = sum_{i >= j} x_ij x_ic, one LDS exchange
// sums the eight parts (d_j is the squared norm), and with v = x_j - alpha e_j
// the reflection updates column c > j by -beta v (d_c - alpha x_jc).  The
// updates are unconditional multiply-adds (a zero factor leaves a column
// unchanged), which keeps the rows in fixed registers; the pivot column keeps
// only its diagonal entry, in a register of its own.
__global__ __launch_bounds__(TS_THREADS) void tsqr_kernel(TallLevel a, TallLevel b, int k)
{
    extern __shared__ __align__(16) unsigned char ts_smem[];
    double* X = (double*)ts_smem;                     // staging: k columns of TS_LD
    double* part = X + TS_KMAX * TS_LD;               // [2][8][64] partial dot products
    double* xrow = part + 2 * 8 * 64;                 // [2][64] row j
    double* vcol = xrow + 2 * 64;                     // [TS_ROWS] column j, zero above row j
    const bool first = (int)blockIdx.x < a.nblk;
    const TallLevel L = first ? a : b;
    const int blk = first ? (int)blockIdx.x : (int)blockIdx.x - a.nblk;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t r0 = (int64_t)blk * TS_ROWS;
    const int nr = (int)(L.rows - r0 < TS_ROWS ? L.rows - r0 : TS_ROWS);
    for (int e = t; e < k * TS_ROWS; e += TS_THREADS) {
        const int c = e / TS_ROWS, i = e - c * TS_ROWS;
        X[c * TS_LD + i] = i < nr ? load_f(L.x, L.dtype, c * L.ld + r0 + i) : 0.0;
    }
    __syncthreads();
    double col[TS_RPW];
    {
        const double* xs = X + (lane < k ? lane : 0) * TS_LD + wave * TS_RPW;
#pragma unroll
        for (int i = 0; i < TS_RPW; ++i) col[i] = lane < k ? xs[i] : 0.0;
    }
    const int g0 = wave * TS_RPW;  // first row of this wavefront
    double* vw = vcol + g0;        // this wavefront's rows of column j
    double diag = 0.0;             // R[c][c] once column c has been the pivot
    for (int j = 0; j < k; ++j) {
        double* pb = part + (j & 1) * (8 * 64);
        double* xr = xrow + (j & 1) * 64;
        if (lane == j) {
#pragma unroll
            for (int i = 0; i < TS_RPW; ++i) vw[i] = g0 + i >= j ? col[i] : 0.0;
        }
        wave_lds_sync();
        double vj[TS_RPW];
#pragma unroll
        for (int i = 0; i < TS_RPW; ++i) vj[i] = vw[i];
        double d4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < TS_RPW; ++i) d4[i & 3] = fma(vj[i], col[i], d4[i & 3]);
        pb[wave * 64 + lane] = (d4[0] + d4[1]) + (d4[2] + d4[3]);
        const bool holds_j = wave == (j >> 5);  // the wavefront holding row j
        if (holds_j) {
            double x = 0.0;
#pragma unroll
            for (int i = 0; i < TS_RPW; ++i) x = g0 + i == j ? col[i] : x;
            xr[lane] = x;
        }
        __syncthreads();
        double nn = 0.0, dc = 0.0;
#pragma unroll
        for (int w = 0; w < 8; ++w) {
            nn += pb[w * 64 + j];
            dc += pb[w * 64 + lane];
        }
        const double x0 = xr[j], xjc = xr[lane];
        const double nrm = sqrt(nn);
        if (nrm == 0.0) continue;  // nothing to annihilate: R[j,j] = 0
        const double alpha = x0 >= 0.0 ? -nrm : nrm;
        const double v0 = x0 - alpha;
        const double beta = 1.0 / (nrm * (nrm + fabs(x0)));  // 2 / (v^T v)
        const double bw = (lane > j && lane < k) ? beta * (dc - alpha * xjc) : 0.0;
        if (holds_j) {
#pragma unroll
            for (int i = 0; i < TS_RPW; ++i) col[i] = fma(-(g0 + i == j ? v0 : vj[i]), bw, col[i]);
        } else {
#pragma unroll
            for (int i = 0; i < TS_RPW; ++i) col[i] = fma(-vj[i], bw, col[i]);
        }
        if (lane == j) diag = alpha;
    }
    // the k x k triangle, rows 0 .. k - 1 (wavefronts 0 and 1)
    if (g0 < k && lane < k) {
        const int64_t ld_out = (int64_t)L.nblk * k;
        double* o = L.out + lane * ld_out + (int64_t)blk * k;
#pragma unroll
        for (int i = 0; i < TS_RPW; ++i)
            if (g0 + i < k) o[g0 + i] = g0 + i < lane ? col[i] : (g0 + i == lane ? diag : 0.0);
    }
}

// Column-pivoted Householder QR of the k x k matrix A (column-major, ld
// CORE_LD, in LDS) by one wavefront, in place: A P = Q R with R left in A,
// its columns in pivot order, and piv[q] the original index of the column at
// position q.  At step j the remaining column of largest norm over rows j..
// takes position j (the lowest current position among equals), the norms
// recomputed each step.  Lane c keeps column c in registers for the whole
// factorisation together with its current position; the reflector's entries
// are read from the pivot lane's registers.
template <int KM>
DI void qrp_wave(double* A, int32_t* piv, double* vbuf, int k)
{
    const int lane = threadIdx.x & 63;
    double col[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) col[i] = (lane < k && i < k) ? A[(lane < k ? lane : 0) * CORE_LD + i] : 0.0;
    int pos = lane;
    bool done = lane >= k;
    double diag = 0.0;  // R's diagonal entry of this lane's column, once it is the pivot
    for (int j = 0; j < k; ++j) {
        double s = 0.0, xj = 0.0;
#pragma unroll
        for (int i = 0; i < KM; ++i) {
            const double x = i >= j ? col[i] : 0.0;
            s = fma(x, x, s);
            xj = i == j ? col[i] : xj;
        }
        // argmax: largest norm, then lowest current position
        double bv = done ? -1.0 : s;
        int bp = done ? (1 << 20) : pos, bl = lane;
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o);
            const int op = __shfl_xor(bp, o), ol = __shfl_xor(bl, o);
            if (ov > bv || (ov == bv && op < bp)) {
                bv = ov;
                bp = op;
                bl = ol;
            }
        }
        const int p = __builtin_amdgcn_readfirstlane(bl);
        const int ppos = __builtin_amdgcn_readfirstlane(bp);
        if (!done && pos == j) pos = ppos;  // the interchange moves position j's column to ppos
        if (lane == p) {
            pos = j;
            // the pivot column, zero above row j, for every lane to read
#pragma unroll
            for (int i = 0; i < KM; ++i) vbuf[i] = i >= j ? col[i] : 0.0;
        }
        wave_lds_sync();
        double vj[KM];
#pragma unroll
        for (int i = 0; i < KM; ++i) vj[i] = vbuf[i];
        const double nrm = sqrt(readlane_d(s, p));
        const double x0 = readlane_d(xj, p);
        if (nrm != 0.0) {
            const double alpha = x0 >= 0.0 ? -nrm : nrm;
            const double v0 = x0 - alpha;
            const double beta = 1.0 / (nrm * (nrm + fabs(x0)));
            double d4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < KM; ++i) d4[i & 3] = fma(vj[i], col[i], d4[i & 3]);
            // v^T x_c = sum_{i >= j} x_ip x_ic - alpha x_jc
            const double w = ((d4[0] + d4[1]) + (d4[2] + d4[3])) - alpha * xj;
            const double bw = (!done && lane != p) ? beta * w : 0.0;
#pragma unroll
            for (int i = 0; i < KM; ++i) col[i] = fma(-(i == j ? v0 : vj[i]), bw, col[i]);
            if (lane == p) diag = alpha;
        }
        if (lane == p) done = true;
        wave_lds_sync();  // every lane has read vbuf before the next pivot writes it
    }
    if (lane < k) {
        piv[pos] = lane;
#pragma unroll
        for (int i = 0; i < KM; ++i)
            if (i < k) A[pos * CORE_LD + i] = i < pos ? col[i] : (i == pos ? diag : 0.0);
    }
}

// B[:, c] := U^{-1} B[:, c] for the r x r upper triangle U of A (ld CORE_LD)
// and the r columns of B (ld CORE_LD): lane c of one wavefront holds column c
// in registers; every lane reads the same entries of U (broadcast loads).
template <int KM>
DI void core_backsolve(const double* A, double* B, int r, int c)
{
    if (c < r) {
        double b[KM];
#pragma unroll
        for (int i = 0; i < KM; ++i) b[i] = i < r ? B[c * CORE_LD + i] : 0.0;
#pragma unroll
        for (int i = KM - 1; i >= 0; --i) {
            if (i < r) {
                const double xi = b[i] / A[i * CORE_LD + i];
                b[i] = xi;
#pragma unroll
                for (int l = 0; l < i; ++l) b[l] = fma(-A[i * CORE_LD + l], xi, b[l]);
            }
        }
#pragma unroll
        for (int i = 0; i < KM; ++i)
            if (i < r) B[c * CORE_LD + i] = b[i];
    }
}

// One-sided Jacobi (Hestenes) on the r columns of Y (r x r, ld CORE_LD),
// accumulating the rotations in V: Y V = S_bar Sigma at convergence.
// Round-robin order over rp = r rounded up to even players (player 0 fixed,
// a bye when r is odd), so each round rotates disjoint pairs at once; pair g
// of a round belongs to the 8 threads 8 g .. 8 g + 7, each holding RPT rows
// (RPT = 8 covers r <= 64).  Rutishauser's rotation; a pair is rotated while
// its cosine exceeds 16 r u (the rounding of the r-term dot products is up to
// r u: a threshold at that level keeps rotating on noise).  At most 40 sweeps;
// returns the number run.
template <int RPT>
DI int jacobi_sweeps(double* Y, double* V, int r, int32_t* flag)
{
    const int t = threadIdx.x;
    const int rp = (r + 1) & ~1;
    const int g = t >> 3, sub = t & 7;
    const double rot_tol = 16.0 * r * 1.1102230246251565e-16;
    int sweep = 0;
    for (; sweep < 40; ++sweep) {
        if (t == 0) flag[0] = 0;
        __syncthreads();
        for (int round = 0; round < rp - 1; ++round) {
            int p = -1, q = -1;
            if (g < rp / 2) {
                const int s1 = g, s2 = rp - 1 - g;
                p = s1 == 0 ? 0 : 1 + (s1 - 1 + round) % (rp - 1);
                q = 1 + (s2 - 1 + round) % (rp - 1);
                if (p > q) {
                    const int x = p;
                    p = q;
                    q = x;
                }
            }
            // whole 8-lane groups take the branch together (DPP sums below)
            if (p >= 0 && q < r) {
                double yp[RPT], yq[RPT], vp[RPT], vq[RPT];
#pragma unroll
                for (int e = 0; e < RPT; ++e) {
                    const int i = sub + 8 * e < r ? sub + 8 * e : sub;
                    yp[e] = Y[p * CORE_LD + i];
                    yq[e] = Y[q * CORE_LD + i];
                    vp[e] = V[p * CORE_LD + i];
                    vq[e] = V[q * CORE_LD + i];
                }
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int e = 0; e < RPT; ++e)
                    if (sub + 8 * e < r) {
                        al = fma(yp[e], yp[e], al);
                        be = fma(yq[e], yq[e], be);
                        ga = fma(yp[e], yq[e], ga);
                    }
                al = sum8(al);
                be = sum8(be);
                ga = sum8(ga);
                if (fabs(ga) > rot_tol * sqrt(al * be) && ga != 0.0) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double tn = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double cs = 1.0 / sqrt(1.0 + tn * tn), sn = cs * tn;
#pragma unroll
                    for (int e = 0; e < RPT; ++e) {
                        const int i = sub + 8 * e;
                        if (i < r) {
                            Y[p * CORE_LD + i] = cs * yp[e] - sn * yq[e];
                            Y[q * CORE_LD + i] = sn * yp[e] + cs * yq[e];
                            V[p * CORE_LD + i] = cs * vp[e] - sn * vq[e];
                            V[q * CORE_LD + i] = sn * vp[e] + cs * vq[e];
                        }
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
    return sweep;
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
    double* w = nrm2 + 64;                   // 128: pivot columns of the two QRs
    int32_t* pc = (int32_t*)(w + 128);       // 64
    int32_t* pr = pc + 64;                   // 64
    int32_t* flag = pr + 64;                 // 68: rotations in the sweep; sort ranks
    const int t = threadIdx.x;
    if (t == 0) out->tick[0] = wall_clock64();
    // a NaN or Inf anywhere in C or R reaches the triangles
    int nonfinite = 0;
    for (int e = t; e < k * k; e += 256) {
        const int c = e / k, i = e - c * k;
        const double x1 = RC[c * k + i], x2 = RR[c * k + i];
        nonfinite |= !(fabs(x1) <= 1.7976931348623157e308) || !(fabs(x2) <= 1.7976931348623157e308);
        A1[c * CORE_LD + i] = x1;
        A2[c * CORE_LD + i] = x2;
    }
    if (__syncthreads_or(nonfinite)) {
        if (t == 0) out->status = -6;
        return;
    }
    // the two pivoted QRs run side by side on wavefronts 0 and 1
    if (k <= 32) {
        if (t < 64) qrp_wave<32>(A1, pc, w, k);
        else if (t < 128) qrp_wave<32>(A2, pr, w + 64, k);
    } else {
        if (t < 64) qrp_wave<64>(A1, pc, w, k);
        else if (t < 128) qrp_wave<64>(A2, pr, w + 64, k);
    }
    __syncthreads();
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
    if (t == 0) out->tick[1] = wall_clock64();
    // W~[a][b] = W[pc[a]][pr[b]], staged in Y (free until the middle factor)
    for (int e = t; e < k * k; e += 256) {
        const int c = e / k, b = e - c * k;
        Y[b * CORE_LD + c] = W[pc[c] * k + pr[b]];
    }
    __syncthreads();
    // B = R_C[:r,:] W~ (R_C upper triangular)
    for (int e = t; e < r * k; e += 256) {
        const int b = e / r, a = e - b * r;
        double s = 0.0;
        for (int c = a; c < k; ++c) s = fma(A1[c * CORE_LD + a], Y[b * CORE_LD + c], s);
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
    if (t == 0) out->tick[2] = wall_clock64();
    // one-sided Jacobi on the columns of Y: Y V = S_bar Sigma
    int sweep;
    if (r <= 16) sweep = jacobi_sweeps<2>(Y, V, r, flag);
    else if (r <= 32) sweep = jacobi_sweeps<4>(Y, V, r, flag);
    else sweep = jacobi_sweeps<8>(Y, V, r, flag);
    if (t == 0) out->tick[3] = wall_clock64();
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
    if (t == 0) out->tick[4] = wall_clock64();
    // the two triangular solves side by side on wavefronts 0 and 1
    if (r <= 32) {
        if (t < 64) core_backsolve<32>(A1, Y, r, t);
        else if (t < 128) core_backsolve<32>(A2, V, r, t - 64);
    } else {
        if (t < 64) core_backsolve<64>(A1, Y, r, t);
        else if (t < 128) core_backsolve<64>(A2, V, r, t - 64);
    }
    __syncthreads();
    for (int e = t; e < r * r; e += 256) {
        const int c = e / r, i = e - c * r;
        out->ms[i * r + flag[1 + c]] = Y[c * CORE_LD + i];
        out->nt[i * r + flag[1 + c]] = V[c * CORE_LD + i];
    }
    if (t == 0) {
        out->status = 0;
        out->sweeps = sweep;
        out->tick[5] = wall_clock64();
    }
}

// S (m x r, column-major) = (C P_C)[:, :r] M_S and
// T^T (r x n, row-major) = N^T (P_R^T R)[:r, :].  A block takes 64 rows of S
// (or columns of T^T), one per lane, and its four wavefronts split the r
// outputs of a row (output a to wavefront a mod 4); blocks [0, bs) cover S,
// the rest T^T.
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
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t i = (int64_t)(isS ? blockIdx.x : blockIdx.x - bs) * 64 + lane;
    if (isS ? i >= m : i >= n) return;
    const void* base = isS ? C : R;
    const int64_t ld = isS ? ldc : ldr;
    double v[TS_KMAX];
#pragma unroll
    for (int b = 0; b < TS_KMAX; ++b) v[b] = b < r ? load_f(base, dtype, P[b < r ? b : 0] * ld + i) : 0.0;
    double* out = isS ? S : Tt;
    const int64_t ldo = isS ? lds : ldt;
    for (int a = wave; a < r; a += 4) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int b = 0; b < TS_KMAX; b += 2) {
            if (b < r) s0 = fma(v[b], M[b * r + a], s0);
            if (b + 1 < r) s1 = fma(v[b + 1], M[(b + 1) * r + a], s1);
        }
        out[a * ldo + i] = s0 + s1;
    }
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------

size_t tsqr_lds_bytes() { return (size_t)(TS_KMAX * TS_LD + 2 * 8 * 64 + 2 * 64 + TS_ROWS) * sizeof(double); }
size_t core_lds_bytes() { return (size_t)(4 * TS_KMAX * CORE_LD + 64 + 128) * sizeof(double) + (64 + 64 + 68) * 4; }
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
    hipLaunchKernelGGL(tsqr_kernel, dim3((unsigned)(nblk_a + nblk_b)), dim3(TS_THREADS), tsqr_lds_bytes(), stream, a, b,
                       k);
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
    const int bs = (int)((m + 63) / 64), bt = (int)((n + 63) / 64);
    hipLaunchKernelGGL(topsvd_apply_kernel, dim3((unsigned)(bs + bt)), dim3(256), 0, stream, C, ldc, R, ldr, dtype, m,
                       n, r, (const CoreOut*)core, bs, S, lds, Tt, ldt);
    return hipGetLastError();
}

// Host view of the core kernel's output block.
void topsvd_core_fields(const void* host_copy, int32_t* status, int32_t* sweeps, const int32_t** pc,
                        const int32_t** pr, const double** sigma, const int64_t** ticks)
{
    const CoreOut* c = (const CoreOut*)host_copy;
    *ticks = c->tick;
    *status = c->status;
    *sweeps = c->sweeps;
    *pc = c->pc;
    *pr = c->pr;
    *sigma = c->sigma;
}

}  // namespace lra
