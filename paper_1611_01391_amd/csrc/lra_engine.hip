// lra_engine.hip -- gfx950 kernels of the C-A / CUR library.
//
// One persistent kernel runs whole C-A / CUR problems.  A problem is owned by
// a *team* of workgroups; every pivot decision (a partial-pivot LU step or a
// maxvol swap) is one team-wide argmax: each workgroup reduces its rows
// (wavefront shuffles, then LDS), publishes its best key and candidate row in
// a slot in global memory, and after one team barrier every workgroup reduces
// the slots and reads the winning row.  A team of one workgroup needs no
// barrier at all.  A workgroup keeps its rows of the strip in LDS when they
// fit, else in a global strip buffer.
//
// Method (arXiv:1611.01391): C-A iterations of Section 6.5 in the dual order
// of Remark rec-atnsr (vertical step first); each step picks a k x k
// submatrix of locally maximal volume (Section 6.5, footnote on the volume;
// cost model Remark "re vlmmx") by maxvol: partial-pivot LU start, basis
// B = C C[I,:]^{-1}, swap while max|B| > 1 + tau (|det| grows by |B_ij| per
// swap); nucleus U = A[I,J]^{-1} (Section 12.2, eq. (eqtsts1)); sampled
// residual on a q x s submatrix (Appendix F); rank growth on failure
// (Algorithm 5.1, footnotes).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lra_internal.h"

namespace lra {

constexpr int NWAVE = NT / 64;
#define AGENT __HIP_MEMORY_SCOPE_AGENT

// ----------------------------------------------------------------------------
// entries
// ----------------------------------------------------------------------------

__device__ __forceinline__ double load_elem(const void* p, int dtype, int64_t off)
{
    return dtype == 0 ? (double)((const float*)p)[off] : ((const double*)p)[off];
}

// Entry from a coordinate difference d (binary64): 1/d or 1/|d| (0 at d = 0).
template <typename T>
__device__ __forceinline__ T kernel_entry(int kind, double d);

template <>
__device__ __forceinline__ double kernel_entry<double>(int kind, double d)
{
    if (kind == 1) return 1.0 / d;
    double ad = fabs(d);
    return ad == 0.0 ? 0.0 : 1.0 / ad;
}

template <>
__device__ __forceinline__ float kernel_entry<float>(int kind, double d)
{
    if (kind == 1) return 1.0f / (float)d;
    double ad = fabs(d);
    return ad == 0.0 ? 0.0f : 1.0f / (float)ad;
}

template <typename T>
__device__ __forceinline__ T dense_entry(const DevSource& s, int64_t i, int64_t j);

template <>
__device__ __forceinline__ double dense_entry<double>(const DevSource& s, int64_t i, int64_t j)
{
    int64_t off = s.col_major ? j * s.lda + i : i * s.lda + j;
    return load_elem(s.a, s.dtype, off);
}

template <>
__device__ __forceinline__ float dense_entry<float>(const DevSource& s, int64_t i, int64_t j)
{
    int64_t off = s.col_major ? j * s.lda + i : i * s.lda + j;
    return s.dtype == 0 ? ((const float*)s.a)[off] : (float)((const double*)s.a)[off];
}

template <typename T>
__device__ __forceinline__ T entry_t(const DevSource& s, int64_t i, int64_t j)
{
    if (s.kind == 0) return dense_entry<T>(s, i, j);
    double d = load_elem(s.x, s.dtype, i) - load_elem(s.y, s.dtype, j);
    return kernel_entry<T>(s.kind, d);
}

__device__ __forceinline__ double entry64(const DevSource& s, int64_t i, int64_t j)
{
    return entry_t<double>(s, i, j);
}

// ----------------------------------------------------------------------------
// argmax keys: larger |value|, then smaller row, then smaller column
// ----------------------------------------------------------------------------

struct Key {
    double v;
    int64_t r;
    int32_t c;
    int32_t w;  // owning workgroup (carried, not compared)
};

__device__ __forceinline__ Key key_none()
{
    Key k;
    k.v = -1.0;
    k.r = INT64_MAX;
    k.c = INT32_MAX;
    k.w = -1;
    return k;
}

__device__ __forceinline__ bool kbetter(const Key& a, const Key& b)
{
    return a.v > b.v || (a.v == b.v && (a.r < b.r || (a.r == b.r && a.c < b.c)));
}

__device__ __forceinline__ Key wave_reduce(Key k)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        Key o;
        o.v = __shfl_xor(k.v, off);
        o.r = __shfl_xor(k.r, off);
        o.c = __shfl_xor(k.c, off);
        o.w = __shfl_xor(k.w, off);
        if (kbetter(o, k)) k = o;
    }
    return k;
}

// ----------------------------------------------------------------------------
// shared memory of one workgroup
// ----------------------------------------------------------------------------

template <typename T, int KMAX>
struct Smem {
    int64_t I[KMAX], J[KMAX], prevI[KMAX], prevJ[KMAX];
    double LU[KMAX * KMAX];   // k x k work matrix (row stride KMAX)
    double red[NT];           // fixed-order reductions
    double pts[KMAX];         // coordinates of the fixed index set (generated sources)
    T g[KMAX];                // swap update vector
    T pay[KMAX];              // candidate / winning row
    int32_t perm[KMAX];
    Key kred[NWAVE];
    Key win;
    // problem state (mirrors TaskState)
    int32_t k, phase, sweep_in_level, status, warn, have_I, had_I_sweep, k_sweep_start;
    int32_t swaps_total, sweeps_done, phases_run;
    int64_t cand_next, entries_read;
    double est_rel, est_abs, mean, var, cond1;
    int32_t flag, fetch, ok, kstep_res;
    double thresh;
};

template <typename T, int KMAX>
__device__ __forceinline__ Key block_reduce(Key k, Smem<T, KMAX>& sm)
{
    k = wave_reduce(k);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sm.kred[w] = k;
    __syncthreads();
    Key b = sm.kred[0];
#pragma unroll
    for (int i = 1; i < NWAVE; ++i)
        if (kbetter(sm.kred[i], b)) b = sm.kred[i];
    __syncthreads();
    return b;
}

// ----------------------------------------------------------------------------
// team synchronisation
// ----------------------------------------------------------------------------

struct Team {
    uint8_t* ctl;
    int size;
    int rank;
    uint32_t epoch;
    bool failed;
    uint32_t* err;
    int64_t timeout;
};

__device__ __forceinline__ uint8_t* slot_ptr(const Team& tm, int parity, int wg)
{
    return tm.ctl + CTL_HDR + (int64_t)(parity * tm.size + wg) * SLOT_STRIDE;
}

// Team barrier on a monotone arrival counter; thread 0 waits with a time-out.
template <typename T, int KMAX>
__device__ void team_barrier(Team& tm, Smem<T, KMAX>& sm)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t* ctr = (uint32_t*)tm.ctl;
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, AGENT);
        const uint32_t target = (tm.epoch + 1) * (uint32_t)tm.size;
        const int64_t t0 = wall_clock64();
        int bad = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (wall_clock64() - t0 > tm.timeout) {
                atomicOr(tm.err, 1u);
                bad = 1;
                break;
            }
        }
        sm.flag = bad;
    }
    __syncthreads();
    tm.epoch++;
    if (sm.flag) tm.failed = true;
}

// Team-wide argmax: publish this workgroup's best key and its candidate row
// (sm.pay[0..n)), then every workgroup reduces all slots and loads the
// winning row into sm.pay.  With one workgroup the local result is final.
template <typename T, int KMAX>
__device__ Key team_argmax(Team& tm, Smem<T, KMAX>& sm, Key mine, int n)
{
    if (tm.size == 1) return mine;
    const int par = tm.epoch & 1;
    uint8_t* my = slot_ptr(tm, par, tm.rank);
    double* mypay = (double*)(my + 32);
    if (threadIdx.x < n)
        __hip_atomic_store(mypay + threadIdx.x, (double)sm.pay[threadIdx.x], __ATOMIC_RELAXED, AGENT);
    if (threadIdx.x == 0) {
        __hip_atomic_store((double*)my, mine.v, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store((int64_t*)(my + 8), mine.r, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store((int32_t*)(my + 16), mine.c, __ATOMIC_RELAXED, AGENT);
    }
    team_barrier(tm, sm);
    if (tm.failed) return key_none();
    Key best = key_none();
    for (int w = threadIdx.x; w < tm.size; w += NT) {
        const uint8_t* sp = slot_ptr(tm, par, w);
        Key o;
        o.v = __hip_atomic_load((double*)sp, __ATOMIC_RELAXED, AGENT);
        o.r = __hip_atomic_load((int64_t*)(sp + 8), __ATOMIC_RELAXED, AGENT);
        o.c = __hip_atomic_load((int32_t*)(sp + 16), __ATOMIC_RELAXED, AGENT);
        o.w = w;
        if (kbetter(o, best)) best = o;
    }
    best = block_reduce(best, sm);
    if (threadIdx.x < n) {
        const double* wp = (const double*)(slot_ptr(tm, par, best.w) + 32);
        sm.pay[threadIdx.x] = (T)__hip_atomic_load(wp + threadIdx.x, __ATOMIC_RELAXED, AGENT);
    }
    __syncthreads();
    return best;
}

// ----------------------------------------------------------------------------
// a workgroup's slice of the strip
// ----------------------------------------------------------------------------

template <typename T>
struct Rows {
    T* B;        // element (r, c) of the slice at B[c * ld + r]
    int64_t ld;
    int64_t r0;  // first global row of the slice
    int nrows;
};

// Gather rows [r0, r0 + nrows) of the strip: column step A[:, F], row step
// A[F, :]^T.  Physical column c of the slice receives logical column
// cmap[c] (cmap == nullptr: identity).  Returns this thread's max |entry|
// (+inf if an entry is not finite).
template <typename T, int KMAX>
__device__ double gather_rows(const DevSource& s, int transpose, const Smem<T, KMAX>& sm,
                              const int64_t* F, const int32_t* cmap, int k, const Rows<T>& rw)
{
    double lmax = 0.0;
    for (int r = threadIdx.x; r < rw.nrows; r += NT) {
        const int64_t gi = rw.r0 + r;
        T v[KMAX];
        if (s.kind == 0) {
#pragma unroll
            for (int c = 0; c < KMAX; ++c)
                if (c < k) {
                    const int64_t f = F[cmap ? cmap[c] : c];
                    v[c] = transpose ? dense_entry<T>(s, f, gi) : dense_entry<T>(s, gi, f);
                }
        } else {
            const double own = transpose ? load_elem(s.y, s.dtype, gi) : load_elem(s.x, s.dtype, gi);
#pragma unroll
            for (int c = 0; c < KMAX; ++c)
                if (c < k) {
                    const double pt = sm.pts[cmap ? cmap[c] : c];
                    v[c] = kernel_entry<T>(s.kind, transpose ? pt - own : own - pt);
                }
        }
#pragma unroll
        for (int c = 0; c < KMAX; ++c)
            if (c < k) {
                double a = fabs((double)v[c]);
                if (!(a <= 1.0e308)) a = INFINITY;  // NaN or Inf
                lmax = fmax(lmax, a);
                rw.B[c * rw.ld + r] = v[c];
            }
    }
    return lmax;
}

// ----------------------------------------------------------------------------
// k x k partial-pivot LU in LDS (row stride KMAX), rows pivoted as in LAPACK
// getrf (first maximum).  perm[t] = original row now at t.  Stops at an exact
// zero pivot and returns 0; else returns 1.  sm.thresh receives the smallest
// pivot modulus.
// ----------------------------------------------------------------------------

template <typename T, typename LT, int KMAX>
__device__ int lu_kxk(LT* LU, Smem<T, KMAX>& sm, int k)
{
    if (threadIdx.x < k) sm.perm[threadIdx.x] = threadIdx.x;
    if (threadIdx.x == 0) sm.thresh = INFINITY;
    __syncthreads();
    int ok = 1;
    for (int t = 0; t < k; ++t) {
        if (threadIdx.x < 64) {
            Key kk = key_none();
            const int s = t + threadIdx.x;
            if (s < k) { kk.v = fabs((double)LU[s * KMAX + t]); kk.r = s; kk.c = 0; }
            kk = wave_reduce(kk);
            if (threadIdx.x == 0) {
                sm.win = kk;
                sm.ok = kk.v != 0.0;
                sm.thresh = fmin(sm.thresh, kk.v);
            }
        }
        __syncthreads();
        if (!sm.ok) { ok = 0; break; }
        const int p = (int)sm.win.r;
        if (p != t) {
            for (int c = threadIdx.x; c < k; c += NT) {
                LT tmp = LU[t * KMAX + c];
                LU[t * KMAX + c] = LU[p * KMAX + c];
                LU[p * KMAX + c] = tmp;
            }
            if (threadIdx.x == 0) {
                int tp = sm.perm[t];
                sm.perm[t] = sm.perm[p];
                sm.perm[p] = tp;
            }
        }
        __syncthreads();
        const LT piv = LU[t * KMAX + t];
        for (int s = t + 1 + threadIdx.x; s < k; s += NT) LU[s * KMAX + t] = LU[s * KMAX + t] / piv;
        __syncthreads();
        const int w = k - t - 1;
        for (int e = threadIdx.x; e < w * w; e += NT) {
            const int s = t + 1 + e / w, c = t + 1 + e % w;
            LU[s * KMAX + c] -= LU[s * KMAX + t] * LU[t * KMAX + c];
        }
        __syncthreads();
    }
    __syncthreads();
    return ok;
}

// ----------------------------------------------------------------------------
// one maxvol step (Section 6.5): column step (transpose = 0) picks I from
// A[:, J]; row step (transpose = 1) picks J from A[I, :]^T.
// ----------------------------------------------------------------------------

template <typename T, int KMAX>
__device__ void maxvol_step(const TaskDesc& td, Smem<T, KMAX>& sm, Team& tm, int transpose,
                            int lds_b_bytes, T* Blds)
{
    const int k = sm.k;
    const int64_t M = transpose ? td.n : td.m;
    const int64_t* F = transpose ? sm.I : sm.J;
    int64_t* X = transpose ? sm.J : sm.I;
    const bool have_X = transpose ? true : (sm.have_I != 0);
    const bool warm = have_X && td.warm_start;
    const double u = sizeof(T) == 8 ? 0x1p-53 : 0x1p-24;

    const int64_t R = (M + tm.size - 1) / tm.size;
    Rows<T> rw;
    rw.r0 = (int64_t)tm.rank * R;
    {
        int64_t r1 = rw.r0 + R < M ? rw.r0 + R : M;
        rw.nrows = r1 > rw.r0 ? (int)(r1 - rw.r0) : 0;
    }
    if ((int64_t)R * k * (int64_t)sizeof(T) <= lds_b_bytes) {
        rw.B = Blds;
        rw.ld = R;
    } else {
        rw.B = (T*)td.strip + rw.r0;
        rw.ld = M;
    }
    const int64_t rend = rw.r0 + rw.nrows;

    // Warm start: partial-pivot LU of Chat^T (Chat = strip[X, :]) before the
    // gather, so that its row permutation becomes the gather's column order
    // and both triangular solves below run in place.
    T* LUt = (T*)sm.LU;
    int warm_lu = 0;
    double minpiv = 0.0;
    if (warm) {
        for (int e = threadIdx.x; e < k * k; e += NT) {
            const int c = e / k, s = e % k;  // (Chat^T)[c][s] = strip(X[s], c)
            LUt[c * KMAX + s] = transpose ? entry_t<T>(td.src, F[c], X[s]) : entry_t<T>(td.src, X[s], F[c]);
        }
        __syncthreads();
        warm_lu = lu_kxk<T, T, KMAX>(LUt, sm, k);
        minpiv = sm.thresh;
    }

    // 1. gather this workgroup's rows of the strip
    if (td.src.kind != 0) {
        if (threadIdx.x < k)
            sm.pts[threadIdx.x] = transpose ? load_elem(td.src.x, td.src.dtype, F[threadIdx.x])
                                            : load_elem(td.src.y, td.src.dtype, F[threadIdx.x]);
        __syncthreads();
    }
    double lmax = gather_rows<T, KMAX>(td.src, transpose, sm, F, warm_lu ? sm.perm : nullptr, k, rw);

    // 2. team-wide max |entry| (non-finite -> +inf)
    Key km = key_none();
    km.v = lmax;
    km.r = 0;
    km.c = 0;
    km = block_reduce(km, sm);
    km = team_argmax(tm, sm, km, 0);
    if (tm.failed) return;
    if (threadIdx.x == 0) sm.entries_read += M * k;
    if (isinf(km.v)) {
        if (threadIdx.x == 0) { sm.status = -6; sm.phase = PH_DONE; }
        __syncthreads();
        return;
    }
    const double thresh = 64.0 * u * km.v;

    // 3. basis B = C C[X,:]^{-1}
    int keff = k;
    const int started = warm_lu && minpiv > thresh;
    if (started) {
        // B Chat = C  <=>  Chat^T B^T = C^T, P Chat^T = L U: the slice already
        // holds P C^T row-wise; L w = (P c), U x = w, in place.
        for (int r = threadIdx.x; r < rw.nrows; r += NT) {
            T* b = rw.B + r;
            for (int s = 1; s < k; ++s) {
                T acc = b[s * rw.ld];
                for (int d = 0; d < s; ++d) acc -= LUt[s * KMAX + d] * b[d * rw.ld];
                b[s * rw.ld] = acc;
            }
            for (int s = k - 1; s >= 0; --s) {
                T acc = b[s * rw.ld];
                for (int d = s + 1; d < k; ++d) acc -= LUt[s * KMAX + d] * b[d * rw.ld];
                b[s * rw.ld] = acc / LUt[s * KMAX + s];
            }
        }
        __syncthreads();
    } else {
        if (warm_lu) {
            // gathered in pivot order for a start that was rejected: gather again
            (void)gather_rows<T, KMAX>(td.src, transpose, sm, F, nullptr, k, rw);
            __syncthreads();
        }
        // partial-pivot LU of the strip: k team-wide pivot searches
        Key kl = key_none();
        for (int r = threadIdx.x; r < rw.nrows; r += NT) {
            Key o;
            o.v = fabs((double)rw.B[r]);
            o.r = rw.r0 + r;
            o.c = 0;
            o.w = tm.rank;
            if (kbetter(o, kl)) kl = o;
        }
        for (int t = 0; t < k; ++t) {
            kl = block_reduce(kl, sm);
            if (threadIdx.x < k && kl.r >= rw.r0 && kl.r < rend)
                sm.pay[threadIdx.x] = rw.B[threadIdx.x * rw.ld + (kl.r - rw.r0)];
            __syncthreads();
            Key wv = team_argmax(tm, sm, kl, k);
            if (tm.failed) return;
            if (wv.v == 0.0) {
                if (threadIdx.x == 0) { sm.status = -2; sm.phase = PH_DONE; }
                __syncthreads();
                return;
            }
            if (wv.v < thresh) { keff = t; break; }
            if (threadIdx.x == 0) X[t] = wv.r;
            if (threadIdx.x < t) LUt[t * KMAX + threadIdx.x] = sm.pay[threadIdx.x];
            const T piv = sm.pay[t];
            kl = key_none();
            for (int r = threadIdx.x; r < rw.nrows; r += NT) {
                const T l = rw.B[t * rw.ld + r] / piv;
                rw.B[t * rw.ld + r] = l;
                for (int c = t + 1; c < k; ++c) rw.B[c * rw.ld + r] -= l * sm.pay[c];
                if (t + 1 < k) {
                    Key o;
                    o.v = fabs((double)rw.B[(t + 1) * rw.ld + r]);
                    o.r = rw.r0 + r;
                    o.c = 0;
                    o.w = tm.rank;
                    if (kbetter(o, kl)) kl = o;
                }
            }
            __syncthreads();
        }
        // B = L L1^{-1}: x L1 = l, descending, in place
        for (int r = threadIdx.x; r < rw.nrows; r += NT) {
            T* b = rw.B + r;
            for (int c = keff - 2; c >= 0; --c) {
                T x = b[c * rw.ld];
                for (int s2 = c + 1; s2 < keff; ++s2) x -= b[s2 * rw.ld] * LUt[s2 * KMAX + c];
                b[c * rw.ld] = x;
            }
        }
        __syncthreads();
    }
    // rows of the chosen set are unit rows of B
    for (int e = threadIdx.x; e < keff * keff; e += NT) {
        const int s = e / keff, c = e % keff;
        const int64_t gr = X[s];
        if (gr >= rw.r0 && gr < rend) rw.B[c * rw.ld + (gr - rw.r0)] = (T)(c == s ? 1 : 0);
    }
    __syncthreads();

    // 4. swaps: while max|B| > 1 + tau, bring the winning row into its column's slot
    const double lim = 1.0 + td.tau;
    const int max_swaps = td.max_swaps > 0 ? td.max_swaps : 4 * keff + 64;
    int swaps = 0;
    Key kl = key_none();
    for (int r = threadIdx.x; r < rw.nrows; r += NT)
        for (int c = 0; c < keff; ++c) {
            Key o;
            o.v = fabs((double)rw.B[c * rw.ld + r]);
            o.r = rw.r0 + r;
            o.c = c;
            o.w = tm.rank;
            if (kbetter(o, kl)) kl = o;
        }
    for (;;) {
        kl = block_reduce(kl, sm);
        if (threadIdx.x < keff && kl.r >= rw.r0 && kl.r < rend)
            sm.pay[threadIdx.x] = rw.B[threadIdx.x * rw.ld + (kl.r - rw.r0)];
        __syncthreads();
        Key wv = team_argmax(tm, sm, kl, keff);
        if (tm.failed) return;
        if (!(wv.v > lim)) break;
        if (swaps == max_swaps) {
            if (threadIdx.x == 0) sm.warn |= W_CAP;
            break;
        }
        const int js = wv.c;
        const int64_t is = wv.r;
        const T piv = sm.pay[js];
        if (threadIdx.x < keff) sm.g[threadIdx.x] = (sm.pay[threadIdx.x] - (T)(threadIdx.x == js ? 1 : 0)) / piv;
        __syncthreads();
        if (threadIdx.x == 0) X[js] = is;
        ++swaps;
        kl = key_none();
        for (int r = threadIdx.x; r < rw.nrows; r += NT) {
            const T f = rw.B[js * rw.ld + r];
            const bool unit = (rw.r0 + r == is);
            for (int c = 0; c < keff; ++c) {
                T v = unit ? (T)(c == js ? 1 : 0) : rw.B[c * rw.ld + r] - f * sm.g[c];
                rw.B[c * rw.ld + r] = v;
                Key o;
                o.v = fabs((double)v);
                o.r = rw.r0 + r;
                o.c = c;
                o.w = tm.rank;
                if (kbetter(o, kl)) kl = o;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sm.swaps_total += swaps;
        if (keff < k) {
            sm.warn |= W_NUMRANK;
            sm.k = keff;
        }
    }
    __syncthreads();
}

// ----------------------------------------------------------------------------
// optional CUR factors: C = A[:, J] (m x k column-major), R = A[I, :] (k x n)
// ----------------------------------------------------------------------------

template <typename T, int KMAX>
__device__ void write_factors(const TaskDesc& td, Smem<T, KMAX>& sm, const Team& tm)
{
    const int k = sm.k;
    if (td.C_out) {
        T* C = (T*)td.C_out;
        const int64_t R = (td.m + tm.size - 1) / tm.size;
        const int64_t a = (int64_t)tm.rank * R, b = a + R < td.m ? a + R : td.m;
        for (int64_t i = a + threadIdx.x; i < b; i += NT)
            for (int c = 0; c < k; ++c) C[c * td.m + i] = entry_t<T>(td.src, i, sm.J[c]);
    }
    if (td.R_out) {
        T* Rm = (T*)td.R_out;
        const int64_t R = (td.n + tm.size - 1) / tm.size;
        const int64_t a = (int64_t)tm.rank * R, b = a + R < td.n ? a + R : td.n;
        for (int c = 0; c < k; ++c)
            for (int64_t j = a + threadIdx.x; j < b; j += NT) Rm[c * td.n + j] = entry_t<T>(td.src, sm.I[c], j);
    }
}

// Fixed-order block sum (every thread passes its partial; all get the total).
template <typename T, int KMAX>
__device__ double block_sum(double v, Smem<T, KMAX>& sm)
{
    sm.red[threadIdx.x] = v;
    __syncthreads();
    for (int h = NT / 2; h >= 1; h >>= 1) {
        if (threadIdx.x < h) sm.red[threadIdx.x] += sm.red[threadIdx.x + h];
        __syncthreads();
    }
    double r = sm.red[0];
    __syncthreads();
    return r;
}

// ----------------------------------------------------------------------------
// nucleus U = A[I,J]^{-1} and the sampled residual (leader workgroup only)
// ----------------------------------------------------------------------------

template <typename T, int KMAX>
__device__ void final_leader(const TaskDesc& td, Smem<T, KMAX>& sm)
{
    const int k = sm.k;
    double* LU = sm.LU;
    for (int e = threadIdx.x; e < k * k; e += NT) {
        const int s = e / k, t = e % k;
        const double v = entry64(td.src, sm.I[s], sm.J[t]);
        LU[s * KMAX + t] = v;
        td.G[s * k + t] = v;
    }
    __syncthreads();
    if (!lu_kxk<T, double, KMAX>(LU, sm, k)) {
        if (threadIdx.x == 0) { sm.status = -2; sm.phase = PH_DONE; }
        __syncthreads();
        return;
    }
    // U: column t solves G u = e_t (L y = P e_t, U_f u = y), in place in td.U
    if (threadIdx.x < k) {
        const int t = threadIdx.x;
        double* u = td.U + t;
        for (int s = 0; s < k; ++s) {
            double a = sm.perm[s] == t ? 1.0 : 0.0;
            for (int c = 0; c < s; ++c) a -= LU[s * KMAX + c] * u[c * k];
            u[s * k] = a;
        }
        for (int s = k - 1; s >= 0; --s) {
            double a = u[s * k];
            for (int c = s + 1; c < k; ++c) a -= LU[s * KMAX + c] * u[c * k];
            u[s * k] = a / LU[s * KMAX + s];
        }
    }
    __threadfence_block();
    __syncthreads();
    // exact 1-norm condition number ||G||_1 ||U||_1
    {
        double cg = 0.0, cu = 0.0;
        if (threadIdx.x < k)
            for (int s = 0; s < k; ++s) {
                cg += fabs(td.G[s * k + threadIdx.x]);
                cu += fabs(td.U[s * k + threadIdx.x]);
            }
        Key a = key_none();
        a.v = cg;
        a.r = 0;
        a.c = 0;
        Key b = key_none();
        b.v = cu;
        b.r = 0;
        b.c = 0;
        a = block_reduce(a, sm);
        b = block_reduce(b, sm);
        if (threadIdx.x == 0) sm.cond1 = a.v * b.v;
    }
    // residual on Q x S: W = G^{-1} A[I,S] through the LU, E = A[Q,S] - A[Q,J] W
    const int q = td.q, s = td.s;
    double* AQJ = td.work;                 // q x k
    double* W = td.work + (int64_t)q * k;  // k x s
    double* E = W + (int64_t)k * s;        // q x s
    for (int e = threadIdx.x; e < q * k; e += NT) {
        const int a = e / k, t = e % k;
        AQJ[e] = entry64(td.src, td.Q[a], sm.J[t]);
    }
    for (int b = threadIdx.x; b < s; b += NT) {
        double* w = W + b;
        for (int a = 0; a < k; ++a) {
            double y = entry64(td.src, sm.I[sm.perm[a]], td.S[b]);
            for (int c = 0; c < a; ++c) y -= LU[a * KMAX + c] * w[c * s];
            w[a * s] = y;
        }
        for (int a = k - 1; a >= 0; --a) {
            double y = w[a * s];
            for (int c = a + 1; c < k; ++c) y -= LU[a * KMAX + c] * w[c * s];
            w[a * s] = y / LU[a * KMAX + a];
        }
    }
    __threadfence_block();
    __syncthreads();
    double se = 0.0, sa = 0.0, sum = 0.0;
    for (int e = threadIdx.x; e < q * s; e += NT) {
        const int a = e / s, b = e % s;
        double cur = 0.0;
        for (int t = 0; t < k; ++t) cur += AQJ[a * k + t] * W[t * s + b];
        const double av = entry64(td.src, td.Q[a], td.S[b]);
        const double ev = av - cur;
        E[e] = ev;
        se += ev * ev;
        sa += av * av;
        sum += ev;
    }
    se = block_sum(se, sm);
    sa = block_sum(sa, sm);
    sum = block_sum(sum, sm);
    const double cnt = (double)q * (double)s;
    const double mean = sum / cnt;
    double vs = 0.0;
    for (int e = threadIdx.x; e < q * s; e += NT) vs += (E[e] - mean) * (E[e] - mean);
    vs = block_sum(vs, sm);
    if (threadIdx.x == 0) {
        const double ne = sqrt(se), na = sqrt(sa);
        sm.mean = mean;
        sm.var = vs / cnt;
        sm.est_abs = sqrt((double)td.m * (double)td.n / cnt) * ne;
        sm.est_rel = na > 0.0 ? ne / na : (ne > 0.0 ? INFINITY : 0.0);
        sm.entries_read += (int64_t)k * k + (int64_t)q * k + (int64_t)k * s + (int64_t)q * s;
        // decision: done, or grow the rank (Algorithm 5.1: raise the rank on failure)
        if (!(td.tol > 0.0) || !(sm.est_rel > td.tol)) {
            sm.phase = PH_DONE;
        } else if ((sm.warn & W_NUMRANK) || k >= td.kmax) {
            sm.warn |= W_TOL;
            sm.phase = PH_DONE;
        } else {
            int room = td.kmax - k < td.kstep ? td.kmax - k : td.kstep;
            int added = 0;
            while (added < room && sm.cand_next < td.n_cand) {
                const int64_t cnd = td.cand[sm.cand_next++];
                int dup = 0;
                for (int c = 0; c < k + added; ++c)
                    if (sm.J[c] == cnd) { dup = 1; break; }
                if (!dup) sm.J[k + added++] = cnd;
            }
            if (added == 0) {
                sm.warn |= W_TOL;
                sm.phase = PH_DONE;
            } else {
                sm.k = k + added;
                sm.have_I = 0;
                sm.sweep_in_level = 0;
                sm.phase = PH_COL;
            }
        }
    }
    __syncthreads();
}

// ----------------------------------------------------------------------------
// state transfer between the team's workgroups and across launches
// ----------------------------------------------------------------------------

template <typename T, int KMAX>
__device__ void load_state(const TaskDesc& td, Smem<T, KMAX>& sm)
{
    if (threadIdx.x == 0) {
        const TaskState* st = td.st;
        sm.phase = __hip_atomic_load(&st->phase, __ATOMIC_RELAXED, AGENT);
        sm.k = __hip_atomic_load(&st->k, __ATOMIC_RELAXED, AGENT);
        sm.sweep_in_level = __hip_atomic_load(&st->sweep_in_level, __ATOMIC_RELAXED, AGENT);
        sm.status = __hip_atomic_load(&st->status, __ATOMIC_RELAXED, AGENT);
        sm.warn = __hip_atomic_load(&st->warn, __ATOMIC_RELAXED, AGENT);
        sm.have_I = __hip_atomic_load(&st->have_I, __ATOMIC_RELAXED, AGENT);
        sm.had_I_sweep = __hip_atomic_load(&st->had_I_sweep, __ATOMIC_RELAXED, AGENT);
        sm.k_sweep_start = __hip_atomic_load(&st->k_sweep_start, __ATOMIC_RELAXED, AGENT);
        sm.swaps_total = __hip_atomic_load(&st->swaps_total, __ATOMIC_RELAXED, AGENT);
        sm.sweeps_done = __hip_atomic_load(&st->sweeps_done, __ATOMIC_RELAXED, AGENT);
        sm.phases_run = __hip_atomic_load(&st->phases_run, __ATOMIC_RELAXED, AGENT);
        sm.cand_next = __hip_atomic_load(&st->cand_next, __ATOMIC_RELAXED, AGENT);
        sm.entries_read = __hip_atomic_load(&st->entries_read, __ATOMIC_RELAXED, AGENT);
        sm.est_rel = __hip_atomic_load(&st->est_rel, __ATOMIC_RELAXED, AGENT);
        sm.est_abs = __hip_atomic_load(&st->est_abs, __ATOMIC_RELAXED, AGENT);
        sm.mean = __hip_atomic_load(&st->mean, __ATOMIC_RELAXED, AGENT);
        sm.var = __hip_atomic_load(&st->var, __ATOMIC_RELAXED, AGENT);
        sm.cond1 = __hip_atomic_load(&st->cond1, __ATOMIC_RELAXED, AGENT);
    }
    __syncthreads();
    const int kc = td.kmax > td.k0 ? td.kmax : td.k0;
    if (threadIdx.x < kc) {
        const int c = threadIdx.x;
        sm.I[c] = __hip_atomic_load(td.I + c, __ATOMIC_RELAXED, AGENT);
        sm.J[c] = __hip_atomic_load(td.J + c, __ATOMIC_RELAXED, AGENT);
        sm.prevI[c] = __hip_atomic_load(td.prevI + c, __ATOMIC_RELAXED, AGENT);
        sm.prevJ[c] = __hip_atomic_load(td.prevJ + c, __ATOMIC_RELAXED, AGENT);
    }
    __syncthreads();
}

template <typename T, int KMAX>
__device__ void store_state(const TaskDesc& td, Smem<T, KMAX>& sm)
{
    const int kc = td.kmax > td.k0 ? td.kmax : td.k0;
    if (threadIdx.x < kc) {
        const int c = threadIdx.x;
        __hip_atomic_store(td.I + c, sm.I[c], __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(td.J + c, sm.J[c], __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(td.prevI + c, sm.prevI[c], __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(td.prevJ + c, sm.prevJ[c], __ATOMIC_RELAXED, AGENT);
    }
    if (threadIdx.x == 0) {
        TaskState* st = td.st;
        __hip_atomic_store(&st->phase, sm.phase, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->k, sm.k, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->sweep_in_level, sm.sweep_in_level, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->status, sm.status, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->warn, sm.warn, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->have_I, sm.have_I, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->had_I_sweep, sm.had_I_sweep, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->k_sweep_start, sm.k_sweep_start, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->swaps_total, sm.swaps_total, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->sweeps_done, sm.sweeps_done, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->phases_run, sm.phases_run, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->cand_next, sm.cand_next, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->entries_read, sm.entries_read, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->est_rel, sm.est_rel, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->est_abs, sm.est_abs, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->mean, sm.mean, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->var, sm.var, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->cond1, sm.cond1, __ATOMIC_RELAXED, AGENT);
    }
    __threadfence();
    __syncthreads();
}

// Run one problem for up to `budget` phases.
template <typename T, int KMAX>
__device__ void run_task(const TaskDesc& td, Smem<T, KMAX>& sm, Team& tm, const EngineArgs& ea, T* Blds)
{
    load_state(td, sm);
    int budget = ea.phase_budget;
    while (sm.phase != PH_DONE && budget > 0) {
        --budget;
        const int ph = sm.phase;
        if (ph == PH_COL) {
            if (threadIdx.x < sm.k) {
                sm.prevI[threadIdx.x] = sm.I[threadIdx.x];
                sm.prevJ[threadIdx.x] = sm.J[threadIdx.x];
            }
            if (threadIdx.x == 0) {
                sm.had_I_sweep = sm.have_I;
                sm.k_sweep_start = sm.k;
            }
            __syncthreads();
            maxvol_step<T, KMAX>(td, sm, tm, 0, ea.lds_b_bytes, Blds);
            if (tm.failed) return;
            if (threadIdx.x == 0 && sm.phase != PH_DONE) {
                sm.have_I = 1;
                sm.phase = PH_ROW;
            }
            __syncthreads();
        } else if (ph == PH_ROW) {
            maxvol_step<T, KMAX>(td, sm, tm, 1, ea.lds_b_bytes, Blds);
            if (tm.failed) return;
            if (threadIdx.x == 0 && sm.phase != PH_DONE) {
                sm.sweeps_done += 1;
                sm.sweep_in_level += 1;
                int next = sm.sweep_in_level >= td.sweeps ? PH_FINAL : PH_COL;
                if (td.tol > 0.0 && sm.had_I_sweep && sm.k == sm.k_sweep_start) {
                    int same = 1;
                    for (int c = 0; c < sm.k; ++c)
                        if (sm.I[c] != sm.prevI[c] || sm.J[c] != sm.prevJ[c]) same = 0;
                    if (same) next = PH_FINAL;
                }
                sm.phase = next;
            }
            __syncthreads();
        } else {  // PH_FINAL
            write_factors<T, KMAX>(td, sm, tm);
            if (tm.rank == 0) final_leader<T, KMAX>(td, sm);
            if (tm.size > 1) {
                // the leader's decision reaches the team through global memory
                if (tm.rank == 0) store_state(td, sm);
                team_barrier(tm, sm);
                if (tm.failed) return;
                if (tm.rank != 0) load_state(td, sm);
            }
        }
        if (threadIdx.x == 0) sm.phases_run += 1;
        __syncthreads();
        if (tm.rank == 0) store_state(td, sm);
    }
}

template <typename T, int KMAX>
__global__ __launch_bounds__(NT) void engine_kernel(EngineArgs ea)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Smem<T, KMAX>& sm = *reinterpret_cast<Smem<T, KMAX>*>(smem_raw);
    T* Blds = reinterpret_cast<T*>(smem_raw + ((sizeof(Smem<T, KMAX>) + 255) & ~(size_t)255));
    const int team = ea.wg_team[blockIdx.x];
    const TeamInfo ti = ea.teams[team];
    Team tm;
    tm.ctl = ea.team_ctl + (int64_t)team * ea.team_ctl_stride;
    tm.size = ti.size;
    tm.rank = blockIdx.x - ti.first_wg;
    tm.epoch = 0;
    tm.failed = false;
    tm.err = ea.error_flag;
    tm.timeout = ea.timeout_ticks;
    for (;;) {
        const int par = tm.epoch & 1;
        int32_t* fetch = (int32_t*)(tm.ctl + 64) + par;
        if (threadIdx.x == 0 && tm.rank == 0) {
            const int idx = (int)atomicAdd(ea.queue_head + ti.queue, 1u);
            sm.fetch = idx;
            if (tm.size > 1) __hip_atomic_store(fetch, idx, __ATOMIC_RELAXED, AGENT);
        }
        if (tm.size > 1) {
            team_barrier(tm, sm);
            if (tm.failed) return;
            if (threadIdx.x == 0 && tm.rank != 0) sm.fetch = __hip_atomic_load(fetch, __ATOMIC_RELAXED, AGENT);
        }
        __syncthreads();
        const int idx = sm.fetch;
        __syncthreads();
        if (idx >= ea.queue_len[ti.queue]) break;
        const int task = ea.queue_items[ea.queue_off[ti.queue] + idx];
        run_task<T, KMAX>(ea.tasks[task], sm, tm, ea, Blds);
        if (tm.failed) return;
    }
}

// Zero-fill used instead of hipMemsetAsync (safe to record in a graph).
__global__ void zero_kernel(uint32_t* p, int64_t n_words)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_words;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ----------------------------------------------------------------------------
// host-side launch helpers (C++ linkage inside the library)
// ----------------------------------------------------------------------------

template <typename T, int KMAX>
static const void* engine_fn()
{
    return reinterpret_cast<const void*>(&engine_kernel<T, KMAX>);
}

size_t engine_smem_fixed(int prec64, int kmax)
{
    auto sz = [](size_t s) { return (s + 255) & ~(size_t)255; };
    if (prec64) {
        if (kmax <= 8) return sz(sizeof(Smem<double, 8>));
        if (kmax <= 16) return sz(sizeof(Smem<double, 16>));
        if (kmax <= 32) return sz(sizeof(Smem<double, 32>));
        return sz(sizeof(Smem<double, 64>));
    }
    if (kmax <= 8) return sz(sizeof(Smem<float, 8>));
    if (kmax <= 16) return sz(sizeof(Smem<float, 16>));
    if (kmax <= 32) return sz(sizeof(Smem<float, 32>));
    return sz(sizeof(Smem<float, 64>));
}

const void* engine_kernel_ptr(int prec64, int kmax)
{
    if (prec64) {
        if (kmax <= 8) return engine_fn<double, 8>();
        if (kmax <= 16) return engine_fn<double, 16>();
        if (kmax <= 32) return engine_fn<double, 32>();
        return engine_fn<double, 64>();
    }
    if (kmax <= 8) return engine_fn<float, 8>();
    if (kmax <= 16) return engine_fn<float, 16>();
    if (kmax <= 32) return engine_fn<float, 32>();
    return engine_fn<float, 64>();
}

hipError_t launch_engine(int prec64, int kmax, int grid, size_t smem, bool cooperative,
                         const EngineArgs& ea, hipStream_t stream)
{
    const void* fn = engine_kernel_ptr(prec64, kmax);
    EngineArgs a = ea;
    void* args[] = {&a};
    if (cooperative)
        return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(NT), args, (unsigned)smem, stream);
    return hipLaunchKernel(fn, dim3(grid), dim3(NT), args, smem, stream);
}

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t stream)
{
    const int64_t words = (bytes + 3) / 4;
    int blocks = (int)((words + 255) / 256);
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, stream, (uint32_t*)p, words);
    return hipGetLastError();
}

}  // namespace lra
