// lra_engine.hip -- gfx950 kernels of the C-A / CUR library.
//
// One persistent kernel runs whole C-A / CUR problems.  A problem is owned by
// a *team* of workgroups; every pivot decision (a partial-pivot LU step or a
// maxvol swap) is one team-wide argmax: each workgroup reduces its rows
// (DPP wavefront max, then LDS), publishes its best key and candidate row in
// a slot in global memory, and after one team barrier every workgroup reduces
// the slots and reads the winning row.  A team of one workgroup needs no
// barrier at all.  A workgroup keeps its rows of the strip in LDS when they
// fit, else in a global strip buffer.  The basis product C * Chat^{-1} runs
// on the matrix cores (16x16x4 MFMA, binary64 or binary32).
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

#include <mutex>
#include <type_traits>

#include "lra_internal.h"

namespace lra {

constexpr int NWAVE = NT / 64;
#define AGENT __HIP_MEMORY_SCOPE_AGENT
#define DI __device__ __forceinline__

// ----------------------------------------------------------------------------
// entries
// ----------------------------------------------------------------------------

DI double load_elem(const void* p, int dtype, int64_t off)
{
    return dtype == 0 ? (double)((const float*)p)[off] : ((const double*)p)[off];
}

// Entry from a coordinate difference d (binary64): 1/d or 1/|d| (0 at d = 0).
template <typename T>
DI T kernel_entry(int kind, double d);

// Branch-free: |1/d| = 1/|d| exactly (the quotient's sign is the divisor's).
template <>
DI double kernel_entry<double>(int kind, double d)
{
    const double r = 1.0 / d;
    return kind == 1 ? r : (d == 0.0 ? 0.0 : fabs(r));
}

template <>
DI float kernel_entry<float>(int kind, double d)
{
    const float r = 1.0f / (float)d;
    return kind == 1 ? r : (d == 0.0 ? 0.0f : fabsf(r));
}

// Device allocations (sources, descriptors' arrays, control blocks, trace)
// are accessed through global-address-space pointers: generic (flat)
// accesses also count against the LDS wait counter, so that every wait for
// an LDS value would wait for them too.  Never for LDS or stack objects.
#define GL __attribute__((address_space(1)))
template <typename T>
DI GL T* gl(T* p)
{
    return (GL T*)p;
}
template <typename E>
DI const GL E* gptr(const void* p)
{
    return (const GL E*)p;
}

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): value number ctr of stream
// seed; the pre-processing signs are the top bits of its values.
DI uint64_t splitmix64(uint64_t seed, uint64_t ctr)
{
    uint64_t z = seed + (ctr + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Entry (i, j) of F A H (kind 3): F = D_F H_{pm,d} / 2^{d/2} and
// H = H_{pn,d} D_H / 2^{d/2} with the d-abridged Hadamard matrix
// H_{n,d} = H_{2^d} (Sylvester, entry (a,b) = (-1)^popcount(a & b)) times
// I_{n/2^d} in the Kronecker sense, and sign diagonals D_F, D_H from the
// SplitMix64 streams seed and seed + 1.  The sum runs over the 2^d x 2^d
// entries A[i mod s + t s, j mod s' + u s'] (s = pm / 2^d, s' = pn / 2^d),
// t outer, u inner, in binary64; the signs and 2^-d are exact factors.
// Out of line, with the source's fields by value: it is the slow path of the
// batched gathers, whose other paths keep their operands in registers.  Two
// entries per call, so that their loads are in flight together.
struct Pair {
    double a, b;
};

template <typename E>
__device__ __attribute__((noinline)) Pair preprocessed_pair(const void* ap, int64_t lda, int col_major, int d,
                                                            uint64_t seed, int64_t pm, int64_t pn, int64_t i0,
                                                            int64_t j0, int64_t i1, int64_t j1)
{
    const auto* a = gptr<E>(ap);
    const int64_t bm = pm >> d, bn = pn >> d;
    const int nb = 1 << d, nn = nb * nb;
    int64_t ib[2], ir[2], jb[2], jr[2];
    ib[0] = i0 / bm;
    ir[0] = i0 - ib[0] * bm;
    jb[0] = j0 / bn;
    jr[0] = j0 - jb[0] * bn;
    ib[1] = i1 / bm;
    ir[1] = i1 - ib[1] * bm;
    jb[1] = j1 / bn;
    jr[1] = j1 - jb[1] * bn;
    // the 4^d terms of each entry in the order e = t 2^d + u, loaded 16 at a
    // time (indices past the end repeat the chunk's first) and added in that
    // order
    double acc[2] = {0.0, 0.0};
    for (int e0 = 0; e0 < nn; e0 += 16) {
        double v[2][16];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int e = e0 + q < nn ? e0 + q : e0;
                const int64_t ii = ir[p] + (int64_t)(e >> d) * bm, jj = jr[p] + (int64_t)(e & (nb - 1)) * bn;
                v[p][q] = (double)a[col_major ? jj * lda + ii : ii * lda + jj];
            }
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int e = e0 + q;
                if (e < nn) {
                    const int neg = (__popcll((unsigned long long)(ib[p] & (e >> d))) +
                                     __popcll((unsigned long long)((e & (nb - 1)) & jb[p]))) & 1;
                    acc[p] += neg ? -v[p][q] : v[p][q];
                }
            }
    }
    Pair out;
    out.a = acc[0] * ((splitmix64(seed, (uint64_t)i0) >> 63) ? -1.0 : 1.0) *
            ((splitmix64(seed + 1, (uint64_t)j0) >> 63) ? -1.0 : 1.0) * ldexp(1.0, -d);
    out.b = acc[1] * ((splitmix64(seed, (uint64_t)i1) >> 63) ? -1.0 : 1.0) *
            ((splitmix64(seed + 1, (uint64_t)j1) >> 63) ? -1.0 : 1.0) * ldexp(1.0, -d);
    return out;
}

// Entries (ri[n], cj[n]) of a batch, element type E of the source: every
// load of the batch is unconditional, so all are in flight together.
template <typename E, typename T, int N>
DI void entries_e(const DevSource& s, const int64_t* ri, const int64_t* cj, T* out)
{
    if (s.kind == 0) {
        const auto* a = gptr<E>(s.a);
        E v[N];
#pragma unroll
        for (int n = 0; n < N; ++n) v[n] = a[s.col_major ? cj[n] * s.lda + ri[n] : ri[n] * s.lda + cj[n]];
#pragma unroll
        for (int n = 0; n < N; ++n) out[n] = (T)v[n];
    } else if (s.kind == 3) {
#pragma unroll
        for (int n = 0; n < N; n += 2) {
            const int n1 = n + 1 < N ? n + 1 : n;
            const Pair pr = preprocessed_pair<E>(s.a, s.lda, s.col_major, s.depth, s.seed, s.pm, s.pn, ri[n], cj[n],
                                                 ri[n1], cj[n1]);
            out[n] = (T)pr.a;
            if (n + 1 < N) out[n + 1] = (T)pr.b;
        }
    } else {
        const auto* x = gptr<E>(s.x);
        const auto* y = gptr<E>(s.y);
        E xv[N], yv[N];
#pragma unroll
        for (int n = 0; n < N; ++n) {
            xv[n] = x[ri[n]];
            yv[n] = y[cj[n]];
        }
#pragma unroll
        for (int n = 0; n < N; ++n) out[n] = kernel_entry<T>(s.kind, (double)xv[n] - (double)yv[n]);
    }
}

// Entries e in [0, total) taken by threads tid, tid + nth, ... in batches of
// PB per thread: idx(e, i, j) names entry e, st(e, value) stores it.  The
// source's kind and element type are uniform, so one branch on them encloses
// a whole batch; indices past the end repeat the batch's first (valid) one,
// so that only the stores are guarded.
template <typename T, int PB, typename IDX, typename ST>
DI void load_entries(const DevSource& s, int total, int tid, int nth, IDX idx, ST st)
{
    for (int e0 = tid; e0 < total; e0 += nth * PB) {
        int64_t ri[PB], cj[PB];
        T v[PB];
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            const int e = e0 + b * nth;
            idx(e < total ? e : e0, ri[b], cj[b]);
        }
        if (s.dtype == 0)
            entries_e<float, T, PB>(s, ri, cj, v);
        else
            entries_e<double, T, PB>(s, ri, cj, v);
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            const int e = e0 + b * nth;
            if (e < total) st(e, v[b]);
        }
    }
}

// ----------------------------------------------------------------------------
// argmax keys: (hi, lo) compared lexicographically; hi = bit pattern of a
// non-negative binary64 |value| (ordered like the value), lo = ~(row << 8 |
// col), so ties go to the smaller row, then the smaller column.
// ----------------------------------------------------------------------------

struct K2 {
    uint64_t hi, lo;
};

DI K2 k2_none() { return K2{0ull, 0ull}; }

DI bool k2_better(const K2& a, const K2& b) { return a.hi > b.hi || (a.hi == b.hi && a.lo > b.lo); }

DI K2 k2_make(double absv, int64_t row, int col)
{
    return K2{(uint64_t)__double_as_longlong(absv), ~(((uint64_t)row << 8) | (uint64_t)col)};
}

DI int64_t k2_row(const K2& k) { return (int64_t)((~k.lo) >> 8); }
DI int k2_col(const K2& k) { return (int)((~k.lo) & 0xFFull); }
DI double k2_val(const K2& k) { return __longlong_as_double((long long)k.hi); }

template <int CTRL, int ROWMASK>
DI uint64_t dpp64(uint64_t v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROWMASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, ROWMASK, 0xF, false);
    return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}

DI uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }

DI uint64_t readlane64(uint64_t v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Maximum over the 64 lanes of a full wavefront (row shifts 1, 2, 4, 8 within
// each row of 16 lanes, then the row-15 and row-31 broadcasts; lane 63 ends
// with the maximum, which is then read as a uniform value).
DI uint64_t wave_max_u64(uint64_t v)
{
    v = umax64(v, dpp64<0x111, 0xF>(v));
    v = umax64(v, dpp64<0x112, 0xF>(v));
    v = umax64(v, dpp64<0x114, 0xF>(v));
    v = umax64(v, dpp64<0x118, 0xF>(v));
    v = umax64(v, dpp64<0x142, 0xA>(v));
    v = umax64(v, dpp64<0x143, 0xC>(v));
    return readlane64(v, 63);
}

DI K2 wave_argmax(const K2& k)
{
    const uint64_t mh = wave_max_u64(k.hi);
    const uint64_t ball = __ballot(k.hi == mh);
    uint64_t lo;
    if (__popcll(ball) == 1)
        lo = readlane64(k.lo, __ffsll((unsigned long long)ball) - 1);
    else
        lo = wave_max_u64(k.hi == mh ? k.lo : 0ull);
    return K2{mh, lo};
}

// ----------------------------------------------------------------------------
// shared memory of one workgroup
// ----------------------------------------------------------------------------

template <typename T, int KMAX>
struct Smem {
    int64_t I[KMAX], J[KMAX], prevI[KMAX], prevJ[KMAX];
    double AUG[KMAX * 2 * KMAX];  // [M | right-hand sides], row stride 2 KMAX (T view for the strip)
    double lucol[NWAVE][KMAX];    // register LU, per wavefront: the pivot column
    double lumul[NWAVE][KMAX];    // register LU, per wavefront: the step's multipliers
    double red[4 * NWAVE];    // fixed-order reductions: wavefront partials
    double pts[KMAX];         // coordinates of the fixed index set (generated sources)
    T g[KMAX];                // swap update vector
    T pay[KMAX];              // candidate / winning row
    int32_t perm[KMAX];
    K2 kred[2][NWAVE];
    // problem state (mirrors TaskState)
    int32_t k, phase, sweep_in_level, status, warn, have_I, had_I_sweep, k_sweep_start;
    int32_t swaps_total, sweeps_done, phases_run;
    int64_t cand_next, entries_read;
    double est_rel, est_abs, mean, var, cond1;
    int32_t flag, fetch, ok, pivp;
    int32_t w_valid;          // AUG's right half holds C[X,:]^{-1} of the last step
    int32_t jsweeps;          // Jacobi sweeps of the last truncated nucleus (trace)
    double minpiv;
};

struct Team {
    uint8_t* ctl;
    int size;
    int rank;
    uint32_t epoch;   // team barriers passed
    uint32_t xepoch;  // argmax exchanges done
    int32_t failed;   // 0 or 1 (a full word: the struct has no padding to copy)
    int tog;          // LDS double-buffer selector of block_argmax
    uint32_t* err;
    int64_t timeout;
    uint64_t* trace;
    int32_t trace_cap;
    int32_t trace_n;
};

// Workgroup argmax: wavefront maxima, then one LDS exchange.  The two LDS
// banks alternate between calls, so one barrier per call suffices.
template <typename T, int KMAX>
DI K2 block_argmax(const K2& k, Smem<T, KMAX>& sm, Team& tm)
{
    const K2 w = wave_argmax(k);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sm.kred[tm.tog][wv] = w;
    __syncthreads();
    K2 b = sm.kred[tm.tog][0];
#pragma unroll
    for (int i = 1; i < NWAVE; ++i)
        if (k2_better(sm.kred[tm.tog][i], b)) b = sm.kred[tm.tog][i];
    tm.tog ^= 1;
    return b;
}

// Optional event trace: thread 0 of the first workgroup of team 0 records
// (event, wall clock) pairs with plain stores; the count goes to trace[0].
DI void trace_ev(Team& tm, int ev, int64_t arg)
{
    if (tm.trace == nullptr || tm.rank != 0 || threadIdx.x != 0) return;
    const int idx = tm.trace_n++;
    if (idx >= tm.trace_cap) return;
    GL uint64_t* tr = gl(tm.trace);
    tr[1 + 2 * idx] = ((uint64_t)ev << 56) | ((uint64_t)arg & 0x00FFFFFFFFFFFFFFull);
    tr[2 + 2 * idx] = wall_clock64();
    tr[0] = (uint64_t)(idx + 1);
}

// ----------------------------------------------------------------------------
// team synchronisation.  Only wavefront 0 of a workgroup writes data that
// other workgroups read (slots, state); thread 0's release on the arrival
// counter publishes them, its acquire plus the workgroup barrier makes the
// other workgroups' data visible.
// ----------------------------------------------------------------------------

DI GL uint8_t* slot_ptr(const Team& tm, int parity, int wg)
{
    return gl(tm.ctl) + CTL_HDR + (int64_t)(parity * tm.size + wg) * SLOT_STRIDE;
}

DI int32_t* lds_flag();

DI void team_barrier(Team& tm)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        GL uint32_t* ctr = (GL uint32_t*)gl(tm.ctl);
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, AGENT);
        const uint32_t target = (tm.epoch + 1) * (uint32_t)tm.size;
        const int64_t t0 = wall_clock64();
        int bad = 0;
        // relaxed polling, one acquire fence once the count is reached (an
        // acquire load per iteration would invalidate the caches each time)
        for (uint32_t spins = 1; __hip_atomic_load(ctr, __ATOMIC_RELAXED, AGENT) < target; ++spins) {
            __builtin_amdgcn_s_sleep(1);
            if ((spins & 63) == 0 && wall_clock64() - t0 > tm.timeout) {
                __hip_atomic_fetch_or(gl(tm.err), 1u, __ATOMIC_RELAXED, AGENT);
                bad = 1;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *lds_flag() = bad;
    }
    __syncthreads();
    tm.epoch++;
    if (*lds_flag()) tm.failed = true;
}

// Team-wide argmax: publish this workgroup's best key and its candidate row
// (sm.pay[0..n)) in its own slot; thread i of every workgroup waits for slot
// i, so no counter is contended.  Then every workgroup reduces all slots and
// loads the winning row (owner = row / rows_per_wg) into sm.pay.  Slots
// alternate between two banks: a workgroup can only publish exchange x + 1
// after every slot of exchange x arrived, i.e. after every workgroup finished
// reading exchange x - 1.  With one workgroup the local result is final.
//
// The key words carry the exchange's version in their top bit, which a key
// does not use (hi holds the bits of a modulus, sign 0; lo the complement of
// row << 8 | col, top bit 1, or 0 for "no candidate"): version 1 for
// exchanges 0 and 1, then alternating per use of a bank, so the zeroed
// control block and the bank's previous exchange both read as not arrived.
// The writer orders its row before the key words with one release fence; a
// reader that sees both words at the current version has the key in hand
// (no second round trip for it), and its acquire fence makes the row visible.
// Work that needs no exchange result can run while the slots travel: an
// optional hook (every thread, after this workgroup has published) and an
// optional LDS row to publish instead of sm.pay.
struct NoHook {
    static constexpr bool active = false;
    DI void operator()() const {}
};

template <typename F>
struct Hook {
    static constexpr bool active = true;
    F f;
    DI void operator()() const { f(); }
};

template <typename F>
DI Hook<F> make_hook(F f) { return Hook<F>{f}; }

template <typename T, int KMAX, typename H = NoHook>
DI K2 team_argmax(Team& tm, Smem<T, KMAX>& sm, const K2& mine, int n, int64_t rows_per_wg, const H& hook = H(),
                  const double* cand = nullptr)
{
    if (tm.size == 1) {
        if constexpr (H::active) {
            hook();
            __syncthreads();
        }
        return mine;
    }
    const int par = tm.xepoch & 1;
    constexpr uint64_t TOP = 1ull << 63;
    const uint64_t ver = ((uint64_t)(((tm.xepoch >> 1) & 1u) ^ 1u)) << 63;
    tm.xepoch++;
    GL uint8_t* my = slot_ptr(tm, par, tm.rank);
    GL double* mypay = (GL double*)(my + 32);
    // written by wavefront 0 only: the release fence below orders all of them
    if (threadIdx.x < n)
        __hip_atomic_store(mypay + threadIdx.x, cand ? cand[threadIdx.x] : (double)sm.pay[threadIdx.x], __ATOMIC_RELAXED,
                           AGENT);
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store((GL uint64_t*)my, mine.hi | ver, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store((GL uint64_t*)(my + 8), (mine.lo & ~TOP) | ver, __ATOMIC_RELAXED, AGENT);
    }
    if constexpr (H::active) hook();
    // a slot that never arrives yields the reserved key K2_FAIL, which wins
    // the reduction (keys of moduli, +inf included, have smaller hi words)
    K2 o = k2_none();
    if (threadIdx.x < tm.size) {
        const GL uint64_t* sp = (const GL uint64_t*)slot_ptr(tm, par, threadIdx.x);
        const int64_t t0 = wall_clock64();
        bool bad = false;
        uint64_t h, l;
        for (uint32_t spins = 1;; ++spins) {
            h = __hip_atomic_load(sp, __ATOMIC_RELAXED, AGENT);
            l = __hip_atomic_load(sp + 1, __ATOMIC_RELAXED, AGENT);
            if ((h & TOP) == ver && (l & TOP) == ver) break;
            __builtin_amdgcn_s_sleep(1);
            if ((spins & 63) == 0 && wall_clock64() - t0 > tm.timeout) {
                __hip_atomic_fetch_or(gl(tm.err), 1u, __ATOMIC_RELAXED, AGENT);
                bad = true;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (bad) {
            o = K2{~0ull, ~0ull};
        } else {
            o.hi = h & ~TOP;
            o.lo = (l & ~TOP) ? (l | TOP) : 0ull;
        }
    }
    const K2 best = block_argmax(o, sm, tm);
    if (best.hi == ~0ull) {
        tm.failed = true;
        return k2_none();
    }
    if (n > 0) {
        // no candidate anywhere (key 0): the callers stop without reading a row
        if (best.lo != 0ull && threadIdx.x < n) {
            const int64_t wo = k2_row(best) / rows_per_wg;
            const int w = wo < tm.size ? (int)wo : tm.size - 1;
            const GL double* wp = (const GL double*)(slot_ptr(tm, par, w) + 32);
            sm.pay[threadIdx.x] = (T)__hip_atomic_load(wp + threadIdx.x, __ATOMIC_RELAXED, AGENT);
        }
        __syncthreads();
    }
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
// A[F, :]^T, by threads tid of nth.  Returns this thread's max |entry| (+inf
// if an entry is not finite).  Dense sources: up to 32 columns of a row
// loaded together, columns past k repeating column c0 so that every load is
// unconditional.  Generated sources: 8 columns at a time (ranks grow in
// steps of 8), from the coordinates of the index set held in LDS.
template <typename T, int CH>
DI double store_chunk(const T* v, int c0, int k, const Rows<T>& rw, int r, double lmax)
{
#pragma unroll
    for (int cc = 0; cc < CH; ++cc) {
        const int c = c0 + cc;
        if (c < k) {
            double a = fabs((double)v[cc]);
            if (!(a <= 1.0e308)) a = INFINITY;  // NaN or Inf
            lmax = fmax(lmax, a);
            rw.B[c * rw.ld + r] = v[cc];
        }
    }
    return lmax;
}

// Dense sources, CH columns of a row loaded together (the chunk width is
// chosen from k, so that a small rank issues no loads for columns it lacks).
template <typename T, int CH>
DI double gather_dense_rows(const DevSource& s, int transpose, const int64_t* F, int k, const Rows<T>& rw, int tid,
                            int nth)
{
    double lmax = 0.0;
    for (int r = tid; r < rw.nrows; r += nth) {
        const int64_t gi = rw.r0 + r;
        for (int c0 = 0; c0 < k; c0 += CH) {
            int64_t ri[CH], cj[CH];
            T v[CH];
#pragma unroll
            for (int cc = 0; cc < CH; ++cc) {
                const int c = c0 + cc < k ? c0 + cc : c0;
                ri[cc] = transpose ? F[c] : gi;
                cj[cc] = transpose ? gi : F[c];
            }
            if (s.dtype == 0)
                entries_e<float, T, CH>(s, ri, cj, v);
            else
                entries_e<double, T, CH>(s, ri, cj, v);
            lmax = store_chunk<T, CH>(v, c0, k, rw, r, lmax);
        }
    }
    return lmax;
}

template <typename T, int KMAX>
DI double gather_rows(const DevSource& src, int transpose, const Smem<T, KMAX>& sm, const int64_t* F, int k,
                      const Rows<T>& rw, int tid, int nth)
{
    const DevSource s = src;  // read once: stores to a global strip could alias it
    double lmax = 0.0;
    if (s.kind == 0 || s.kind == 3) {
        constexpr int C16 = KMAX < 16 ? KMAX : 16, C32 = KMAX < 32 ? KMAX : 32;
        if (k <= 8)
            lmax = gather_dense_rows<T, 8>(s, transpose, F, k, rw, tid, nth);
        else if (k <= C16)
            lmax = gather_dense_rows<T, C16>(s, transpose, F, k, rw, tid, nth);
        else
            lmax = gather_dense_rows<T, C32>(s, transpose, F, k, rw, tid, nth);
    } else {
        constexpr int CH = 8;
        for (int r = tid; r < rw.nrows; r += nth) {
            const int64_t gi = rw.r0 + r;
            const double own = transpose ? load_elem(s.y, s.dtype, gi) : load_elem(s.x, s.dtype, gi);
            for (int c0 = 0; c0 < k; c0 += CH) {
                T v[CH];
#pragma unroll
                for (int cc = 0; cc < CH; ++cc) {
                    const int c = c0 + cc < k ? c0 + cc : c0;
                    v[cc] = kernel_entry<T>(s.kind, transpose ? sm.pts[c] - own : own - sm.pts[c]);
                }
                lmax = store_chunk<T, CH>(v, c0, k, rw, r, lmax);
            }
        }
    }
    return lmax;
}

// ----------------------------------------------------------------------------
// small dense solves by one wavefront
// ----------------------------------------------------------------------------

// Orders the LDS accesses of wavefront 0 across lanes: the lanes of a
// wavefront execute in lockstep and LDS serves one wavefront's requests in
// order, so it suffices that the compiler keeps program order here.
DI void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

DI double readlane_t(double v, int lane)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    return __longlong_as_double((long long)readlane64(b, lane));
}

DI float readlane_t(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Solve M X = R for the k x k matrix M held in columns [0, k) of A (row
// stride LD) and the nr right-hand sides in columns [rhs0, rhs0 + nr):
// partial-pivot LU with the elimination carried along on the right-hand
// sides (rows interchanged in place, pivots chosen as in LAPACK getrf:
// larger modulus, then smaller position), then back substitution.  On
// return row t of the right-hand-side block holds unknown t.
//
// Wavefront 0 does the whole solve with no workgroup barrier inside: for
// the pivot search and the multipliers lane s stands for row s (k <= 64);
// for the updates lane c owns the columns c, c + 64, ... still in use, and
// the multiplier of row s reaches every lane by a lane read.  Lanes without
// a column of their own address column t instead, which is dead by then
// (its rows past the pivot are never read again), so the loads and stores
// need no per-lane branches and stay pipelined.  Wavefront 0 alone; writes
// sm.ok (0 on an exact zero pivot) and sm.minpiv (the smallest pivot
// modulus).
template <typename T, int KMAX, typename LT, int LD, int NB>
DI void lu_aug_wave0(LT* A, int k, int rhs0, int nr, Smem<T, KMAX>& sm)
{
    {
        const int lane = threadIdx.x;
        double minpiv = INFINITY;
        int ok = 1;
        LT dreg = (LT)0;  // lane t keeps pivot t
        for (int t = 0; t < k; ++t) {
            K2 key = (lane >= t && lane < k) ? k2_make(fabs((double)A[lane * LD + t]), lane, 0) : k2_none();
            key = wave_argmax(key);
            const double pav = k2_val(key);
            if (pav == 0.0) {
                ok = 0;
                break;
            }
            minpiv = fmin(minpiv, pav);
            const int p = (int)k2_row(key);
            const LT piv = A[p * LD + t];
            if (lane == t) dreg = piv;
            // multiplier of the row that lands in position s after the interchange
            const int srow = lane < k ? (lane == p ? t : lane) : t;
            const LT lm = A[srow * LD + t] / piv;
            const int wl = k - t - 1;
            const int w = wl + nr;
            int col[NB];
            bool act[NB];
#pragma unroll
            for (int jb = 0; jb < NB; ++jb) {
                const int cc = lane + 64 * jb;
                act[jb] = cc < w;
                col[jb] = act[jb] ? (cc < wl ? t + 1 + cc : rhs0 + cc - wl) : t;
            }
            wave_lds_sync();
            // interchange rows t and p in the columns still in use; keep the new row t
            LT prow[NB];
#pragma unroll
            for (int jb = 0; jb < NB; ++jb) {
                const LT a = A[t * LD + col[jb]];
                const LT b = A[p * LD + col[jb]];
                prow[jb] = act[jb] ? b : (LT)0;
                A[t * LD + col[jb]] = act[jb] ? b : a;
                A[p * LD + col[jb]] = act[jb] ? a : b;
            }
            wave_lds_sync();
            // rows below the pivot, four at a time (all loads before the stores)
            int s2 = t + 1;
            for (; s2 + 4 <= k; s2 += 4) {
                LT f[4], v[4][NB];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    f[i] = readlane_t(lm, s2 + i);
#pragma unroll
                    for (int jb = 0; jb < NB; ++jb) v[i][jb] = A[(s2 + i) * LD + col[jb]];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int jb = 0; jb < NB; ++jb) A[(s2 + i) * LD + col[jb]] = v[i][jb] - f[i] * prow[jb];
            }
            for (; s2 < k; ++s2) {
                const LT f = readlane_t(lm, s2);
#pragma unroll
                for (int jb = 0; jb < NB; ++jb) A[s2 * LD + col[jb]] = A[s2 * LD + col[jb]] - f * prow[jb];
            }
            wave_lds_sync();
        }
        if (ok) {
            for (int t = k - 1; t >= 0; --t) {
                const LT d = readlane_t(dreg, t);
                const LT u = A[(lane < t ? lane : t) * LD + t];  // column t of U above the diagonal
                int col[NB];
                LT x[NB];
#pragma unroll
                for (int jb = 0; jb < NB; ++jb) {
                    const int c = lane + 64 * jb;
                    col[jb] = c < nr ? rhs0 + c : t;
                    x[jb] = A[t * LD + col[jb]] / d;
                    A[t * LD + col[jb]] = x[jb];
                }
                int s2 = 0;
                for (; s2 + 4 <= t; s2 += 4) {
                    LT f[4], v[4][NB];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        f[i] = readlane_t(u, s2 + i);
#pragma unroll
                        for (int jb = 0; jb < NB; ++jb) v[i][jb] = A[(s2 + i) * LD + col[jb]];
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int jb = 0; jb < NB; ++jb) A[(s2 + i) * LD + col[jb]] = v[i][jb] - f[i] * x[jb];
                }
                for (; s2 < t; ++s2) {
                    const LT f = readlane_t(u, s2);
#pragma unroll
                    for (int jb = 0; jb < NB; ++jb) A[s2 * LD + col[jb]] = A[s2 * LD + col[jb]] - f * x[jb];
                }
                wave_lds_sync();
            }
        }
        if (lane == 0) {
            sm.ok = ok;
            sm.minpiv = minpiv;
        }
    }
}

// Inverse of the unit lower-triangular k x k matrix in columns [0, k) of A
// (row stride LD; only the part below the diagonal is read) by elimination
// on the right-hand sides [KMAX, KMAX + k), which hold the identity on entry
// and the inverse on exit.  No pivot search: the multipliers of the strip's
// partial-pivot LU are at most 1 in modulus, so partial pivoting would keep
// every diagonal pivot, and the unit pivots make the divisions exact.
// Wavefront 0 only; lane c owns right-hand-side column c (k <= 64).
template <typename T, int KMAX, int LD>
DI void unit_lower_inv_wave0(T* A, int k)
{
    const int lane = threadIdx.x;
    const bool act = lane < k;
    for (int t = 0; t + 1 < k; ++t) {
        const T lm = A[(act ? lane : t) * LD + t];   // lane s: multiplier of row s
        const int col = act ? KMAX + lane : t;       // inactive lanes touch dead column t
        const T prow = act ? A[t * LD + col] : (T)0;
        wave_lds_sync();
        int s2 = t + 1;
        for (; s2 + 4 <= k; s2 += 4) {
            T f[4], v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                f[i] = readlane_t(lm, s2 + i);
                v[i] = A[(s2 + i) * LD + col];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) A[(s2 + i) * LD + col] = v[i] - f[i] * prow;
        }
        for (; s2 < k; ++s2) {
            const T f = readlane_t(lm, s2);
            A[s2 * LD + col] = A[s2 * LD + col] - f * prow;
        }
        wave_lds_sync();
    }
}


// The same inverse with each lane's column in registers (k <= KR <= 32),
// both loops unrolled: per step one batch of broadcast LDS reads of the
// multipliers (column t of L), then the updates; the same operations in the
// same order as above.
template <typename T, int KMAX, int LD, int KR>
DI void unit_lower_inv_reg(T* A, int k)
{
    const int lane = threadIdx.x;
    T x[KR];
#pragma unroll
    for (int r = 0; r < KR; ++r) x[r] = (T)(r == lane ? 1 : 0);
#pragma unroll
    for (int t = 0; t + 1 < KR; ++t) {
        if (t + 1 < k) {
            T l[KR];
#pragma unroll
            for (int s2 = t + 1; s2 < KR; ++s2) l[s2] = A[s2 * LD + t];
#pragma unroll
            for (int s2 = t + 1; s2 < KR; ++s2) x[s2] = x[s2] - l[s2] * x[t];
        }
    }
    if (lane < k) {
#pragma unroll
        for (int r = 0; r < KR; ++r)
            if (r < k) A[r * LD + KMAX + lane] = x[r];
    }
}

template <typename T, int KMAX, int LD>
DI void unit_lower_inv_solve(T* A, int k)
{
    constexpr int K16 = KMAX < 16 ? KMAX : 16, K32 = KMAX < 32 ? KMAX : 32;
    if (k <= 8)
        unit_lower_inv_reg<T, KMAX, LD, 8>(A, k);
    else if (k <= K16)
        unit_lower_inv_reg<T, KMAX, LD, K16>(A, k);
    else if (k <= K32)
        unit_lower_inv_reg<T, KMAX, LD, K32>(A, k);
    else
        unit_lower_inv_wave0<T, KMAX, LD>(A, k);
}

// A column of up to KR values of type LT held in registers, readable and
// writable at a wavefront-uniform run-time row (lowered to register-indexed
// moves; a vector of at most 32 dwords stays in registers, larger arrays
// would go to scratch).  binary64: 16 rows per vector, as dword pairs.
typedef uint32_t u32x32 __attribute__((ext_vector_type(32)));

template <typename LT, int KR>
struct RegCol;

template <int KR>
struct RegCol<double, KR> {
    static constexpr int NV = (KR + 15) / 16;
    u32x32 v[NV];
    DI double get(int r) const
    {
        const u32x32& w = v[r >> 4];
        const int e = 2 * (r & 15);
        return __longlong_as_double((long long)(((uint64_t)w[e + 1] << 32) | w[e]));
    }
    DI void set(int r, double x)
    {
        u32x32& w = v[r >> 4];
        const int e = 2 * (r & 15);
        const uint64_t b = (uint64_t)__double_as_longlong(x);
        w[e] = (uint32_t)b;
        w[e + 1] = (uint32_t)(b >> 32);
    }
    // i uniform across the wavefront; every chunk is indexed (no branch,
    // so no copies of whole vectors), the owning chunk's value is kept
    DI double dget(int i) const
    {
        double x = get_in(v[0], i & 15);
#pragma unroll
        for (int c = 1; c < NV; ++c) {
            const double y = get_in(v[c], i & 15);
            x = (i >> 4) == c ? y : x;
        }
        return x;
    }
    DI void dset(int i, double x)
    {
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            const double old = get_in(v[c], i & 15);
            set_in(v[c], i & 15, (i >> 4) == c ? x : old);
        }
    }
    static DI double get_in(const u32x32& w, int j)
    {
        return __longlong_as_double((long long)(((uint64_t)w[2 * j + 1] << 32) | w[2 * j]));
    }
    static DI void set_in(u32x32& w, int j, double x)
    {
        const uint64_t b = (uint64_t)__double_as_longlong(x);
        w[2 * j] = (uint32_t)b;
        w[2 * j + 1] = (uint32_t)(b >> 32);
    }
};

template <int KR>
struct RegCol<float, KR> {
    static_assert(KR <= 32, "one vector");
    u32x32 v;
    DI float get(int r) const { return __uint_as_float(v[r]); }
    DI void set(int r, float x) { v[r] = __float_as_uint(x); }
    DI float dget(int i) const { return __uint_as_float(v[i]); }
    DI void dset(int i, float x) { v[i] = __float_as_uint(x); }
};

// The same solve with the matrix in registers, for k <= KR <= 32, on any one
// wavefront (each has its own scratch): lane c holds column c (and c + 64
// when NB = 2) of [M | R], rows 0..KR-1, loaded
// once from A and the right-hand-side block stored back at the end, so the
// elimination makes no LDS or global round trip per row.  Per step, lane t
// passes its column through sm.lucol for the pivot search (lane s = row s)
// and sm.lumul carries the multipliers back.  Rows are not interchanged:
// lane s tracks the position its row would have after the interchanges
// (pos), which breaks ties exactly as the interchanging form does, and every
// row sees the same operations in the same order, so the results are the
// same bits.  pv (lane t) is the row chosen at step t; one pass puts the rows
// in pivot order before the back substitution.  Writes sm.ok and sm.minpiv;
// wavefronts that solve with the same M at once write the same values.
template <typename T, int KMAX, typename LT, int LD, int KR, int NB>
DI void lu_reg_wave0(LT* A, int k, int rhs0, int nr, Smem<T, KMAX>& sm)
{
    static_assert(KR <= KMAX && KR <= 32, "rows in registers");
    const int lane = threadIdx.x & 63;
    const int W = k + nr;
    int lc[NB];
    bool act[NB];
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) {
        const int cc = lane + 64 * jb;
        act[jb] = cc < W;
        lc[jb] = cc < k ? cc : (act[jb] ? rhs0 + cc - k : 0);
    }
    RegCol<LT, KR> a[NB];
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
        for (int r = 0; r < KR; ++r) {
            const LT v = A[(r < k ? r : 0) * LD + lc[jb]];
            a[jb].set(r, (act[jb] && r < k) ? v : (LT)0);
        }
    LT* cb = (LT*)sm.lucol[threadIdx.x >> 6];
    LT* lb = (LT*)sm.lumul[threadIdx.x >> 6];
    double minpiv = INFINITY;
    int ok = 1;
    LT dreg = (LT)0;    // lane t: pivot of step t
    int pv = 0;         // lane t: row chosen at step t
    int pos = lane;     // lane s: position of row s
    bool used = false;  // lane s: row s already a pivot row
    for (int t = 0; t < k; ++t) {
        if (lane == t) {
#pragma unroll
            for (int r = 0; r < KR; ++r) cb[r] = a[0].get(r);
        }
        wave_lds_sync();
        const LT cv = cb[lane < KR ? lane : 0];  // lane s: entry s of column t
        K2 key = (!used && lane < k) ? k2_make(fabs((double)cv), pos, lane) : k2_none();
        key = wave_argmax(key);
        const double pav = k2_val(key);
        if (pav == 0.0) {
            ok = 0;
            break;
        }
        minpiv = fmin(minpiv, pav);
        const int p = k2_col(key);
        const LT piv = readlane_t(cv, p);
        if (lane == t) {
            dreg = piv;
            pv = p;
        }
        const int ppos = __builtin_amdgcn_readlane(pos, p);
        const LT lm = (!used && lane < k && lane != p) ? cv / piv : (LT)0;
        if (lane < KR) lb[lane] = lm;
        pos = lane == p ? t : (pos == t ? ppos : pos);
        used = used || lane == p;
        LT prow[NB];
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) prow[jb] = a[jb].dget(p);
        wave_lds_sync();
        LT f[KR];
#pragma unroll
        for (int r = 0; r < KR; ++r) f[r] = lb[r];
#pragma unroll
        for (int rb = 0; rb < KR; rb += 4) {
            if (rb < k) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int jb = 0; jb < NB; ++jb) a[jb].set(rb + i, a[jb].get(rb + i) - f[rb + i] * prow[jb]);
            }
        }
        wave_lds_sync();
    }
    if (ok) {
        // rows in pivot order
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
            RegCol<LT, KR> b;
#pragma unroll
            for (int t = 0; t < KR; ++t) b.set(t, t < k ? a[jb].dget(__builtin_amdgcn_readlane(pv, t)) : (LT)0);
            a[jb] = b;
        }
        bool rhs[NB];
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) rhs[jb] = act[jb] && lane + 64 * jb >= k;
#pragma unroll
        for (int t = KR - 1; t >= 0; --t) {
            if (t < k) {
                const LT d = readlane_t(dreg, t);
                LT x[NB];
#pragma unroll
                for (int jb = 0; jb < NB; ++jb) {
                    x[jb] = rhs[jb] ? a[jb].get(t) / d : (LT)0;
                    a[jb].set(t, rhs[jb] ? x[jb] : a[jb].get(t));
                }
#pragma unroll
                for (int s2 = 0; s2 < t; ++s2) {
                    const LT u = readlane_t(a[0].get(s2), t);
#pragma unroll
                    for (int jb = 0; jb < NB; ++jb) a[jb].set(s2, a[jb].get(s2) - u * x[jb]);
                }
            }
        }
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
            if (rhs[jb])
#pragma unroll
                for (int r = 0; r < KR; ++r)
                    if (r < k) A[r * LD + lc[jb]] = a[jb].get(r);
        }
    }
    if (lane == 0) {
        sm.ok = ok;
        sm.minpiv = minpiv;
    }
}

// The wavefront-0 solve: rows in registers up to k = 32 (NBR column blocks,
// k + nr <= 64 NBR), else the LDS form.
template <typename T, int KMAX, typename LT, int LD, int NB, int NBR>
DI void lu_solve_wave0(LT* A, int k, int rhs0, int nr, Smem<T, KMAX>& sm)
{
    constexpr int K16 = KMAX < 16 ? KMAX : 16, K32 = KMAX < 32 ? KMAX : 32;
    if (k <= 8)
        lu_reg_wave0<T, KMAX, LT, LD, 8, NBR>(A, k, rhs0, nr, sm);
    else if (k <= K16)
        lu_reg_wave0<T, KMAX, LT, LD, K16, NBR>(A, k, rhs0, nr, sm);
    else if (k <= K32)
        lu_reg_wave0<T, KMAX, LT, LD, K32, NBR>(A, k, rhs0, nr, sm);
    else
        lu_aug_wave0<T, KMAX, LT, LD, NB>(A, k, rhs0, nr, sm);
}

// Pins a loaded value in straight-line code: a value used only under a
// condition would otherwise have its load sunk into a branch of its own,
// each with its own wait.  Pin a group of loads after issuing them all.
DI double keep(double v)
{
    asm volatile("" : "+v"(v));
    return v;
}
DI float keep(float v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// Runs body(width, c) over columns [c, end) in chunks of W, then one chunk
// each of 8, 4, 2, 1 as needed: every load inside a chunk is unconditional
// and no column is loaded twice (width is a std::integral_constant).
template <int W, typename BODY>
DI void column_chunks(int c, int end, BODY body)
{
    for (; c + W <= end; c += W) body(std::integral_constant<int, W>{}, c);
    if (W > 8 && c + 8 <= end) { body(std::integral_constant<int, 8>{}, c); c += 8; }
    if (c + 4 <= end) { body(std::integral_constant<int, 4>{}, c); c += 4; }
    if (c + 2 <= end) { body(std::integral_constant<int, 2>{}, c); c += 2; }
    if (c < end) body(std::integral_constant<int, 1>{}, c);
}

// ----------------------------------------------------------------------------
// basis product on the matrix cores: slice <- slice(:, 0:kd) * W, W[d][c] at
// W[d * wsd + c * wsc], d, c < kd.  Each wavefront owns 16-row tiles and
// loads a tile's inputs before storing any output, so it runs in place.
// ----------------------------------------------------------------------------

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

DI d4_t mfma16(double a, double b, d4_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
DI f4_t mfma16(float a, float b, f4_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

template <typename T>
struct Acc4;
template <>
struct Acc4<double> {
    typedef d4_t type;
    // output element r of lane l is row 4 r + l / 16, column l % 16
    static DI int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <>
struct Acc4<float> {
    typedef f4_t type;
    // output element r of lane l is row 4 (l / 16) + r, column l % 16
    static DI int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// KD: the widest kd this instance serves; smaller ranks run the instance of
// their own width, so that no load is issued for steps beyond kd.
template <typename T, int KD>
DI void basis_product_k(const Rows<T>& rw, int kd, const T* W, int wsd, int wsc)
{
    typedef typename Acc4<T>::type acc_t;
    constexpr int KB = KD / 4;
    constexpr int CT = (KD + 15) / 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ntiles = (rw.nrows + 15) / 16;
    // only the 4-deep steps and 16-wide column tiles that k reaches
    const int kbn = (kd + 3) / 4, ctn = (kd + 15) / 16;
    for (int tile = wv; tile < ntiles; tile += NWAVE) {
        const int r = tile * 16 + (lane & 15);
        const bool rok = r < rw.nrows;
        // loads at clamped (in-bounds) indices, all issued before they are
        // pinned, zero selected outside: no per-load branch or wait
        const int rc = rok ? r : 0;
        T a[KB];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const int d = kb * 4 + (lane >> 4);
            a[kb] = rw.B[(d < kd ? d : 0) * rw.ld + rc];
        }
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) a[kb] = keep(a[kb]);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const int d = kb * 4 + (lane >> 4);
            a[kb] = (kb < kbn && rok && d < kd) ? a[kb] : (T)0;
        }
        acc_t out[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            acc_t acc = {0, 0, 0, 0};
            if (ct < ctn) {
                const int c = ct * 16 + (lane & 15);
                T w[KB];
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    const int d = kb * 4 + (lane >> 4);
                    w[kb] = W[(d < kd ? d : 0) * wsd + (c < kd ? c : 0) * wsc];
                }
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) w[kb] = keep(w[kb]);
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    const int d = kb * 4 + (lane >> 4);
                    w[kb] = (d < kd && c < kd) ? w[kb] : (T)0;
                }
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
                    if (kb < kbn) acc = mfma16(a[kb], w[kb], acc);
            }
            out[ct] = acc;
        }
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            if (ct < ctn) {
                const int c = ct * 16 + (lane & 15);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int rr = tile * 16 + Acc4<T>::row(lane, e);
                    if (rr < rw.nrows && c < kd) rw.B[c * rw.ld + rr] = out[ct][e];
                }
            }
        }
    }
}

template <typename T, int KMAX>
DI void basis_product(const Rows<T>& rw, int kd, const T* W, int wsd, int wsc)
{
    constexpr int K16 = KMAX < 16 ? KMAX : 16, K32 = KMAX < 32 ? KMAX : 32;
    if (kd <= 8)
        basis_product_k<T, 8>(rw, kd, W, wsd, wsc);
    else if (kd <= K16)
        basis_product_k<T, K16>(rw, kd, W, wsd, wsc);
    else if (kd <= K32)
        basis_product_k<T, K32>(rw, kd, W, wsd, wsc);
    else
        basis_product_k<T, KMAX>(rw, kd, W, wsd, wsc);
}

// ----------------------------------------------------------------------------
// one maxvol step (Section 6.5): column step (transpose = 0) picks I from
// A[:, J]; row step (transpose = 1) picks J from A[I, :]^T.
// ----------------------------------------------------------------------------

// ----------------------------------------------------------------------------
// The step is split into separately compiled phases (each gets its own
// register allocation; a single inlined kernel spilled scalar registers).
// Callees find their LDS through the extern symbol below, so LDS accesses
// stay ds_* instructions; the team state is copied in and out.
// ----------------------------------------------------------------------------

extern __shared__ __align__(16) unsigned char lra_smem[];

// Dynamic LDS: a small header shared by every variant (the fetched task and
// the team-barrier flag), then the variant's Smem, then its strip rows.
constexpr int LDS_HDR = 64;

DI int32_t* lds_fetch() { return reinterpret_cast<int32_t*>(lra_smem); }
DI int32_t* lds_flag() { return reinterpret_cast<int32_t*>(lra_smem) + 1; }

template <typename T, int KMAX>
DI Smem<T, KMAX>& smem_ref() { return *reinterpret_cast<Smem<T, KMAX>*>(lra_smem + LDS_HDR); }

template <typename T, int KMAX>
DI T* blds_ptr()
{
    return reinterpret_cast<T*>(lra_smem + LDS_HDR + ((sizeof(Smem<T, KMAX>) + 255) & ~(size_t)255));
}

template <typename T, int KMAX>
constexpr int variant_of()
{
    return 4 * (sizeof(T) == 8 ? 1 : 0) + (KMAX <= 8 ? 0 : KMAX <= 16 ? 1 : KMAX <= 32 ? 2 : 3);
}

#define NOINL __device__ __noinline__

// This workgroup's slice of the current strip.
template <typename T, int KMAX, bool LDSB>
DI Rows<T> slice_of(const TaskDesc& td, const Team& tm, int transpose, int64_t& R)
{
    const int64_t M = transpose ? td.n : td.m;
    R = (M + tm.size - 1) / tm.size;
    Rows<T> rw;
    rw.r0 = (int64_t)tm.rank * R;
    const int64_t r1 = rw.r0 + R < M ? rw.r0 + R : M;
    rw.nrows = r1 > rw.r0 ? (int)(r1 - rw.r0) : 0;
    if (LDSB) {
        // an odd leading dimension: a column-parallel access (one row, many
        // columns) spreads over the LDS banks
        rw.B = blds_ptr<T, KMAX>();
        rw.ld = R | 1;
    } else {
        rw.B = (T*)td.strip + rw.r0;
        rw.ld = M;
    }
    return rw;
}

// Warm start: M = Chat^T (Chat = strip[X, :]) beside the identity in AUG;
// the partial-pivot LU solve then leaves M^{-1} in the right half (so that
// B = C Chat^{-1} = C (M^{-1})^T).
template <typename T, int KMAX>
DI void warm_load(const TaskDesc& td, Smem<T, KMAX>& sm, int transpose, bool keep_right)
{
    const int k = sm.k;
    const int64_t* F = transpose ? sm.I : sm.J;
    const int64_t* X = transpose ? sm.J : sm.I;
    constexpr int LD = 2 * KMAX;
    T* AUG = (T*)sm.AUG;
    // M[c][s] = strip(X[s], c); batches as wide as k^2 needs (a small rank in
    // a wide variant would otherwise read or generate mostly repeated entries)
    const int kk = k * k;
    const auto idx = [&](int e, int64_t& i, int64_t& j) {
        const int c = e / k, s2 = e % k;
        i = transpose ? F[c] : X[s2];
        j = transpose ? X[s2] : F[c];
    };
    const auto st = [&](int e, T v) {
        const int c = e / k, s2 = e % k;
        AUG[c * LD + s2] = v;
        if (!keep_right) AUG[c * LD + KMAX + s2] = (T)(c == s2 ? 1 : 0);
    };
    constexpr int PBF = (KMAX * KMAX + NT - 1) / NT, PB4 = PBF < 4 ? PBF : 4;
    if (kk <= NT)
        load_entries<T, 1>(td.src, kk, threadIdx.x, NT, idx, st);
    else if (kk <= PB4 * NT)
        load_entries<T, PB4>(td.src, kk, threadIdx.x, NT, idx, st);
    else
        load_entries<T, PBF>(td.src, kk, threadIdx.x, NT, idx, st);
}

// Warm start from the last step's inverse (binary64): that step ended with
// W = C[X,:]^{-1} maintained through its swaps in AUG's right half (stored as
// W^T); the transposed strip of this step has C'[X',:] = C[X,:]^T, so its
// right half is the transpose of the last one.  Wavefront 0 transposes it in
// place and takes it when ||C'[X',:]||_1 ||W'||_1 u <= 2^-40 (the swaps'
// rounding in W stays far below the decisions' margins); otherwise it
// restores the identity and solves.  Same outputs as the solve: sm.ok,
// sm.minpiv (+inf when carried: the pivot test cannot fail at this
// conditioning, since C[X,:] holds the strip's dominant rows).
template <typename T, int KMAX>
DI void warm_carry_wave0(Smem<T, KMAX>& sm, int k)
{
    constexpr int LD = 2 * KMAX;
    T* AUG = (T*)sm.AUG;
    const int lane = threadIdx.x & 63;
    for (int e = lane; e < k * k; e += 64) {
        const int c = e / k, d = e % k;
        if (c < d) {
            const T a = AUG[c * LD + KMAX + d], b = AUG[d * LD + KMAX + c];
            AUG[c * LD + KMAX + d] = b;
            AUG[d * LD + KMAX + c] = a;
        }
    }
    wave_lds_sync();
    double nc = 0.0, nw = 0.0;
    if (lane < k)
        for (int d = 0; d < k; ++d) {
            nc += fabs((double)AUG[lane * LD + d]);         // row of M = column of C[X,:]
            nw += fabs((double)AUG[lane * LD + KMAX + d]);  // row of W^T = column of W
        }
    const double kappa = __longlong_as_double((long long)wave_max_u64((uint64_t)__double_as_longlong(nc))) *
                         __longlong_as_double((long long)wave_max_u64((uint64_t)__double_as_longlong(nw)));
    if (kappa * 0x1p-53 <= 0x1p-40) {
        if (lane == 0) {
            sm.ok = 1;
            sm.minpiv = INFINITY;
        }
        return;
    }
    for (int e = lane; e < k * k; e += 64) {
        const int c = e / k, d = e % k;
        AUG[c * LD + KMAX + d] = (T)(c == d ? 1 : 0);
    }
    wave_lds_sync();
    lu_solve_wave0<T, KMAX, T, LD, (LD + 63) / 64, 1>(AUG, k, KMAX, k, sm);
}

// Gather this workgroup's rows of the strip and return the team-wide max
// |entry| (+inf when an entry is not finite, -1 when the team failed).  With
// warm, wavefront 0 meanwhile solves the warm-start system (it depends on
// the index sets only), leaving sm.ok and sm.minpiv, while the other
// wavefronts gather.
template <typename T, int KMAX, bool LDSB>
NOINL double gather_phase(const TaskDesc& td, Team& tio, int transpose, int warm)
{
    Team tm = tio;
    Smem<T, KMAX>& sm = smem_ref<T, KMAX>();
    const int k = sm.k;
    const int64_t* F = transpose ? sm.I : sm.J;
    int64_t R;
    const Rows<T> rw = slice_of<T, KMAX, LDSB>(td, tm, transpose, R);
    if ((td.src.kind == 1 || td.src.kind == 2) && threadIdx.x < k)
        sm.pts[threadIdx.x] = transpose ? load_elem(td.src.x, td.src.dtype, F[threadIdx.x])
                                        : load_elem(td.src.y, td.src.dtype, F[threadIdx.x]);
    // the last step's inverse is carried on the binary64 path
    const bool carry = warm && sizeof(T) == 8 && sm.w_valid;
    if (warm) warm_load<T, KMAX>(td, sm, transpose, carry);
    __syncthreads();
    double lmax = 0.0;
    if (warm) {
        if (threadIdx.x < 64) {
            if (carry) warm_carry_wave0<T, KMAX>(sm, k);
            else lu_solve_wave0<T, KMAX, T, 2 * KMAX, (2 * KMAX + 63) / 64, 1>((T*)sm.AUG, k, KMAX, k, sm);
        } else {
            lmax = gather_rows<T, KMAX>(td.src, transpose, sm, F, k, rw, threadIdx.x - 64, NT - 64);
        }
    } else {
        lmax = gather_rows<T, KMAX>(td.src, transpose, sm, F, k, rw, threadIdx.x, NT);
    }
    K2 km = block_argmax(k2_make(lmax, 0, 0), sm, tm);
    trace_ev(tm, EV_WARM_LU, warm);
    km = team_argmax(tm, sm, km, 0, R);
    tio = tm;
    if (tm.failed) return -1.0;
    return k2_val(km);
}

// Partial-pivot LU of the strip (k team-wide pivot searches), then the rows
// of L1 (unit lower) are left in AUG.  Returns the effective rank, or -1 if
// the team failed or the strip has no nonzero entry at all (status set).
template <typename T, int KMAX, bool LDSB>
NOINL int gepp_phase(const TaskDesc& td, Team& tio, int transpose, double thresh)
{
    Team tm = tio;
    Smem<T, KMAX>& sm = smem_ref<T, KMAX>();
    const int k = sm.k;
    int64_t* X = transpose ? sm.J : sm.I;
    int64_t R;
    const Rows<T> rw = slice_of<T, KMAX, LDSB>(td, tm, transpose, R);
    const int64_t rend = rw.r0 + rw.nrows;
    constexpr int LD = 2 * KMAX;
    T* AUG = (T*)sm.AUG;
    int keff = k;
    double bv = -1.0;
    int br = 0;
    for (int r = threadIdx.x; r < rw.nrows; r += NT) {
        const double v = fabs((double)rw.B[r]);
        if (v > bv) { bv = v; br = r; }
    }
    K2 kl = bv >= 0.0 ? k2_make(bv, rw.r0 + br, 0) : k2_none();
    for (int t = 0; t < k; ++t) {
        const K2 wb = block_argmax(kl, sm, tm);
        const int64_t wr = k2_row(wb);
        if (threadIdx.x < k && wr >= rw.r0 && wr < rend) sm.pay[threadIdx.x] = rw.B[threadIdx.x * rw.ld + (wr - rw.r0)];
        const K2 wv = team_argmax(tm, sm, wb, k, R);
        if (tm.failed) { tio = tm; return -1; }
        // a team exchange ends with a barrier after the winning row; alone,
        // the row written above must reach every wavefront
        if (tm.size == 1) __syncthreads();
        const double pav = k2_val(wv);
        if (pav == 0.0 && t == 0) {  // a zero strip: no pivot at all
            if (threadIdx.x == 0) { sm.status = -2; sm.phase = PH_DONE; }
            __syncthreads();
            tio = tm;
            return -1;
        }
        if (pav < thresh || pav == 0.0) { keff = t; break; }
        if (threadIdx.x == 0) X[t] = k2_row(wv);
        // row t of L1: the pivot row's multipliers, a unit diagonal, zeros above
        if (threadIdx.x < k) AUG[t * LD + threadIdx.x] = threadIdx.x < t ? sm.pay[threadIdx.x] : (T)(threadIdx.x == t ? 1 : 0);
        trace_ev(tm, EV_PIVOT, t);
        const T piv = sm.pay[t];
        bv = -1.0;
        for (int r = threadIdx.x; r < rw.nrows; r += NT) {
            T* b = rw.B + r;
            const T l = b[t * rw.ld] / piv;
            b[t * rw.ld] = l;
            column_chunks<8>(t + 1, k, [&](auto w, int c0) {
                constexpr int CW = decltype(w)::value;
                T v[CW], pv[CW];
#pragma unroll
                for (int cc = 0; cc < CW; ++cc) {
                    v[cc] = b[(c0 + cc) * rw.ld];
                    pv[cc] = sm.pay[c0 + cc];
                }
#pragma unroll
                for (int cc = 0; cc < CW; ++cc) {
                    v[cc] = v[cc] - l * pv[cc];
                    b[(c0 + cc) * rw.ld] = v[cc];
                }
                if (c0 == t + 1) {
                    const double a = fabs((double)v[0]);
                    if (a > bv) { bv = a; br = r; }
                }
            });
        }
        // no barrier here: the next reduction's barrier orders these updates
        // before the next pivot row is read and sm.pay is rewritten
        kl = bv >= 0.0 ? k2_make(bv, rw.r0 + br, 0) : k2_none();
    }
    tio = tm;
    return keff;
}

// B = C Chat^{-1} (warm start) or B = L L1^{-1} (after the strip LU) on the
// matrix cores, then the rows of the chosen set become unit rows.
template <typename T, int KMAX, bool LDSB>
NOINL void basis_phase(const TaskDesc& td, Team& tio, int transpose, int started, int keff)
{
    Team tm = tio;
    Smem<T, KMAX>& sm = smem_ref<T, KMAX>();
    const int64_t* X = transpose ? sm.J : sm.I;
    int64_t R;
    const Rows<T> rw = slice_of<T, KMAX, LDSB>(td, tm, transpose, R);
    const int64_t rend = rw.r0 + rw.nrows;
    constexpr int LD = 2 * KMAX;
    T* AUG = (T*)sm.AUG;
    if (started) {
        // W[d][c] = M^{-1}[c][d] sits in the right half of AUG; a copy with c
        // contiguous in the left half (free once the warm start is done)
        // keeps the product's loads of W off a single LDS bank
        for (int e = threadIdx.x; e < keff * keff; e += NT) {
            const int d = e / keff, c = e - d * keff;
            AUG[d * LD + c] = AUG[c * LD + KMAX + d];
        }
        __syncthreads();
        basis_product<T, KMAX>(rw, keff, AUG, LD, 1);
    } else {
        // L1^{-1} by unit-triangular elimination on I, then L L1^{-1}
        for (int e = threadIdx.x; e < keff * keff; e += NT)
            AUG[(e / keff) * LD + KMAX + e % keff] = (T)((e / keff) == (e % keff));
        __syncthreads();
        if (threadIdx.x < 64) unit_lower_inv_solve<T, KMAX, LD>(AUG, keff);
        __syncthreads();
        basis_product<T, KMAX>(rw, keff, AUG + KMAX, LD, 1);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < keff * keff; e += NT) {
        const int s2 = e / keff, c = e % keff;
        const int64_t gr = X[s2];
        if (gr >= rw.r0 && gr < rend) rw.B[c * rw.ld + (gr - rw.r0)] = (T)(c == s2 ? 1 : 0);
    }
    __syncthreads();
    trace_ev(tm, EV_BASIS, started);
    tio = tm;
}

// Swaps: while max|B| > 1 + tau, bring the winning row into its column's
// slot (rank-one update of B; |det| grows by the winning entry).  Returns the
// number of swaps, or -1 if the team failed.
template <typename T, int KMAX, bool LDSB>
NOINL int swap_phase(const TaskDesc& td, Team& tio, int transpose, int keff, int wmaint)
{
    Team tm = tio;
    Smem<T, KMAX>& sm = smem_ref<T, KMAX>();
    int64_t* X = transpose ? sm.J : sm.I;
    // wmaint: AUG's right half holds W^T, W = C[X,:]^{-1}; each swap updates it
    // like B (B = C W: B - B[:,j] g = C (W - W[:,j] g)), so that the next
    // step can start from it
    constexpr int LDW = 2 * KMAX;
    T* Wr = (T*)sm.AUG + KMAX;
    int64_t R;
    const Rows<T> rw = slice_of<T, KMAX, LDSB>(td, tm, transpose, R);
    const int64_t rend = rw.r0 + rw.nrows;
    const double lim = 1.0 + td.tau;
    const int max_swaps = td.max_swaps > 0 ? td.max_swaps : 4 * keff + 64;
    int swaps = 0;
    if (threadIdx.x >= keff && threadIdx.x < KMAX) sm.g[threadIdx.x] = (T)0;
    if (KMAX <= 32 && R <= NT) {
        // at most one row per thread: the row stays in registers for all
        // swaps; columns keff..KMAX-1 are carried as zeros (their g is 0), so
        // the unrolled loops need no per-column guards
        const bool has = threadIdx.x < rw.nrows;
        const int64_t myrow = rw.r0 + threadIdx.x;
        T row[KMAX];
        {
            const T* p = rw.B + (has ? threadIdx.x : 0);
#pragma unroll
            for (int c = 0; c < KMAX; ++c) {
                const T v = *p;
                row[c] = c < keff ? v : (T)0;
                if (c + 1 < keff) p += rw.ld;
            }
        }
        double bv = -1.0;
        int bc = 0;
#pragma unroll
        for (int c = 0; c < KMAX; ++c) {
            const double a = fabs((double)row[c]);
            if (a > bv) { bv = a; bc = c; }
        }
        if (!has) bv = -1.0;
        // the last swap's update of W^T is applied while the next exchange's
        // slots travel (it is needed only once the exchange has returned)
        bool wpend = false;
        const auto wupdate = make_hook([&]() {
            if (wpend)
                for (int e = threadIdx.x; e < keff * keff; e += NT) {
                    const int c = e / keff, d = e % keff;
                    Wr[c * LDW + d] -= (T)sm.lumul[0][d] * sm.g[c];
                }
        });
        const int wave = threadIdx.x >> 6;
        for (;;) {
            const K2 kl = bv >= 0.0 ? k2_make(bv, myrow, bc) : k2_none();
            // each wavefront's best row goes to LDS before the workgroup
            // reduction's barrier, so the winner's row is in place after it
            const K2 ww = wave_argmax(kl);
            if (has && ww.lo != 0ull && k2_row(ww) == myrow) {
#pragma unroll
                for (int c = 0; c < KMAX; ++c) sm.lucol[wave][c] = (double)row[c];
            }
            if ((threadIdx.x & 63) == 0) sm.kred[tm.tog][wave] = ww;
            __syncthreads();
            K2 wb = sm.kred[tm.tog][0];
            int wbw = 0;
#pragma unroll
            for (int i = 1; i < NWAVE; ++i)
                if (k2_better(sm.kred[tm.tog][i], wb)) {
                    wb = sm.kred[tm.tog][i];
                    wbw = i;
                }
            tm.tog ^= 1;
            trace_ev(tm, EV_SWAP_RED, 0);
            const K2 wv = team_argmax(tm, sm, wb, keff, R, wupdate, sm.lucol[wbw]);
            wpend = false;
            if (tm.failed) { tio = tm; return -1; }
            trace_ev(tm, EV_SWAP_XCH, 0);
            if (!(k2_val(wv) > lim)) break;
            if (swaps == max_swaps) {
                if (threadIdx.x == 0) sm.warn |= W_CAP;
                break;
            }
            const int js = k2_col(wv);
            const int64_t is = k2_row(wv);
            if (threadIdx.x < keff) {
                // the winning row: from the exchange, or this workgroup's own
                // when it is the whole team
                const bool own = tm.size == 1;
                const T pc = own ? (T)sm.lucol[wbw][threadIdx.x] : sm.pay[threadIdx.x];
                const T pj = own ? (T)sm.lucol[wbw][js] : sm.pay[js];
                sm.g[threadIdx.x] = (pc - (T)(threadIdx.x == js ? 1 : 0)) / pj;
                if (wmaint) sm.lumul[0][threadIdx.x] = (double)Wr[js * LDW + threadIdx.x];
            }
            if (threadIdx.x == 0) X[js] = is;
            __syncthreads();
            wpend = wmaint != 0;
            ++swaps;
            trace_ev(tm, EV_SWAP, swaps);
            T gv[KMAX];
#pragma unroll
            for (int c = 0; c < KMAX; ++c) gv[c] = sm.g[c];
            T f = (T)0;
#pragma unroll
            for (int c = 0; c < KMAX; ++c) f = c == js ? row[c] : f;
            const bool unit = myrow == is;
            bv = -1.0;
#pragma unroll
            for (int c = 0; c < KMAX; ++c) {
                const T nv = unit ? (T)(c == js ? 1 : 0) : row[c] - f * gv[c];
                row[c] = nv;
                const double a = fabs((double)nv);
                if (a > bv) { bv = a; bc = c; }
            }
            if (!has) bv = -1.0;
        }
    } else {
        double bv = -1.0;
        int br = 0, bc = 0;
        for (int r = threadIdx.x; r < rw.nrows; r += NT)
            for (int c = 0; c < keff; ++c) {
                const double v = fabs((double)rw.B[c * rw.ld + r]);
                if (v > bv) { bv = v; br = r; bc = c; }
            }
        for (;;) {
            const K2 kl = bv >= 0.0 ? k2_make(bv, rw.r0 + br, bc) : k2_none();
            const K2 wb = block_argmax(kl, sm, tm);
            trace_ev(tm, EV_SWAP_RED, 0);
            const int64_t wr = k2_row(wb);
            if (threadIdx.x < keff && wr >= rw.r0 && wr < rend) sm.pay[threadIdx.x] = rw.B[threadIdx.x * rw.ld + (wr - rw.r0)];
            const K2 wv = team_argmax(tm, sm, wb, keff, R);
            if (tm.failed) { tio = tm; return -1; }
            trace_ev(tm, EV_SWAP_XCH, 0);
            if (!(k2_val(wv) > lim)) break;
            if (swaps == max_swaps) {
                if (threadIdx.x == 0) sm.warn |= W_CAP;
                break;
            }
            const int js = k2_col(wv);
            const int64_t is = k2_row(wv);
            if (threadIdx.x < keff) {
                sm.g[threadIdx.x] = (sm.pay[threadIdx.x] - (T)(threadIdx.x == js ? 1 : 0)) / sm.pay[js];
                if (wmaint) sm.lumul[0][threadIdx.x] = (double)Wr[js * LDW + threadIdx.x];
            }
            if (threadIdx.x == 0) X[js] = is;
            __syncthreads();
            if (wmaint)
                for (int e = threadIdx.x; e < keff * keff; e += NT) {
                    const int c = e / keff, d = e % keff;
                    Wr[c * LDW + d] -= (T)sm.lumul[0][d] * sm.g[c];
                }
            ++swaps;
            trace_ev(tm, EV_SWAP, swaps);
            constexpr int CH = KMAX < 16 ? KMAX : 16;
            bv = -1.0;
            for (int r = threadIdx.x; r < rw.nrows; r += NT) {
                T* b = rw.B + r;
                const T f = b[js * rw.ld];
                const bool unit = (rw.r0 + r == is);
                column_chunks<CH>(0, keff, [&](auto w, int c0) {
                    constexpr int CW = decltype(w)::value;
                    T v[CW], gv[CW];
#pragma unroll
                    for (int cc = 0; cc < CW; ++cc) {
                        v[cc] = b[(c0 + cc) * rw.ld];
                        gv[cc] = sm.g[c0 + cc];
                    }
#pragma unroll
                    for (int cc = 0; cc < CW; ++cc) {
                        const int c = c0 + cc;
                        const T nv = unit ? (T)(c == js ? 1 : 0) : v[cc] - f * gv[cc];
                        b[c * rw.ld] = nv;
                        const double a = fabs((double)nv);
                        if (a > bv) { bv = a; br = r; bc = c; }
                    }
                });
            }
        }
    }
    trace_ev(tm, EV_STEP_END, swaps);
    __syncthreads();
    tio = tm;
    return swaps;
}

// ----------------------------------------------------------------------------
// swaps with a BF16 shortlist (binary32 path, k <= 32, one row per thread, the
// slice in LDS).  The basis is never formed: W = C[X,:]^{-1} (binary32, from
// the warm-start solve) is kept and updated by the same rank-one formula as
// B (B = C W, so B - B[:,j] g = C (W - W[:,j] g)).  Each round:
//   1. the selection product C W on the matrix cores with both operands
//      rounded to bfloat16 and binary32 accumulation (16x16x32 tiles) into
//      an LDS copy beside the slice;
//   2. every row's largest approximate entry, the 8 best rows of each
//      wavefront (rows of X excluded);
//   3. those rows' entries recomputed in binary32 (C[i,:] W), their exact
//      argmax reduced over the workgroup and exchanged over the team with the
//      winning row as payload; the stop test and the swap use these values.
// With entrywise error d of the bfloat16 product, the true argmax is on the
// shortlist whenever it leads the rest by more than 2 d, and at the stop
// every |C W| entry is at most 1 + tau + 2 d.
// ----------------------------------------------------------------------------

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

DI uint64_t shfl_xor_u64(uint64_t v, int m)
{
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

template <typename T, int KMAX>
NOINL int swap_phase_bsel(const TaskDesc& td, Team& tio, int transpose, int keff)
{
    Team tm = tio;
    Smem<T, KMAX>& sm = smem_ref<T, KMAX>();
    int64_t* X = transpose ? sm.J : sm.I;
    int64_t R;
    const Rows<T> rw = slice_of<T, KMAX, true>(td, tm, transpose, R);
    float* Bs = (float*)rw.B + rw.ld * KMAX;  // approximate C W, column-major, ld R
    constexpr int LD = 2 * KMAX;
    float* Wt = (float*)sm.AUG + KMAX;    // Wt[c * LD + a] = W[a][c]
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double lim = 1.0 + td.tau;
    const int max_swaps = td.max_swaps > 0 ? td.max_swaps : 4 * keff + 64;
    const bool has = threadIdx.x < rw.nrows;
    const int64_t myrow = rw.r0 + threadIdx.x;
    bool inX = false;
    for (int c = 0; c < keff; ++c) inX = inX || (X[c] == myrow);
    const int ntiles = (rw.nrows + 15) / 16;
    const int ctn = (keff + 15) / 16;
    int swaps = 0;
    for (;;) {
        // 1. selection product in bfloat16, binary32 accumulation
        for (int tile = wv; tile < ntiles; tile += NWAVE) {
            const int r = tile * 16 + (lane & 15);
            const int rc = r < rw.nrows ? r : 0;
            bf16x8 a;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int d = 8 * (lane >> 4) + j;
                const float v = rw.B[(d < keff ? d : 0) * rw.ld + rc];
                a[j] = (__bf16)(d < keff ? v : 0.0f);
            }
            for (int ct = 0; ct < ctn; ++ct) {
                const int c = ct * 16 + (lane & 15);
                bf16x8 b;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int d = 8 * (lane >> 4) + j;
                    const float v = Wt[(c < keff ? c : 0) * LD + (d < keff ? d : 0)];
                    b[j] = (__bf16)((d < keff && c < keff) ? v : 0.0f);
                }
                f4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int rr = tile * 16 + 4 * (lane >> 4) + e;
                    if (rr < rw.nrows && c < keff) Bs[c * R + rr] = acc[e];
                }
            }
        }
        __syncthreads();
        // 2. this row's largest approximate entry; the wavefront's 8 best rows
        K2 key = k2_none();
        {
            // all of the row's loads first (clamped columns), then the scan
            const int rr = has ? (int)threadIdx.x : 0;
            float bsv[KMAX];
#pragma unroll
            for (int c = 0; c < KMAX; ++c) bsv[c] = Bs[(c < keff ? c : 0) * R + rr];
            float bv = -1.0f;
            int bc = 0;
#pragma unroll
            for (int c = 0; c < KMAX; ++c) {
                const float v = c < keff ? fabsf(bsv[c]) : -1.0f;
                if (v > bv) {
                    bv = v;
                    bc = c;
                }
            }
            if (has && !inX) key = k2_make((double)bv, myrow, bc);
        }
        K2 cand[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            cand[q] = wave_argmax(key);
            if (key.hi == cand[q].hi && key.lo == cand[q].lo) key = k2_none();
        }
        trace_ev(tm, EV_SWAP_RED, 1);
        // 3. recheck in binary32: lanes 8q .. 8q + 7 take candidate q, columns
        //    lane % 8 + 8 j
        const int q = lane >> 3, c0 = lane & 7;
        K2 mc = cand[0];
#pragma unroll
        for (int qq = 1; qq < 8; ++qq)
            if (qq == q) mc = cand[qq];
        const bool valid = mc.lo != 0ull;
        const int lr = valid ? (int)(k2_row(mc) - rw.r0) : 0;
        constexpr int NJ = (KMAX + 7) / 8;
        float ex[NJ];
        K2 best = k2_none();
        // the candidate row of C, loaded once (clamped columns, zero past k)
        float cr[KMAX];
#pragma unroll
        for (int a = 0; a < KMAX; ++a) cr[a] = rw.B[(a < keff ? a : 0) * rw.ld + lr];
#pragma unroll
        for (int a = 0; a < KMAX; ++a) cr[a] = a < keff ? cr[a] : 0.0f;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int c = c0 + 8 * j;
            const int cc = c < keff ? c : 0;
            float wr[KMAX];
#pragma unroll
            for (int a = 0; a < KMAX; ++a) wr[a] = Wt[cc * LD + (a < keff ? a : 0)];
#pragma unroll
            for (int a = 0; a < KMAX; ++a) wr[a] = a < keff ? wr[a] : 0.0f;
            float acc = 0.0f;
#pragma unroll
            for (int a = 0; a < KMAX; ++a) acc = fmaf(cr[a], wr[a], acc);
            ex[j] = acc;
            if (valid && c < keff) {
                const K2 kk = k2_make(fabs((double)acc), k2_row(mc), c);
                if (k2_better(kk, best)) best = kk;
            }
        }
#pragma unroll
        for (int o = 4; o >= 1; o >>= 1) {
            const K2 other{shfl_xor_u64(best.hi, o), shfl_xor_u64(best.lo, o)};
            if (k2_better(other, best)) best = other;
        }
        const K2 gb = block_argmax(best, sm, tm);
        if (valid && gb.lo != 0ull && k2_row(mc) == k2_row(gb)) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int c = c0 + 8 * j;
                if (c < keff) sm.pay[c] = ex[j];
            }
        }
        __syncthreads();
        const K2 wv2 = team_argmax(tm, sm, gb, keff, R);
        if (tm.failed) {
            tio = tm;
            return -1;
        }
        trace_ev(tm, EV_SWAP_XCH, 1);
        if (!(k2_val(wv2) > lim)) break;
        if (swaps == max_swaps) {
            if (threadIdx.x == 0) sm.warn |= W_CAP;
            break;
        }
        const int js = k2_col(wv2);
        const int64_t is = k2_row(wv2);
        const int64_t was = X[js];
        if (threadIdx.x < keff) {
            sm.g[threadIdx.x] = (sm.pay[threadIdx.x] - (T)(threadIdx.x == js ? 1 : 0)) / sm.pay[js];
            sm.lumul[0][threadIdx.x] = Wt[js * LD + threadIdx.x];  // W[:, js]
        }
        __syncthreads();
        if (threadIdx.x == 0) X[js] = is;
        for (int e = threadIdx.x; e < keff * keff; e += NT) {
            const int c = e / keff, a = e % keff;
            Wt[c * LD + a] -= (float)sm.lumul[0][a] * sm.g[c];
        }
        inX = has && (myrow == is || (inX && myrow != was));
        ++swaps;
        trace_ev(tm, EV_SWAP, swaps);
        __syncthreads();
    }
    trace_ev(tm, EV_STEP_END, swaps);
    __syncthreads();
    tio = tm;
    return swaps;
}

// ----------------------------------------------------------------------------
// one maxvol step (Section 6.5): column step (transpose = 0) picks I from
// A[:, J]; row step (transpose = 1) picks J from A[I, :]^T.
// ----------------------------------------------------------------------------

template <typename T, int KMAX, bool LDSB>
DI void maxvol_step(const TaskDesc& td, Team& tm, int transpose, int lds_b_bytes)
{
    Smem<T, KMAX>& sm = smem_ref<T, KMAX>();
    const int k = sm.k;
    const int64_t M = transpose ? td.n : td.m;
    const bool have_X = transpose ? true : (sm.have_I != 0);
    const bool warm = have_X && td.warm_start;
    const double u = sizeof(T) == 8 ? 0x1p-53 : 0x1p-24;
    // the BF16 shortlist needs one row per thread and room for the
    // approximate product beside the slice in LDS
    bool bsel = false;
    if constexpr (std::is_same<T, float>::value && KMAX <= 32 && LDSB) {
        const int64_t R = (M + tm.size - 1) / tm.size;
        bsel = td.bf16_select != 0 && R <= NT && ((R | 1) + R) * KMAX * (int64_t)sizeof(T) <= lds_b_bytes;
    }
    trace_ev(tm, EV_STEP_BEGIN, transpose);

    const double cmax = gather_phase<T, KMAX, LDSB>(td, tm, transpose, warm ? 1 : 0);
    if (tm.failed) return;
    const int warm_ok = warm ? sm.ok : 0;
    const double minpiv = sm.minpiv;
    __syncthreads();
    if (threadIdx.x == 0) sm.w_valid = 0;  // AUG is this step's from here on
    if (threadIdx.x == 0) sm.entries_read += M * k;
    if (isinf(cmax)) {
        if (threadIdx.x == 0) { sm.status = -6; sm.phase = PH_DONE; }
        __syncthreads();
        return;
    }
    const double thresh = 64.0 * u * cmax;
    trace_ev(tm, EV_GATHERED, 0);

    int started = warm_ok && minpiv > thresh;
    int keff = k;
    if (!started) {
        keff = gepp_phase<T, KMAX, LDSB>(td, tm, transpose, thresh);
        if (keff < 0) return;
        if (bsel && keff == k) {
            // the shortlist works from C and C[X,:]^{-1}: gather the strip
            // again and solve with the LU start's rows, as a warm start
            gather_phase<T, KMAX, LDSB>(td, tm, transpose, 1);
            if (tm.failed) return;
            if (threadIdx.x == 0) sm.entries_read += M * k;
            started = sm.ok && sm.minpiv > thresh;
            if (!started) {
                keff = gepp_phase<T, KMAX, LDSB>(td, tm, transpose, thresh);
                if (keff < 0) return;
            }
        }
        bsel = bsel && started;
    }
    // binary64 warm steps keep C[X,:]^{-1} current through the swaps for the
    // next step (the binary32 path solves every step)
    const int wmaint = (sizeof(T) == 8 && started) ? 1 : 0;
    int swaps;
    if constexpr (std::is_same<T, float>::value && KMAX <= 32 && LDSB) {
        if (bsel) {
            swaps = swap_phase_bsel<T, KMAX>(td, tm, transpose, keff);
        } else {
            basis_phase<T, KMAX, LDSB>(td, tm, transpose, started, keff);
            swaps = swap_phase<T, KMAX, LDSB>(td, tm, transpose, keff, wmaint);
        }
    } else {
        basis_phase<T, KMAX, LDSB>(td, tm, transpose, started, keff);
        swaps = swap_phase<T, KMAX, LDSB>(td, tm, transpose, keff, wmaint);
    }
    if (swaps < 0) return;
    if (wmaint) {
        if (threadIdx.x == 0) sm.w_valid = 1;
        // a copy in the problem's work buffer for a later launch (serving)
        if (tm.rank == 0 && td.work) {
            GL T* wg = gl((T*)td.work);
            const T* Wr = (const T*)sm.AUG + KMAX;
            for (int e = threadIdx.x; e < keff * keff; e += NT) wg[e] = Wr[(e / keff) * 2 * KMAX + e % keff];
        }
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

// The slice lives in LDS when this workgroup's rows fit, else in the global
// strip buffer; both variants are compiled so that LDS accesses stay ds_* ops.
template <typename T, int KMAX>
DI void maxvol_dispatch(const TaskDesc& td, Team& tm, int transpose, int lds_b_bytes)
{
    Smem<T, KMAX>& sm = smem_ref<T, KMAX>();
    const int64_t M = transpose ? td.n : td.m;
    const int64_t R = (M + tm.size - 1) / tm.size;
    trace_ev(tm, EV_DISPATCH, transpose);
    if ((R | 1) * sm.k * (int64_t)sizeof(T) <= lds_b_bytes) maxvol_step<T, KMAX, true>(td, tm, transpose, lds_b_bytes);
    else maxvol_step<T, KMAX, false>(td, tm, transpose, lds_b_bytes);
}

// ----------------------------------------------------------------------------
// optional CUR factors: C = A[:, J] (m x k column-major), R = A[I, :] (k x n)
// ----------------------------------------------------------------------------

template <typename T, int KMAX>
NOINL void write_factors(const TaskDesc& td, Smem<T, KMAX>& sm, const Team& tm)
{
    const int k = sm.k;
    // descriptor fields read once, before any store (a store could alias them)
    const DevSource src = td.src;
    const int64_t m = td.m, n = td.n;
    GL T* const C = (GL T*)td.C_out;
    GL T* const Rm = (GL T*)td.R_out;
    if (C) {
        const int64_t R = (m + tm.size - 1) / tm.size;
        const int64_t a = (int64_t)tm.rank * R, b = a + R < m ? a + R : m;
        const int rows = b > a ? (int)(b - a) : 0;
        for (int c = 0; c < k; ++c) {
            const int64_t jc = sm.J[c];
            load_entries<T, 8>(
                src, rows, threadIdx.x, NT,
                [&](int e, int64_t& i, int64_t& j) {
                    i = a + e;
                    j = jc;
                },
                [&](int e, T v) { C[c * m + a + e] = v; });
        }
    }
    if (Rm) {
        const int64_t R = (n + tm.size - 1) / tm.size;
        const int64_t a = (int64_t)tm.rank * R, b = a + R < n ? a + R : n;
        const int cols = b > a ? (int)(b - a) : 0;
        for (int c = 0; c < k; ++c) {
            const int64_t ic = sm.I[c];
            load_entries<T, 8>(
                src, cols, threadIdx.x, NT,
                [&](int e, int64_t& i, int64_t& j) {
                    i = ic;
                    j = a + e;
                },
                [&](int e, T v) { Rm[c * n + a + e] = v; });
        }
    }
}

// Fixed-order block sums of NV values (every thread passes its partials; all
// get the totals): a butterfly inside each wavefront, then the wavefront
// partials in order, with one workgroup barrier.
template <int NV, typename T, int KMAX>
DI void block_sums(double (&v)[NV], Smem<T, KMAX>& sm)
{
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v[i] += __shfl_xor(v[i], o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) sm.red[i * NWAVE + wv] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double r = sm.red[i * NWAVE];
#pragma unroll
        for (int w = 1; w < NWAVE; ++w) r += sm.red[i * NWAVE + w];
        v[i] = r;
    }
    __syncthreads();
}

// ----------------------------------------------------------------------------
// nucleus U = A[I,J]^{-1} and the sampled residual (leader workgroup only)
// ----------------------------------------------------------------------------

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

// The Primitive algorithm's nucleus (Section 6.5): U = (G)_r^+, the
// pseudo-inverse of the rank-r truncation of the generator, by the one-sided
// Jacobi method (Hestenes): W = G V with V = I at the start, rotating column
// pairs of W and V until every pair is orthogonal to working precision
// (|w_p . w_q| <= k u ||w_p|| ||w_q||, at most 100 sweeps).  Each sweep is a
// round-robin tournament of k - 1 rounds (k + 1 for odd k, with a padding
// column that is never rotated); in a round, disjoint pairs rotate at once,
// one pair per group of 8 lanes.  Then sigma_j = ||W[:,j]||, and with the
// r largest (ties: smaller j) U[a][b] = sum_t V[a][j_t] W[b][j_t] / sigma^2.
// F = [G | I | A[I,S]] (row stride LDF) on entry; on exit the middle block
// holds U and the right block U A[I,S]; sm.ok = (sigma_{j_r} > 0).
// jb: when F lives in global memory, LDS room for W and V (2 KMAX (KMAX + 1)
// doubles): the sweeps run there (odd row stride: the 8 rows a lane group
// reads fall in different banks), and the result is copied back; nullptr:
// the sweeps run on F in place.
template <typename T, int KMAX, int LDF>
DI void jacobi_pinv(double* F, int k, int r, int s, Smem<T, KMAX>& sm, double* jb)
{
    const int kk = k + (k & 1);
    const int npair = kk / 2;
    const int grp = threadIdx.x >> 3, g8 = threadIdx.x & 7;
    const double eps = (double)k * 0x1p-53;
    constexpr int JLD = KMAX + 1;
    double* Wb = jb ? jb : F;
    double* Vb = jb ? jb + KMAX * JLD : F + KMAX;
    const int ld = jb ? JLD : LDF;
    if (jb) {
        for (int e = threadIdx.x; e < k * k; e += NT) {
            const int i = e / k, c = e - i * k;
            Wb[i * JLD + c] = F[i * LDF + c];
            Vb[i * JLD + c] = F[i * LDF + KMAX + c];
        }
        __syncthreads();
    }
    for (int sweep = 0; sweep < 100; ++sweep) {
        if (threadIdx.x == 0) sm.flag = 0;
        __syncthreads();
        for (int round = 0; round < kk - 1; ++round) {
            if (grp < npair) {
                const int a = grp, b = kk - 1 - grp;
                const int pa = a == 0 ? 0 : (a - 1 + round) % (kk - 1) + 1;
                const int pb = (b - 1 + round) % (kk - 1) + 1;
                const int P = pa < pb ? pa : pb, Qc = pa < pb ? pb : pa;
                // whole 8-lane groups take this branch together (DPP sums)
                if (Qc < k) {
                    // rows g8, g8 + 8, ...: every load before any store
                    constexpr int RPT = (KMAX + 7) / 8;
                    double wp[RPT], wq[RPT], vp[RPT], vq[RPT];
#pragma unroll
                    for (int e = 0; e < RPT; ++e) {
                        const int i = g8 + 8 * e < k ? g8 + 8 * e : g8;
                        wp[e] = Wb[i * ld + P];
                        wq[e] = Wb[i * ld + Qc];
                        vp[e] = Vb[i * ld + P];
                        vq[e] = Vb[i * ld + Qc];
                    }
                    double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                    for (int e = 0; e < RPT; ++e)
                        if (g8 + 8 * e < k) {
                            al += wp[e] * wp[e];
                            be += wq[e] * wq[e];
                            ga += wp[e] * wq[e];
                        }
                    al = sum8(al);
                    be = sum8(be);
                    ga = sum8(ga);
                    if (fabs(ga) > eps * sqrt(al * be)) {
                        const double zeta = (be - al) / (2.0 * ga);
                        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                        const double c = 1.0 / sqrt(1.0 + t * t);
                        const double sn = c * t;
#pragma unroll
                        for (int e = 0; e < RPT; ++e) {
                            const int i = g8 + 8 * e;
                            if (i < k) {
                                Wb[i * ld + P] = c * wp[e] - sn * wq[e];
                                Wb[i * ld + Qc] = sn * wp[e] + c * wq[e];
                                Vb[i * ld + P] = c * vp[e] - sn * vq[e];
                                Vb[i * ld + Qc] = sn * vp[e] + c * vq[e];
                            }
                        }
                        if (g8 == 0) sm.flag = 1;
                    }
                }
            }
            __threadfence_block();
            __syncthreads();
        }
        const int rotated = sm.flag;
        __syncthreads();
        if (threadIdx.x == 0) sm.jsweeps = sweep + 1;
        if (!rotated) break;
    }
    if (jb) {
        for (int e = threadIdx.x; e < k * k; e += NT) {
            const int i = e / k, c = e - i * k;
            F[i * LDF + c] = Wb[i * JLD + c];
            F[i * LDF + KMAX + c] = Vb[i * JLD + c];
        }
        __threadfence_block();
        __syncthreads();
    }
    // singular values and their order (decreasing; ties by index)
    double* sv = sm.pts;
    if (threadIdx.x < k) {
        double s2 = 0.0;
        for (int i = 0; i < k; ++i) s2 += F[i * LDF + threadIdx.x] * F[i * LDF + threadIdx.x];
        sv[threadIdx.x] = sqrt(s2);
    }
    __syncthreads();
    if (threadIdx.x < k) {
        const int j = threadIdx.x;
        int pos = 0;
        for (int i = 0; i < k; ++i) pos += (sv[i] > sv[j] || (sv[i] == sv[j] && i < j)) ? 1 : 0;
        sm.perm[pos] = j;
    }
    __syncthreads();
    constexpr int PE = (KMAX * KMAX + NT - 1) / NT;
    double u[PE];
#pragma unroll
    for (int q = 0; q < PE; ++q) {
        const int e = threadIdx.x + q * NT;
        double acc = 0.0;
        if (e < k * k) {
            const int a = e / k, b = e % k;
            for (int t = 0; t < r; ++t) {
                const int j = sm.perm[t];
                acc += F[a * LDF + KMAX + j] * (F[b * LDF + j] / (sv[j] * sv[j]));
            }
        }
        u[q] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PE; ++q) {
        const int e = threadIdx.x + q * NT;
        if (e < k * k) F[(e / k) * LDF + KMAX + e % k] = u[q];
    }
    __threadfence_block();
    __syncthreads();
    // U A[I,S] over the right block (A[I,S] read before any of it is overwritten;
    // k s <= 64 KMAX entries)
    constexpr int PW = (KMAX * 64 + NT - 1) / NT;
    double w[PW];
#pragma unroll
    for (int q = 0; q < PW; ++q) {
        const int e = threadIdx.x + q * NT;
        double acc = 0.0;
        if (e < k * s) {
            const int a = e / s, b = e % s;
            for (int c = 0; c < k; ++c) acc += F[a * LDF + KMAX + c] * F[c * LDF + KMAX + k + b];
        }
        w[q] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PW; ++q) {
        const int e = threadIdx.x + q * NT;
        if (e < k * s) F[(e / s) * LDF + KMAX + k + e % s] = w[q];
    }
    if (threadIdx.x == 0) sm.ok = sv[sm.perm[r - 1]] > 0.0 ? 1 : 0;
    __threadfence_block();
    __syncthreads();
}

// FLDS: the work matrices fit the workgroup's LDS (else they live in the
// problem's global work buffer); a compile-time choice keeps LDS accesses
// ds_* instructions.
template <typename T, int KMAX, bool FLDS>
DI void final_core(const TaskDesc& td, Team& tio, int lds_b_bytes)
{
    Team tm = tio;
    Smem<T, KMAX>& sm = smem_ref<T, KMAX>();
    const int k = sm.k;
    const int q = td.q, s = td.s;
    // descriptor fields read once, before any store (a store could alias them)
    GL double* const Gout = gl(td.G);
    GL double* const Uout = gl(td.U);
    const GL int64_t* const Qi = gl(td.Q);
    const GL int64_t* const Si = gl(td.S);
    const DevSource src = td.src;
    const int ntr = td.nucleus_rank;
    // F = [G | I | A[I,S]] (row stride LDF; s <= 64), then A[Q,J] and A[Q,S]
    constexpr int LDF = 2 * KMAX + 64;
    double* Fm = FLDS ? (double*)blds_ptr<T, KMAX>() : td.work;
    double* AQJ = Fm + (int64_t)KMAX * LDF;
    double* E = AQJ + (int64_t)q * k;
    load_entries<double, 8>(
        src, k * k, threadIdx.x, NT,
        [&](int e, int64_t& i, int64_t& j) {
            i = sm.I[e / k];
            j = sm.J[e % k];
        },
        [&](int e, double v) {
            const int a = e / k, t = e % k;
            Fm[a * LDF + t] = v;
            Fm[a * LDF + KMAX + t] = a == t ? 1.0 : 0.0;
            Gout[e] = v;
        });
    load_entries<double, 8>(
        src, k * s, threadIdx.x, NT,
        [&](int e, int64_t& i, int64_t& j) {
            i = sm.I[e / s];
            j = Si[e % s];
        },
        [&](int e, double v) { Fm[(e / s) * LDF + KMAX + k + e % s] = v; });
    __threadfence_block();
    __syncthreads();
    // ||G||_1 before the factorisation overwrites G
    double cg = 0.0;
    if (threadIdx.x < k)
        for (int a = 0; a < k; ++a) cg += fabs(Fm[a * LDF + threadIdx.x]);
    const double ng = k2_val(block_argmax(k2_make(cg, 0, 0), sm, tm));
    __syncthreads();
    // U = G^{-1} and W = G^{-1} A[I,S] by partial-pivot LU solves.  k <= 32:
    // three wavefronts each solve G against a third of the right-hand sides
    // (I; the first and the last 32 columns of A[I,S]) with one column block
    // per lane -- the same pivots, so the same bits as one solve -- while
    // wavefront 3 fetches A[Q,J] and A[Q,S].  Larger k: one solve on
    // wavefront 0, the fetches on the other three.
    constexpr int K32 = KMAX < 32 ? KMAX : 32;
    if (ntr > 0 && ntr < k) {
        // truncated nucleus: the sample blocks first, then the SVD
        load_entries<double, 8>(
            src, q * k, threadIdx.x, NT,
            [&](int e, int64_t& i, int64_t& j) {
                i = Qi[e / k];
                j = sm.J[e % k];
            },
            [&](int e, double v) { AQJ[e] = v; });
        load_entries<double, 8>(
            src, q * s, threadIdx.x, NT,
            [&](int e, int64_t& i, int64_t& j) {
                i = Qi[e / s];
                j = Si[e % s];
            },
            [&](int e, double v) { E[e] = v; });
        // work matrices in global memory: the sweeps run in the (now unused)
        // strip LDS when W and V fit there
        const bool stage = !FLDS && (int64_t)2 * KMAX * (KMAX + 1) * 8 <= lds_b_bytes;
        jacobi_pinv<T, KMAX, LDF>(Fm, k, ntr, s, sm, stage ? (double*)blds_ptr<T, KMAX>() : nullptr);
    } else if (k <= K32 && s <= 64) {
        const int wv = threadIdx.x >> 6;
        if (wv == 0) {
            lu_solve_wave0<T, KMAX, double, LDF, (2 * KMAX + 127) / 64, 1>(Fm, k, KMAX, k, sm);
        } else if (wv == 1) {
            lu_solve_wave0<T, KMAX, double, LDF, (2 * KMAX + 127) / 64, 1>(Fm, k, KMAX + k, s < 32 ? s : 32, sm);
        } else if (wv == 2) {
            if (s > 32) lu_solve_wave0<T, KMAX, double, LDF, (2 * KMAX + 127) / 64, 1>(Fm, k, KMAX + k + 32, s - 32, sm);
        } else {
            load_entries<double, 8>(
                src, q * k, threadIdx.x - 192, 64,
                [&](int e, int64_t& i, int64_t& j) {
                    i = Qi[e / k];
                    j = sm.J[e % k];
                },
                [&](int e, double v) { AQJ[e] = v; });
            load_entries<double, 8>(
                src, q * s, threadIdx.x - 192, 64,
                [&](int e, int64_t& i, int64_t& j) {
                    i = Qi[e / s];
                    j = Si[e % s];
                },
                [&](int e, double v) { E[e] = v; });
        }
    } else if (threadIdx.x < 64) {
        lu_solve_wave0<T, KMAX, double, LDF, (2 * KMAX + 127) / 64, 2>(Fm, k, KMAX, k + s, sm);
    } else {
        load_entries<double, 8>(
            src, q * k, threadIdx.x - 64, NT - 64,
            [&](int e, int64_t& i, int64_t& j) {
                i = Qi[e / k];
                j = sm.J[e % k];
            },
            [&](int e, double v) { AQJ[e] = v; });
        load_entries<double, 8>(
            src, q * s, threadIdx.x - 64, NT - 64,
            [&](int e, int64_t& i, int64_t& j) {
                i = Qi[e / s];
                j = Si[e % s];
            },
            [&](int e, double v) { E[e] = v; });
    }
    __threadfence_block();
    __syncthreads();
    if (!sm.ok) {
        if (threadIdx.x == 0) { sm.status = -2; sm.phase = PH_DONE; }
        __syncthreads();
        tio = tm;
        return;
    }
    __threadfence_block();
    __syncthreads();
    for (int e = threadIdx.x; e < k * k; e += NT) Uout[e] = Fm[(e / k) * LDF + KMAX + e % k];
    const double* W = Fm + KMAX + k;  // W[t][b] at W[t * LDF + b]
    double cu = 0.0;
    if (threadIdx.x < k)
        for (int a = 0; a < k; ++a) cu += fabs(Fm[a * LDF + KMAX + threadIdx.x]);
    const double nu = k2_val(block_argmax(k2_make(cu, 0, 0), sm, tm));
    // E_QS = A[Q,S] - A[Q,J] W on the matrix cores: 16 x 16 output tiles
    // spread over the wavefronts, k in steps of 4; loads at clamped indices,
    // zero selected outside q, s and k
    double se = 0.0, sa = 0.0, sum = 0.0;
    {
        constexpr int KB = KMAX / 4;
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int kbn = (k + 3) / 4;
        const int ctn = (s + 15) / 16, ntiles = ((q + 15) / 16) * ctn;
        for (int tile = wv; tile < ntiles; tile += NWAVE) {
            const int r0 = (tile / ctn) * 16, c0 = (tile % ctn) * 16;
            const int r = r0 + (lane & 15), c = c0 + (lane & 15);
            const int rc = r < q ? r : 0, cc = c < s ? c : 0;
            double av[KB], wv4[KB];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                const int d = kb * 4 + (lane >> 4);
                const int dc = d < k ? d : 0;
                av[kb] = AQJ[rc * k + dc];
                wv4[kb] = W[dc * LDF + cc];
            }
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                av[kb] = keep(av[kb]);
                wv4[kb] = keep(wv4[kb]);
            }
            d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                if (kb < kbn) {
                    const int d = kb * 4 + (lane >> 4);
                    const double x = (d < k && r < q) ? av[kb] : 0.0;
                    const double y = (d < k && c < s) ? wv4[kb] : 0.0;
                    acc = mfma16(x, y, acc);
                }
            }
#pragma unroll
            for (int e4 = 0; e4 < 4; ++e4) {
                const int rr = r0 + Acc4<double>::row(lane, e4);
                if (rr < q && c < s) {
                    const double a0 = E[rr * s + c];
                    const double ev = a0 - acc[e4];
                    E[rr * s + c] = ev;
                    se += ev * ev;
                    sa += a0 * a0;
                    sum += ev;
                }
            }
        }
    }
    {
        double r[3] = {se, sa, sum};
        block_sums<3>(r, sm);
        se = r[0];
        sa = r[1];
        sum = r[2];
    }
    const double cnt = (double)q * (double)s;
    const double mean = sum / cnt;
    double vs = 0.0;
    for (int e = threadIdx.x; e < q * s; e += NT) vs += (E[e] - mean) * (E[e] - mean);
    {
        double r[1] = {vs};
        block_sums<1>(r, sm);
        vs = r[0];
    }
    if (threadIdx.x == 0) {
        const double ne = sqrt(se), na = sqrt(sa);
        sm.cond1 = ng * nu;
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
            const int room = td.kmax - k < td.kstep ? td.kmax - k : td.kstep;
            int added = 0;
            while (added < room && sm.cand_next < td.n_cand) {
                const int64_t cnd = gl(td.cand)[sm.cand_next++];
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
                sm.w_valid = 0;
                sm.sweep_in_level = 0;
                sm.phase = PH_COL;
            }
        }
    }
    __syncthreads();
    tio = tm;
}

template <typename T, int KMAX>
NOINL void final_leader(const TaskDesc& td, Team& tio, int lds_b_bytes)
{
    constexpr int LDF = 2 * KMAX + 64;
    const int64_t need = (int64_t)KMAX * LDF + (int64_t)td.q * smem_ref<T, KMAX>().k + (int64_t)td.q * td.s;
    if (need * 8 <= lds_b_bytes) final_core<T, KMAX, true>(td, tio, lds_b_bytes);
    else final_core<T, KMAX, false>(td, tio, lds_b_bytes);
}

// ----------------------------------------------------------------------------
// the Cynical step (Section 6.5; Section 12.2, Tests 3 and 4): an r x r
// submatrix of locally maximal volume inside the k x k generator A[K, L]
// (leader workgroup only)
// ----------------------------------------------------------------------------
//
// The block A[K, L] is gathered once into the problem's work buffer (strip
// precision, row-major k x k) and becomes a dense source of its own; dual C-A
// sweeps at rank r run on it from J0 = its first r columns, with the same
// maxvol steps as the sweeps on A (a team of one workgroup), until a sweep
// after the first changes nothing or inner_sweeps sweeps are done.  The local
// indices are then mapped back through K and L.  Entries read from A: the
// k^2 of the block (the inner steps read the block only).
template <typename T, int KMAX>
NOINL void reduce_leader(const TaskDesc& td, Team& tio, int lds_b_bytes)
{
    Team one = tio;
    one.size = 1;
    one.rank = 0;
    Smem<T, KMAX>& sm = smem_ref<T, KMAX>();
    const int p = sm.k;
    const int r = td.cur_rank;
    const int inner = td.inner_sweeps;
    const int64_t er0 = sm.entries_read;
    // descriptor fields read before any store (a store could alias them)
    TaskDesc sub = td;
    T* blk = (T*)td.work;
    int64_t* KL = (int64_t*)(blk + ((int64_t)p * p + 1) / 2 * 2);
    T* sstrip = (T*)(KL + 2 * KMAX);
    if (threadIdx.x < p) {
        gl(KL)[threadIdx.x] = sm.I[threadIdx.x];
        gl(KL)[KMAX + threadIdx.x] = sm.J[threadIdx.x];
    }
    load_entries<T, (KMAX * KMAX + NT - 1) / NT>(
        td.src, p * p, threadIdx.x, NT,
        [&](int e, int64_t& i, int64_t& j) {
            i = sm.I[e / p];
            j = sm.J[e % p];
        },
        [&](int e, T v) { gl(blk)[e] = v; });
    __threadfence_block();
    __syncthreads();
    sub.src.kind = 0;
    sub.src.dtype = sizeof(T) == 8 ? 1 : 0;
    sub.src.a = blk;
    sub.src.lda = p;
    sub.src.col_major = 0;
    sub.src.x = nullptr;
    sub.src.y = nullptr;
    sub.m = p;
    sub.n = p;
    sub.strip = sstrip;
    sub.work = nullptr;  // the block lives there: no inverse is saved for a later launch
    if (threadIdx.x == 0) {
        sm.k = r;
        sm.have_I = 0;
        sm.w_valid = 0;
    }
    if (threadIdx.x < r) sm.J[threadIdx.x] = threadIdx.x;
    __syncthreads();
    const bool lds = (int64_t)(p | 1) * r * (int64_t)sizeof(T) <= lds_b_bytes;
    for (int it = 0; it < inner; ++it) {
        const int k_before = sm.k, had = sm.have_I;
        if (threadIdx.x < k_before) {
            sm.prevI[threadIdx.x] = sm.I[threadIdx.x];
            sm.prevJ[threadIdx.x] = sm.J[threadIdx.x];
        }
        __syncthreads();
        if (lds) maxvol_step<T, KMAX, true>(sub, one, 0, lds_b_bytes);
        else maxvol_step<T, KMAX, false>(sub, one, 0, lds_b_bytes);
        if (sm.phase == PH_DONE) break;
        if (threadIdx.x == 0) sm.have_I = 1;
        __syncthreads();
        if (lds) maxvol_step<T, KMAX, true>(sub, one, 1, lds_b_bytes);
        else maxvol_step<T, KMAX, false>(sub, one, 1, lds_b_bytes);
        if (sm.phase == PH_DONE) break;
        if (had && sm.k == k_before) {
            if (threadIdx.x == 0) {
                int same = 1;
                for (int c = 0; c < sm.k; ++c)
                    if (sm.I[c] != sm.prevI[c] || sm.J[c] != sm.prevJ[c]) same = 0;
                sm.flag = same;
            }
            __syncthreads();
            const int same = sm.flag;
            __syncthreads();
            if (same) break;
        }
    }
    __syncthreads();
    if (sm.phase != PH_DONE) {
        const int kf = sm.k;
        if (threadIdx.x < kf) {
            const int64_t il = sm.I[threadIdx.x], jl = sm.J[threadIdx.x];
            sm.I[threadIdx.x] = gl(KL)[il];
            sm.J[threadIdx.x] = gl(KL)[KMAX + jl];
        }
        if (threadIdx.x == 0) {
            sm.entries_read = er0 + (int64_t)p * p;
            sm.have_I = 1;
            sm.w_valid = 0;
            sm.phase = PH_FINAL;
        }
    }
    __syncthreads();
    tio.tog = one.tog;
    tio.trace_n = one.trace_n;
}

// ----------------------------------------------------------------------------
// state transfer between the team's workgroups and across launches
// ----------------------------------------------------------------------------

template <typename T, int KMAX>
DI void load_state(const TaskDesc& td, Smem<T, KMAX>& sm)
{
    // all loads first, then the LDS writes: one memory round trip
    if (threadIdx.x == 0) {
        const GL TaskState* st = gl(td.st);
        const int32_t phase = __hip_atomic_load(&st->phase, __ATOMIC_RELAXED, AGENT);
        const int32_t k = __hip_atomic_load(&st->k, __ATOMIC_RELAXED, AGENT);
        const int32_t sweep_in_level = __hip_atomic_load(&st->sweep_in_level, __ATOMIC_RELAXED, AGENT);
        const int32_t status = __hip_atomic_load(&st->status, __ATOMIC_RELAXED, AGENT);
        const int32_t warn = __hip_atomic_load(&st->warn, __ATOMIC_RELAXED, AGENT);
        const int32_t have_I = __hip_atomic_load(&st->have_I, __ATOMIC_RELAXED, AGENT);
        const int32_t had_I_sweep = __hip_atomic_load(&st->had_I_sweep, __ATOMIC_RELAXED, AGENT);
        const int32_t k_sweep_start = __hip_atomic_load(&st->k_sweep_start, __ATOMIC_RELAXED, AGENT);
        const int32_t swaps_total = __hip_atomic_load(&st->swaps_total, __ATOMIC_RELAXED, AGENT);
        const int32_t sweeps_done = __hip_atomic_load(&st->sweeps_done, __ATOMIC_RELAXED, AGENT);
        const int32_t phases_run = __hip_atomic_load(&st->phases_run, __ATOMIC_RELAXED, AGENT);
        const int32_t w_valid = __hip_atomic_load(&st->w_valid, __ATOMIC_RELAXED, AGENT);
        const int64_t cand_next = __hip_atomic_load(&st->cand_next, __ATOMIC_RELAXED, AGENT);
        const int64_t entries_read = __hip_atomic_load(&st->entries_read, __ATOMIC_RELAXED, AGENT);
        const double est_rel = __hip_atomic_load(&st->est_rel, __ATOMIC_RELAXED, AGENT);
        const double est_abs = __hip_atomic_load(&st->est_abs, __ATOMIC_RELAXED, AGENT);
        const double mean = __hip_atomic_load(&st->mean, __ATOMIC_RELAXED, AGENT);
        const double var = __hip_atomic_load(&st->var, __ATOMIC_RELAXED, AGENT);
        const double cond1 = __hip_atomic_load(&st->cond1, __ATOMIC_RELAXED, AGENT);
        sm.phase = phase;
        sm.k = k;
        sm.sweep_in_level = sweep_in_level;
        sm.status = status;
        sm.warn = warn;
        sm.have_I = have_I;
        sm.had_I_sweep = had_I_sweep;
        sm.k_sweep_start = k_sweep_start;
        sm.swaps_total = swaps_total;
        sm.sweeps_done = sweeps_done;
        sm.phases_run = phases_run;
        sm.w_valid = w_valid;
        sm.cand_next = cand_next;
        sm.entries_read = entries_read;
        sm.est_rel = est_rel;
        sm.est_abs = est_abs;
        sm.mean = mean;
        sm.var = var;
        sm.cond1 = cond1;
    }
    const int kc = td.kmax > td.k0 ? td.kmax : td.k0;
    if (threadIdx.x < kc) {
        const int c = threadIdx.x;
        const int64_t vi = __hip_atomic_load(gl(td.I) + c, __ATOMIC_RELAXED, AGENT);
        const int64_t vj = __hip_atomic_load(gl(td.J) + c, __ATOMIC_RELAXED, AGENT);
        const int64_t pi = __hip_atomic_load(gl(td.prevI) + c, __ATOMIC_RELAXED, AGENT);
        const int64_t pj = __hip_atomic_load(gl(td.prevJ) + c, __ATOMIC_RELAXED, AGENT);
        sm.I[c] = vi;
        sm.J[c] = vj;
        sm.prevI[c] = pi;
        sm.prevJ[c] = pj;
    }
    __syncthreads();
}

// Written by wavefront 0 only (see the team synchronisation notes).
template <typename T, int KMAX>
DI void store_state(const TaskDesc& td, Smem<T, KMAX>& sm)
{
    // descriptor fields read before any store (a store could alias them)
    GL int64_t* const I = gl(td.I);
    GL int64_t* const J = gl(td.J);
    GL int64_t* const pI = gl(td.prevI);
    GL int64_t* const pJ = gl(td.prevJ);
    GL TaskState* const st = gl(td.st);
    const int kc = td.kmax > td.k0 ? td.kmax : td.k0;
    if (threadIdx.x < kc) {
        const int c = threadIdx.x;
        const int64_t vi = sm.I[c], vj = sm.J[c], pi = sm.prevI[c], pj = sm.prevJ[c];
        __hip_atomic_store(I + c, vi, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(J + c, vj, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(pI + c, pi, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(pJ + c, pj, __ATOMIC_RELAXED, AGENT);
    }
    if (threadIdx.x == 0) {
        TaskState v;
        v.phase = sm.phase;
        v.k = sm.k;
        v.sweep_in_level = sm.sweep_in_level;
        v.status = sm.status;
        v.warn = sm.warn;
        v.have_I = sm.have_I;
        v.had_I_sweep = sm.had_I_sweep;
        v.k_sweep_start = sm.k_sweep_start;
        v.swaps_total = sm.swaps_total;
        v.sweeps_done = sm.sweeps_done;
        v.cand_next = sm.cand_next;
        v.entries_read = sm.entries_read;
        v.est_rel = sm.est_rel;
        v.est_abs = sm.est_abs;
        v.mean = sm.mean;
        v.var = sm.var;
        v.cond1 = sm.cond1;
        v.phases_run = sm.phases_run;
        v.w_valid = sm.w_valid;
        __hip_atomic_store(&st->phase, v.phase, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->k, v.k, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->sweep_in_level, v.sweep_in_level, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->status, v.status, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->warn, v.warn, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->have_I, v.have_I, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->had_I_sweep, v.had_I_sweep, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->k_sweep_start, v.k_sweep_start, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->swaps_total, v.swaps_total, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->sweeps_done, v.sweeps_done, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->phases_run, v.phases_run, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->w_valid, v.w_valid, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->cand_next, v.cand_next, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->entries_read, v.entries_read, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->est_rel, v.est_rel, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->est_abs, v.est_abs, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->mean, v.mean, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->var, v.var, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&st->cond1, v.cond1, __ATOMIC_RELAXED, AGENT);
    }
}

// Run one problem for up to `budget` phases.
template <typename T, int KMAX>
DI void run_task(const TaskDesc& td, Team& tm, const EngineArgs& ea)
{
    Smem<T, KMAX>& sm = smem_ref<T, KMAX>();
    const int lds_b = ea.lds_b[variant_of<T, KMAX>()];
    load_state(td, sm);
    if (sm.w_valid) {
        // resumed between steps: the last step's inverse from the work buffer
        const GL T* wg = gl((const T*)td.work);
        T* Wr = (T*)sm.AUG + KMAX;
        const int k = sm.k;
        for (int e = threadIdx.x; e < k * k; e += NT) Wr[(e / k) * 2 * KMAX + e % k] = wg[e];
        __syncthreads();
    }
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
            maxvol_dispatch<T, KMAX>(td, tm, 0, lds_b);
            if (tm.failed) return;
            if (threadIdx.x == 0 && sm.phase != PH_DONE) {
                sm.have_I = 1;
                sm.phase = PH_ROW;
            }
            __syncthreads();
        } else if (ph == PH_ROW) {
            maxvol_dispatch<T, KMAX>(td, tm, 1, lds_b);
            if (tm.failed) return;
            if (threadIdx.x == 0 && sm.phase != PH_DONE) {
                sm.sweeps_done += 1;
                sm.sweep_in_level += 1;
                const int after = (td.cur_rank > 0 && td.cur_rank < sm.k) ? PH_REDUCE : PH_FINAL;
                int next = sm.sweep_in_level >= td.sweeps ? after : PH_COL;
                if (td.tol > 0.0 && sm.had_I_sweep && sm.k == sm.k_sweep_start) {
                    int same = 1;
                    for (int c = 0; c < sm.k; ++c)
                        if (sm.I[c] != sm.prevI[c] || sm.J[c] != sm.prevJ[c]) same = 0;
                    if (same) next = PH_FINAL;
                }
                sm.phase = next;
            }
            __syncthreads();
        } else if (ph == PH_REDUCE) {
            if (tm.rank == 0) reduce_leader<T, KMAX>(td, tm, lds_b);
            if (tm.size > 1) {
                // the leader's generator reaches the team through global memory
                if (tm.rank == 0) store_state(td, sm);
                team_barrier(tm);
                if (tm.failed) return;
                if (tm.rank != 0) load_state(td, sm);
            }
        } else {  // PH_FINAL
            trace_ev(tm, EV_FINAL_BEGIN, 0);
            if (threadIdx.x == 0) sm.jsweeps = 0;
            write_factors<T, KMAX>(td, sm, tm);
            if (tm.rank == 0) final_leader<T, KMAX>(td, tm, lds_b);
            trace_ev(tm, EV_FINAL_END, sm.jsweeps);
            if (tm.size > 1) {
                // the leader's decision reaches the team through global memory
                if (tm.rank == 0) store_state(td, sm);
                team_barrier(tm);
                if (tm.failed) return;
                if (tm.rank != 0) load_state(td, sm);
            }
        }
        if (threadIdx.x == 0) sm.phases_run += 1;
        __syncthreads();
        if (tm.rank == 0) store_state(td, sm);
        trace_ev(tm, EV_PHASE_END, sm.phase);
    }
}

// The persistent loop of a workgroup: its team pulls task indices from the
// team's queue (the leader fetches, the team sees the index through the
// control block) and runs each for up to phase_budget phases.  RUN(td, tm)
// runs one task.
template <typename RUN>
DI void engine_loop(const EngineArgs& ea, RUN run)
{
    const int team = gl(ea.wg_team)[blockIdx.x];
    const TeamInfo ti = ea.teams[team];
    Team tm;
    tm.ctl = ea.team_ctl + (int64_t)team * ea.team_ctl_stride;
    tm.size = ti.size;
    tm.rank = blockIdx.x - ti.first_wg;
    tm.epoch = 0;
    tm.xepoch = 0;
    tm.failed = false;
    tm.tog = 0;
    tm.err = ea.error_flag;
    tm.timeout = ea.timeout_ticks;
    tm.trace = team == 0 ? ea.trace : nullptr;
    tm.trace_cap = ea.trace_cap;
    tm.trace_n = 0;
    for (;;) {
        const int par = tm.epoch & 1;
        GL int32_t* fetch = (GL int32_t*)gl(tm.ctl + 64) + par;
        if (threadIdx.x == 0 && tm.rank == 0) {
            const int idx = (int)__hip_atomic_fetch_add(gl(ea.queue_head) + ti.queue, 1u, __ATOMIC_RELAXED, AGENT);
            *lds_fetch() = idx;
            if (tm.size > 1) __hip_atomic_store(fetch, idx, __ATOMIC_RELAXED, AGENT);
        }
        if (tm.size > 1) {
            team_barrier(tm);
            if (tm.failed) return;
            if (threadIdx.x == 0 && tm.rank != 0) *lds_fetch() = __hip_atomic_load(fetch, __ATOMIC_RELAXED, AGENT);
        }
        __syncthreads();
        const int idx = *lds_fetch();
        __syncthreads();
        if (idx >= gl(ea.queue_len)[ti.queue]) break;
        const int task = gl(ea.queue_items)[gl(ea.queue_off)[ti.queue] + idx];
        trace_ev(tm, EV_TASK_BEGIN, task);
        run(ea.tasks[task], tm);
        trace_ev(tm, EV_TASK_END, task);
        if (tm.failed) return;
    }
}

template <typename T, int KMAX>
__global__ __launch_bounds__(NT) void engine_kernel(EngineArgs ea)
{
    engine_loop(ea, [&](const TaskDesc& td, Team& tm) { run_task<T, KMAX>(td, tm, ea); });
}

// Every variant in one launch (problems of mixed precision and rank bucket,
// e.g. a serving tick): each task runs the variant it names.
__global__ __launch_bounds__(NT) void engine_kernel_all(EngineArgs ea)
{
    engine_loop(ea, [&](const TaskDesc& td, Team& tm) {
        switch (td.variant) {
        case 0: run_task<float, 8>(td, tm, ea); break;
        case 1: run_task<float, 16>(td, tm, ea); break;
        case 2: run_task<float, 32>(td, tm, ea); break;
        case 3: run_task<float, 64>(td, tm, ea); break;
        case 4: run_task<double, 8>(td, tm, ea); break;
        case 5: run_task<double, 16>(td, tm, ea); break;
        case 6: run_task<double, 32>(td, tm, ea); break;
        default: run_task<double, 64>(td, tm, ea); break;
        }
    });
}

// The CUR factors of given index sets (Section 6.5): C = A[:, J] (m x k,
// column-major) and R = A[I, :] (k x n, row-major), by the whole grid.
// Entry e of C is C[e] = A[e % m, J[e / m]] and entry e of R is
// R[e] = A[I[e / n], e % n], so consecutive threads write consecutive
// addresses; each thread keeps 8 entries' loads in flight.  A column of a
// row-major matrix has one entry per memory line: that gather is bound by
// line fetches, the row gather by its bytes.
template <typename T>
__global__ __launch_bounds__(256) void factors_kernel(DevSource src, int64_t m, int64_t n, int k,
                                                      const int64_t* I, const int64_t* J, T* C, T* R)
{
    const int tid = (int)(blockIdx.x * 256 + threadIdx.x), nth = (int)(gridDim.x * 256);
    const GL int64_t* Ig = gl(I);
    const GL int64_t* Jg = gl(J);
    if (C) {
        GL T* Cg = gl(C);
        load_entries<T, 8>(
            src, (int)(m * k), tid, nth,
            [&](int e, int64_t& i, int64_t& j) {
                i = e % m;
                j = Jg[e / m];
            },
            [&](int e, T v) { Cg[e] = v; });
    }
    if (R) {
        GL T* Rg = gl(R);
        load_entries<T, 8>(
            src, (int)(k * n), tid, nth,
            [&](int e, int64_t& i, int64_t& j) {
                i = Ig[e / n];
                j = e % n;
            },
            [&](int e, T v) { Rg[e] = v; });
    }
}

// Zero-fill used instead of hipMemsetAsync (safe to record in a graph).
__global__ void zero_kernel(uint32_t* p, int64_t n_words)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_words; i += (int64_t)gridDim.x * blockDim.x)
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
    auto sz = [](size_t s) { return LDS_HDR + ((s + 255) & ~(size_t)255); };
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

// kmax = 0 selects the all-variant kernel.
const void* engine_kernel_ptr(int prec64, int kmax)
{
    if (kmax == 0) return reinterpret_cast<const void*>(&engine_kernel_all);
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

hipError_t launch_engine(int prec64, int kmax, int grid, size_t smem, bool cooperative, const EngineArgs& ea,
                         hipStream_t stream)
{
    const void* fn = engine_kernel_ptr(prec64, kmax);
    EngineArgs a = ea;
    void* args[] = {&a};
    if (cooperative) return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(NT), args, (unsigned)smem, stream);
    return hipLaunchKernel(fn, dim3(grid), dim3(NT), args, smem, stream);
}

hipError_t launch_factors(const DevSource& src, int64_t m, int64_t n, int k, const int64_t* I, const int64_t* J,
                          int out64, void* C, void* R, hipStream_t stream)
{
    const int64_t most = m * k > k * n ? m * k : k * n;
    int64_t blocks = (most + 256 * 8 - 1) / (256 * 8);
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    if (out64)
        hipLaunchKernelGGL(factors_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, stream, src, m, n, k, I, J,
                           (double*)C, (double*)R);
    else
        hipLaunchKernelGGL(factors_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, stream, src, m, n, k, I, J,
                           (float*)C, (float*)R);
    return hipGetLastError();
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

// ----------------------------------------------------------------------------
// fixed workspace of the allocation-free entry point (lra_ca_cur_noalloc)
// ----------------------------------------------------------------------------
//
// Every device the library runs on holds one copy of this array until the
// process ends.  On the host its name is only a stand-in for the symbol, not a
// device address: host code never passes it to a kernel or a copy.  The device
// address of each device's copy is looked up once, with that device current,
// by noalloc_scratch_init (called from lra_create), and noalloc_scratch hands
// it out afterwards.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_dev[NOALLOC_MAX_DEVICES];
}  // namespace

hipError_t noalloc_scratch_init(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (scratch_dev[device]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    scratch_dev[device] = ptr;
    return hipSuccess;
}

void* noalloc_scratch(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(scratch_mu);
    return scratch_dev[device];
}

}  // namespace lra
