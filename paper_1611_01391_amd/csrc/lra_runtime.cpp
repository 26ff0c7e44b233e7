// lra_runtime.cpp -- host runtime of the C-A / CUR library: contexts,
// workspace, problem set-up, team planning, launches, batching and serving.
// Every step of the method itself runs in the engine kernels
// (lra_engine.hip); this file only marshals, plans and schedules.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/lra.h"
#include "lra_internal.h"

namespace lra {
size_t engine_smem_fixed(int prec64, int kmax);
const void* engine_kernel_ptr(int prec64, int kmax);
hipError_t launch_engine(int prec64, int kmax, int grid, size_t smem, bool cooperative,
                         const EngineArgs& ea, hipStream_t stream);
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t stream);
hipError_t launch_pack_factors(const void* base, const int64_t* off, int np, double* out_g, double* out_u,
                               hipStream_t stream);
hipError_t launch_factors(const DevSource& src, int64_t m, int64_t n, int k, const int64_t* I, const int64_t* J,
                          int out64, void* C, void* R, hipStream_t stream);
hipError_t noalloc_scratch_init(int device);
void* noalloc_scratch(int device);
size_t core_out_bytes();
hipError_t topsvd_set_attributes();
hipError_t launch_tsqr(const void* xa, int64_t rows_a, int64_t lda, int dta, int nblk_a, double* out_a,
                       const void* xb, int64_t rows_b, int64_t ldb, int dtb, int nblk_b, double* out_b, int k,
                       hipStream_t stream);
hipError_t launch_topsvd_core(const double* RC, const double* RR, const double* W, int k, int r, double rank_lim,
                              void* out, hipStream_t stream);
hipError_t launch_topsvd_apply(const void* C, int64_t ldc, const void* R, int64_t ldr, int dtype, int64_t m,
                               int64_t n, int r, const void* core, double* S, int64_t lds, double* Tt, int64_t ldt,
                               hipStream_t stream);
void topsvd_core_fields(const void* host_copy, int32_t* status, int32_t* sweeps, const int32_t** pc,
                        const int32_t** pr, const double** sigma, const int64_t** ticks);
}  // namespace lra

using namespace lra;

namespace {

int log_level()
{
    static int lvl = [] {
        const char* e = std::getenv("LRA_LOG");
        return e ? std::atoi(e) : 0;
    }();
    return lvl;
}

#define LRA_LOG(lvl, ...)                                   \
    do {                                                     \
        if (log_level() >= (lvl)) {                          \
            std::fprintf(stderr, "[lra] " __VA_ARGS__);      \
            std::fputc('\n', stderr);                        \
        }                                                    \
    } while (0)

double now_us()
{
    using namespace std::chrono;
    return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() * 1e-3;
}

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): value number ctr of stream seed.
uint64_t splitmix64(uint64_t seed, uint64_t ctr)
{
    uint64_t z = seed + (ctr + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// cnt distinct indices in [0, n) in draw order (floor(v n / 2^64), repeats
// skipped); an open-addressing set keeps the repeat test O(1).
void draw_distinct(uint64_t seed, int64_t n, int64_t cnt, int64_t* out)
{
    size_t cap = 16;
    while (cap < 2 * (size_t)cnt) cap <<= 1;
    std::vector<int64_t> set(cap, -1);
    int64_t got = 0;
    for (uint64_t ctr = 0; got < cnt; ++ctr) {
        const uint64_t v = splitmix64(seed, ctr);
        const int64_t idx = (int64_t)(((unsigned __int128)v * (unsigned __int128)(uint64_t)n) >> 64);
        size_t h = (size_t)(((uint64_t)idx * 0x9E3779B97F4A7C15ull) >> 20) & (cap - 1);
        bool dup = false;
        while (set[h] >= 0) {
            if (set[h] == idx) { dup = true; break; }
            h = (h + 1) & (cap - 1);
        }
        if (!dup) {
            set[h] = idx;
            out[got++] = idx;
        }
    }
}

int kmax_bucket(int kcap) { return kcap <= 8 ? 8 : kcap <= 16 ? 16 : kcap <= 32 ? 32 : 64; }

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Region layout of one upload/download image.
struct Layout {
    int64_t size = 0;
    int64_t add(int64_t bytes, int64_t align = 256)
    {
        int64_t off = align_up(size, align);
        size = off + bytes;
        return off;
    }
};

}  // namespace

// ----------------------------------------------------------------------------
// context
// ----------------------------------------------------------------------------

struct Buffer {
    void* p = nullptr;
    int64_t bytes = 0;
};

struct Serve;

struct lra_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    size_t budget = 0;       // 0 = unbounded
    int num_cu = 0;
    int max_lds = 0;         // bytes per workgroup
    int64_t wall_rate_khz = 100000;
    double timeout_s = 30.0;
    int lds_b_bytes = 0;     // cap on the LDS for strip rows per workgroup (0: none)
    int lds_cap = 0;         // dynamic LDS per workgroup the kernels may use
    Buffer dev;              // workspace for blocking calls
    Buffer host;             // pinned staging for blocking calls
    int64_t dev_in_use = 0;  // device bytes held: blocking workspace, serving arena and control
    int64_t dev_allocs = 0;  // device allocations made since creation
    std::map<std::string, int> tuned;  // autotuned team sizes by size class
    int64_t floor_rows = -1;           // autotuned planning floor (-1: default)
    bool timing = false;
    int trace = 0;  // LRA_TRACE: 1 summary, 2 also every event
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    lra_stats stats{};
    Serve* srv = nullptr;    // serving scheduler, created by the first serving call
};

static lra_status hip_fail(hipError_t e, const char* what)
{
    LRA_LOG(1, "%s: %s", what, hipGetErrorString(e));
    return LRA_EDEVICE;
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

// Grow a buffer to at least `bytes` (25% headroom, whole MiB).  Device
// buffers count against the context's budget: what the other device buffers
// hold plus the new size must fit, the headroom is clamped to what is left,
// and the replaced buffer is freed first.  Steady-state calls (no larger
// than an earlier one) allocate nothing.
static lra_status ensure(Buffer& b, int64_t bytes, bool pinned, lra_ctx* ctx)
{
    if (b.bytes >= bytes) return LRA_OK;
    int64_t want = std::max<int64_t>(bytes, 1 << 20);
    want = align_up(want + want / 4, 1 << 20);
    if (!pinned && ctx->budget) {
        const int64_t room = (int64_t)ctx->budget - (ctx->dev_in_use - b.bytes);
        if (bytes > room) return LRA_EBUDGET;
        want = std::min(want, room);
    }
    if (b.p) {
        if (pinned) {
            (void)hipHostFree(b.p);
        } else {
            (void)hipFree(b.p);
            ctx->dev_in_use -= b.bytes;
        }
        b.p = nullptr;
        b.bytes = 0;
    }
    hipError_t e = pinned ? hipHostMalloc(&b.p, (size_t)want, hipHostMallocDefault) : hipMalloc(&b.p, (size_t)want);
    if (e != hipSuccess) {
        b.p = nullptr;
        LRA_LOG(1, "allocation of %lld bytes failed: %s", (long long)want, hipGetErrorString(e));
        return LRA_ENOMEM;
    }
    b.bytes = want;
    if (!pinned) {
        ctx->dev_in_use += want;
        ctx->dev_allocs += 1;
    }
    return LRA_OK;
}

extern "C" void lra_default_options(lra_options* o)
{
    std::memset(o, 0, sizeof(*o));
    o->tau = 0.01;
    o->k_max = 0;
    o->k_step = 8;
    o->max_swaps = 0;
    o->warm_start = 1;
    o->precision = LRA_PREC_FP64;
    o->sample_q = 64;
    o->sample_s = 64;
    o->team_wgs = 0;
    o->seed = 0;
    o->cur_rank = 0;
    o->inner_sweeps = 4;
    o->nucleus_rank = 0;
    o->init_rows = nullptr;
}

extern "C" const char* lra_status_str(lra_status s)
{
    switch (s) {
    case LRA_OK: return "ok";
    case LRA_TOL_NOT_MET: return "tolerance not met at k_max";
    case LRA_MAXVOL_CAP: return "maxvol swap cap reached";
    case LRA_NUMERICAL_RANK: return "numerical rank below k";
    case LRA_PENDING: return "pending";
    case LRA_EINVAL: return "invalid argument";
    case LRA_ERANK: return "exactly singular strip or generator";
    case LRA_ENOMEM: return "out of device memory";
    case LRA_EBUDGET: return "exceeds the HBM budget";
    case LRA_EDEVICE: return "device error";
    case LRA_ENONFINITE: return "non-finite entry";
    case LRA_ESCRATCH: return "workspace exceeds the fixed scratch of the allocation-free entry point";
    }
    return "unknown status";
}

extern "C" const char* lra_version(void) { return "lra-gfx950 1.0"; }

extern "C" lra_status lra_create(lra_ctx** out, void* stream, size_t budget)
{
    if (!out) return LRA_EINVAL;
    *out = nullptr;
    auto* c = new lra_ctx();
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) { delete c; return hip_fail(e, "hipGetDevice"); }
    c->stream = (hipStream_t)stream;
    c->budget = budget;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, c->device);
    if (e != hipSuccess) { delete c; return hip_fail(e, "hipGetDeviceProperties"); }
    c->num_cu = prop.multiProcessorCount;
    c->max_lds = (int)prop.sharedMemPerBlock;
    int rate = 0;
    if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, c->device) == hipSuccess && rate > 0)
        c->wall_rate_khz = rate;
    if (const char* t = std::getenv("LRA_TIMEOUT_S")) c->timeout_s = std::atof(t);
    if (const char* t = std::getenv("LRA_TRACE")) c->trace = std::atoi(t);
    // LDS for strip rows: all the device leaves per workgroup after the fixed
    // part of each kernel variant (LRA_LDS_B_BYTES caps it)
    int static_lds = 0;
    for (int p = 0; p < 2; ++p)
        for (int km : {0, 8, 16, 32, 64}) {
            hipFuncAttributes fa;
            e = hipFuncGetAttributes(&fa, engine_kernel_ptr(p, km));
            if (e != hipSuccess) { delete c; return hip_fail(e, "hipFuncGetAttributes"); }
            static_lds = std::max(static_lds, (int)fa.sharedSizeBytes);
        }
    c->lds_cap = (std::min(c->max_lds, 160 * 1024) - static_lds) & ~255;
    if (const char* t = std::getenv("LRA_LDS_B_BYTES")) c->lds_b_bytes = std::atoi(t);
    for (int p = 0; p < 2; ++p)
        for (int km : {0, 8, 16, 32, 64}) {
            e = hipFuncSetAttribute(engine_kernel_ptr(p, km), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    c->lds_cap);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                delete c;
                return hip_fail(e, "hipFuncSetAttribute");
            }
        }
    e = topsvd_set_attributes();
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return hip_fail(e, "hipFuncSetAttribute(top SVD)");
    }
    // device address of this device's copy of the allocation-free entry
    // point's scratch array (once per device)
    e = noalloc_scratch_init(c->device);
    if (e != hipSuccess) { delete c; return hip_fail(e, "hipGetSymbolAddress(scratch)"); }
    LRA_LOG(1, "device %d: %d CUs, %d B LDS/block, wall clock %lld kHz", c->device, c->num_cu, c->max_lds,
            (long long)c->wall_rate_khz);
    *out = c;
    return LRA_OK;
}

// ----------------------------------------------------------------------------
// problem set-up
// ----------------------------------------------------------------------------

static bool src_ok(const lra_source* s)
{
    if (!s) return false;
    if (s->dtype != LRA_F32 && s->dtype != LRA_F64) return false;
    if (s->kind == LRA_SRC_DENSE) return s->a != nullptr && s->lda > 0;
    if (s->kind == LRA_SRC_PREPROCESSED)
        return s->a != nullptr && s->lda > 0 && s->pre_depth >= 1 && s->pre_depth <= 8;
    if (s->kind == LRA_SRC_CAUCHY || s->kind == LRA_SRC_INVDIST) return s->x && s->y;
    return false;
}

// The device view of a source of m x n entries.
static DevSource dev_source(const lra_source* src, int64_t m, int64_t n)
{
    DevSource d;
    std::memset(&d, 0, sizeof(d));
    d.kind = src->kind;
    d.dtype = src->dtype;
    d.a = src->a;
    d.lda = src->lda;
    d.col_major = src->col_major ? 1 : 0;
    d.depth = src->kind == LRA_SRC_PREPROCESSED ? src->pre_depth : 0;
    d.x = src->x;
    d.y = src->y;
    d.seed = src->pre_seed;
    d.pm = m;
    d.pn = n;
    return d;
}

// A pre-processed source needs 2^d to divide both dimensions.
static bool shape_ok(const lra_source* src, int64_t m, int64_t n)
{
    if (src->kind != LRA_SRC_PREPROCESSED) return true;
    const int64_t b = (int64_t)1 << src->pre_depth;
    return m % b == 0 && n % b == 0;
}

// Host-side description of one problem before upload.
struct Prob {
    DevSource src;
    int64_t m, n;
    int k, kcap, kstep, sweeps, max_swaps, warm;
    double tol, tau;
    int q, s;
    std::vector<int64_t> cand, Q, S;
    int team = 1;
    int prec64 = 1, kmx = 8;  // kernel variant the problem runs with
    bool team_fixed = false;  // chosen by the caller: never resized
    bool need_strip = false;
    void* C_out = nullptr;
    void* R_out = nullptr;
    bool have_init_I = false;
    std::vector<int64_t> init_I;
    int cur_rank = 0, inner_sweeps = 4, nucleus_rank = 0;
    int bf16_select = 0;
};

static lra_status make_prob(const lra_source* src, int64_t m, int64_t n, int k, int sweeps, double tol,
                            const lra_options* o, Prob& p, int64_t blk_index)
{
    if (!src_ok(src) || m < 1 || n < 1 || k < 1 || k > 64 || k > m || k > n || sweeps < 0) return LRA_EINVAL;
    // the fixed-rank algorithms (random sets, Cynical step, truncated nucleus) take no tolerance
    if (o->cur_rank < 0 || o->cur_rank > k || o->nucleus_rank < 0 || o->nucleus_rank > k) return LRA_EINVAL;
    const bool fixed_alg = sweeps == 0 || (o->cur_rank > 0 && o->cur_rank < k) ||
                           (o->nucleus_rank > 0 && o->nucleus_rank < k);
    if (fixed_alg && tol > 0.0) return LRA_EINVAL;
    if (o->cur_rank > 0 && o->cur_rank < k && o->inner_sweeps < 1) return LRA_EINVAL;
    if (!(o->tau >= 0.0) || o->k_step < 1 || o->k_max > 64) return LRA_EINVAL;
    if ((src->kind == LRA_SRC_DENSE || src->kind == LRA_SRC_PREPROCESSED) && src->lda < (src->col_major ? m : n))
        return LRA_EINVAL;
    if (!shape_ok(src, m, n)) return LRA_EINVAL;
    if (o->precision != LRA_PREC_FP64 && o->precision != LRA_PREC_MIXED && o->precision != LRA_PREC_BF16SEL)
        return LRA_EINVAL;
    p.src = dev_source(src, m, n);
    p.m = m;
    p.n = n;
    p.k = k;
    p.kcap = std::max(k, (int)std::min<int64_t>(o->k_max, std::min(m, n)));
    p.kstep = o->k_step;
    p.sweeps = sweeps;
    p.max_swaps = o->max_swaps;
    p.warm = o->warm_start ? 1 : 0;
    p.tol = tol;
    p.tau = o->tau;
    p.q = (int)std::min<int64_t>(std::max(1, o->sample_q), m);
    p.s = (int)std::min<int64_t>(std::max(1, o->sample_s), n);
    if (p.q > 64 || p.s > 64) return LRA_EINVAL;
    const uint64_t seed = o->seed + (uint64_t)blk_index * 0x1000003ull;
    if (o->init_cols) {
        if (o->n_init_cols < k) return LRA_EINVAL;
        p.cand.assign(o->init_cols, o->init_cols + o->n_init_cols);
        for (int64_t v : p.cand)
            if (v < 0 || v >= n) return LRA_EINVAL;
        for (int a = 0; a < k; ++a)
            for (int b = a + 1; b < k; ++b)
                if (p.cand[a] == p.cand[b]) return LRA_EINVAL;
    } else {
        p.cand.resize((size_t)std::min<int64_t>(n, 2 * (int64_t)p.kcap));
        draw_distinct(seed, n, (int64_t)p.cand.size(), p.cand.data());
    }
    if (o->sample_rows) {
        p.Q.assign(o->sample_rows, o->sample_rows + p.q);
    } else {
        p.Q.resize(p.q);
        draw_distinct(seed + 1, m, p.q, p.Q.data());
        std::sort(p.Q.begin(), p.Q.end());
    }
    if (o->sample_cols) {
        p.S.assign(o->sample_cols, o->sample_cols + p.s);
    } else {
        p.S.resize(p.s);
        draw_distinct(seed + 2, n, p.s, p.S.data());
        std::sort(p.S.begin(), p.S.end());
    }
    for (int64_t v : p.Q)
        if (v < 0 || v >= m) return LRA_EINVAL;
    for (int64_t v : p.S)
        if (v < 0 || v >= n) return LRA_EINVAL;
    p.bf16_select = o->precision == LRA_PREC_BF16SEL ? 1 : 0;
    p.cur_rank = o->cur_rank < k ? o->cur_rank : 0;
    p.inner_sweeps = o->inner_sweeps;
    p.nucleus_rank = o->nucleus_rank < k ? o->nucleus_rank : 0;
    if (sweeps == 0) {
        // random rows of the generator: the caller's, or drawn from stream seed+3
        p.have_init_I = true;
        if (o->init_rows) {
            p.init_I.assign(o->init_rows, o->init_rows + k);
            for (int a = 0; a < k; ++a) {
                if (p.init_I[a] < 0 || p.init_I[a] >= m) return LRA_EINVAL;
                for (int b = a + 1; b < k; ++b)
                    if (p.init_I[a] == p.init_I[b]) return LRA_EINVAL;
            }
        } else {
            p.init_I.resize(k);
            draw_distinct(seed + 3, m, k, p.init_I.data());
        }
    }
    return LRA_OK;
}

// LDS left for strip rows in a workgroup of the (precision, KMAX) variant.
static int strip_lds(lra_ctx* ctx, int prec64, int kmx)
{
    int b = ctx->lds_cap - (int)engine_smem_fixed(prec64, kmx);
    b = std::max(0, b) & ~1023;
    if (ctx->lds_b_bytes > 0) b = std::min(b, ctx->lds_b_bytes);
    return b;
}

// Size class of a single problem for the tuned team sizes: precision, rank
// bucket and the bit length of its longer side.
static std::string team_key(const Prob& p, int prec64)
{
    const int64_t M = std::max(p.m, p.n);
    char key[96];
    std::snprintf(key, sizeof(key), "%d/%d/%lld", prec64, kmax_bucket(p.kcap),
                  (long long)(64 - __builtin_clzll((unsigned long long)M)));
    return key;
}

// Workgroups per problem: enough that each workgroup's rows fit its LDS,
// within the co-resident limit; an explicit or tuned choice overrides.
static int auto_team(lra_ctx* ctx, const Prob& p, int prec64, bool use_tuned = true)
{
    const int esz = prec64 ? 8 : 4;
    const int64_t M = std::max(p.m, p.n);
    if (use_tuned) {
        auto it = ctx->tuned.find(team_key(p, prec64));
        if (it != ctx->tuned.end()) return it->second;
    }
    int64_t rows_fit = strip_lds(ctx, prec64, kmax_bucket(p.kcap)) / ((int64_t)p.kcap * esz);
    // at most one row per thread keeps the swap loop register-resident
    rows_fit = std::max<int64_t>(64, std::min<int64_t>(rows_fit, NT));
    int64_t t = (M + rows_fit - 1) / rows_fit;
    t = std::min<int64_t>(t, std::min(ctx->num_cu, NT));
    return (int)std::max<int64_t>(1, t);
}

// ----------------------------------------------------------------------------
// device regions of a problem
// ----------------------------------------------------------------------------

// Byte offsets of one problem's device regions, relative to a base pointer.
struct ProbRegions {
    int64_t cand = -1, Q = -1, S = -1;                       // inputs
    int64_t st = -1, I = -1, J = -1;                         // resumable state
    int64_t G = -1, U = -1;                                  // results
    int64_t prevI = -1, prevJ = -1, work = -1, strip = -1;   // scratch (strip: -1 when unused)
};

// Final phase scratch: [G | I | A[I,S]] with row stride 2 KMAX + 64, and
// the q x k and q x s sample blocks.
static int64_t work_bytes(const Prob& p)
{
    const int64_t kb = kmax_bucket(p.kcap), kc = p.kcap;
    const int64_t fin = 8 * (kb * (2 * kb + 64) + (int64_t)p.q * kc + (int64_t)p.q * p.s);
    // Cynical step: the k x k block, K and L (2 KMAX), a k x r strip
    const int64_t red = 8 * (kc * kc + 2 + 2 * kb + kc * kc);
    return std::max(fin, red);
}

static int64_t strip_bytes(const Prob& p, int prec64)
{
    return std::max(p.m, p.n) * (int64_t)p.kcap * (prec64 ? 8 : 4);
}

static void fill_task(TaskDesc& td, const Prob& p, uint8_t* base, const ProbRegions& r)
{
    td.src = p.src;
    td.m = p.m;
    td.n = p.n;
    td.k0 = p.k;
    td.kmax = p.kcap;
    td.kstep = p.kstep;
    td.sweeps = p.sweeps;
    td.tol = p.tol;
    td.tau = p.tau;
    td.max_swaps = p.max_swaps;
    td.warm_start = p.warm;
    td.q = p.q;
    td.s = p.s;
    td.cand = (const int64_t*)(base + r.cand);
    td.n_cand = (int64_t)p.cand.size();
    td.Q = (const int64_t*)(base + r.Q);
    td.S = (const int64_t*)(base + r.S);
    td.I = (int64_t*)(base + r.I);
    td.J = (int64_t*)(base + r.J);
    td.prevI = (int64_t*)(base + r.prevI);
    td.prevJ = (int64_t*)(base + r.prevJ);
    td.G = (double*)(base + r.G);
    td.U = (double*)(base + r.U);
    td.work = (double*)(base + r.work);
    td.strip = r.strip >= 0 ? (void*)(base + r.strip) : nullptr;
    td.C_out = p.C_out;
    td.R_out = p.R_out;
    td.st = (TaskState*)(base + r.st);
    td.variant = variant_index(p.prec64, p.kmx);
    td.cur_rank = p.cur_rank;
    td.inner_sweeps = p.inner_sweeps;
    td.nucleus_rank = p.nucleus_rank;
    td.bf16_select = p.bf16_select;
    td.pad_t = 0;
}

// Host image of the inputs (cand, Q, S) and of the initial state (st, I, J).
static void init_inputs(uint8_t* h, const Prob& p, const ProbRegions& r)
{
    std::memcpy(h + r.cand, p.cand.data(), 8 * p.cand.size());
    std::memcpy(h + r.Q, p.Q.data(), 8 * (size_t)p.q);
    std::memcpy(h + r.S, p.S.data(), 8 * (size_t)p.s);
}

static void init_state(uint8_t* h_st, uint8_t* h_I, uint8_t* h_J, const Prob& p)
{
    int64_t* I = (int64_t*)h_I;
    int64_t* J = (int64_t*)h_J;
    for (int c = 0; c < p.kcap; ++c) {
        I[c] = (p.have_init_I && c < p.k) ? p.init_I[c] : 0;
        J[c] = c < p.k ? p.cand[c] : 0;
    }
    TaskState* st = (TaskState*)h_st;
    std::memset(st, 0, sizeof(*st));
    // no C-A sweeps: straight to the Cynical step or the nucleus
    st->phase = p.sweeps > 0 ? PH_COL : (p.cur_rank > 0 ? PH_REDUCE : PH_FINAL);
    st->k = p.k;
    st->have_I = p.have_init_I ? 1 : 0;
    st->cand_next = p.k;
}

// ----------------------------------------------------------------------------
// team planning
// ----------------------------------------------------------------------------

struct Plan {
    std::vector<TeamInfo> teams;
    std::vector<int32_t> wg_team;
    std::vector<std::vector<int32_t>> queues;
    int max_team = 1;
};

// Work of a problem for planning: a C-A step costs about (rows) k^2 (the
// first step's LU, the basis product, and about k swaps of rows x k updates),
// over 2 sweeps' worth of steps.
static double prob_cost(const Prob& p)
{
    return (double)(p.m + p.n) * (double)p.kcap * (double)p.kcap * (double)p.sweeps;
}

// A problem sharing a launch keeps at least ceil(rows / floor) workgroups
// (at most 32): with one or two workgroups a long strip's first-step LU and
// swap updates run from global memory on a single CU and become the launch's
// critical path.  8192 rows measured best overall on the served stream and
// the far-field blocks; LRA_SHARE_FLOOR_ROWS overrides it (0: no floor).
static int64_t share_floor_rows()
{
    static int64_t v = [] {
        const char* e = std::getenv("LRA_SHARE_FLOOR_ROWS");
        return e ? (int64_t)std::atoll(e) : (int64_t)8192;
    }();
    return v;
}

static int pow2_ceil(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Teams by size class.  Every class first gets one team (the caller makes
// the class sizes fit the grid); the remaining workgroups go to the classes
// in proportion to their work, then greedily to the class with the most work
// per team.  Problems of a class are pulled largest first.
static Plan plan_teams(const std::vector<Prob*>& probs, int max_wgs)
{
    Plan pl;
    std::map<int, std::vector<int32_t>> cls;
    for (int i = 0; i < (int)probs.size(); ++i) cls[probs[i]->team].push_back(i);
    auto cost_of = [&](int i) { return prob_cost(*probs[i]); };
    std::vector<int> size, nteam, nitems;
    std::vector<double> cost;
    int reserved = 0;
    double total = 0.0;
    for (auto& kv : cls) {
        double c = 0.0;
        for (int i : kv.second) c += cost_of(i);
        size.push_back(kv.first);
        nitems.push_back((int)kv.second.size());
        cost.push_back(c);
        nteam.push_back(1);
        reserved += kv.first;
        total += c;
    }
    const int nc = (int)size.size();
    int avail = std::max(0, max_wgs - reserved);
    for (int c = 0; c < nc; ++c) {
        int extra = (int)std::floor((double)avail * cost[c] / std::max(total, 1.0) / size[c]);
        extra = std::max(0, std::min(extra, nitems[c] - 1));
        nteam[c] += extra;
    }
    int used = 0;
    for (int c = 0; c < nc; ++c) used += nteam[c] * size[c];
    for (;;) {
        int best = -1;
        for (int c = 0; c < nc; ++c)
            if (nteam[c] < nitems[c] && used + size[c] <= max_wgs &&
                (best < 0 || cost[c] / nteam[c] > cost[best] / nteam[best]))
                best = c;
        if (best < 0) break;
        nteam[best] += 1;
        used += size[best];
    }
    int c = 0, wg = 0;
    for (auto& kv : cls) {
        auto items = kv.second;
        std::stable_sort(items.begin(), items.end(), [&](int a, int b) { return cost_of(a) > cost_of(b); });
        for (int t = 0; t < nteam[c]; ++t) {
            TeamInfo ti;
            ti.first_wg = wg;
            ti.size = size[c];
            ti.queue = c;
            ti.pad = 0;
            pl.teams.push_back(ti);
            for (int w = 0; w < size[c]; ++w) pl.wg_team.push_back((int32_t)pl.teams.size() - 1);
            wg += size[c];
        }
        pl.queues.push_back(items);
        pl.max_team = std::max(pl.max_team, size[c]);
        ++c;
    }
    return pl;
}

struct LaunchPlan {
    int prec64 = 1;
    int kmx = 8;          // 0: the all-variant kernel
    int lds_b[NVARIANT] = {0};
    int max_wgs = 0;
    int grid = 0;
    size_t smem = 0;
    bool coop = false;
    Plan pl;
};

static int pow2_floor(int v)
{
    int p = 1;
    while (2 * p <= v) p <<= 1;
    return p;
}

// Throughput sizing for problems sharing a launch: each team gets about its
// problem's share of the grid's workgroups (a power of two, at least one),
// never more than the latency-optimal size the problem came with, so that
// large and small problems finish together.
static void share_teams(std::vector<Prob*>& probs, int max_wgs, int64_t floor_rows)
{
    if (probs.size() < 2) return;
    double tot = 0.0;
    for (Prob* p : probs) tot += prob_cost(*p);
    for (Prob* p : probs) {
        if (p->team_fixed) continue;
        const double share = (double)max_wgs * prob_cost(*p) / std::max(tot, 1.0);
        int t = pow2_floor((int)std::max(1.0, std::min(share, (double)max_wgs)));
        if (floor_rows > 0) {
            const int64_t rows = std::max(p->m, p->n);
            const int64_t f = std::min<int64_t>(std::min(32, max_wgs), (rows + floor_rows - 1) / floor_rows);
            t = std::max(t, pow2_floor((int)std::max<int64_t>(1, f)));
        }
        p->team = std::max(1, std::min(p->team, t));
    }
}

// Fit the problems' teams to the co-resident grid of the (precision, KMAX)
// kernel -- or of the all-variant kernel when kmx = 0, each problem then
// running its own variant -- and plan the queues.  With fixed_strip the
// problems already own a global strip region (serving), so any team size is
// safe; otherwise each problem's need for one is decided here.
static lra_status plan_launch(lra_ctx* ctx, std::vector<Prob*>& probs, int prec64, int kmx, bool fixed_strip,
                              LaunchPlan& lp)
{
    lp.prec64 = prec64;
    lp.kmx = kmx;
    for (int p64 = 0; p64 < 2; ++p64)
        for (int km : {8, 16, 32, 64}) lp.lds_b[variant_index(p64, km)] = strip_lds(ctx, p64, km);
    lp.smem = kmx == 0 ? (size_t)ctx->lds_cap
                       : engine_smem_fixed(prec64, kmx) + (size_t)lp.lds_b[variant_index(prec64, kmx)];
    int occ = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, engine_kernel_ptr(prec64, kmx), NT, lp.smem));
    if (occ < 1) return LRA_EDEVICE;
    lp.max_wgs = occ * ctx->num_cu;
    for (Prob* p : probs) p->team = std::max(1, std::min(p->team, lp.max_wgs));
    share_teams(probs, lp.max_wgs, ctx->floor_rows >= 0 ? ctx->floor_rows : share_floor_rows());
    // every size class holds at least one team: halve the largest sizes until
    // the classes take at most half the grid together (the rest is shared out
    // by work)
    for (;;) {
        std::vector<int> sizes;
        for (Prob* p : probs) sizes.push_back(p->team);
        std::sort(sizes.begin(), sizes.end());
        sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
        int64_t sum = 0;
        for (int s : sizes) sum += s;
        if (sum <= std::max(1, lp.max_wgs / 2) || sizes.size() == 1) break;
        const int big = sizes.back();
        for (Prob* p : probs)
            if (p->team == big) p->team = std::max(1, big / 2);
    }
    for (Prob* p : probs) {
        if (fixed_strip) continue;
        const int64_t R = (std::max(p->m, p->n) + p->team - 1) / p->team;
        // the engine's LDS slice has leading dimension R | 1
        p->need_strip = (R | 1) * p->kcap * (p->prec64 ? 8 : 4) > lp.lds_b[variant_index(p->prec64, p->kmx)];
    }
    lp.pl = plan_teams(probs, lp.max_wgs);
    lp.grid = (int)lp.pl.wg_team.size();
    lp.coop = lp.pl.max_team > 1;
    return LRA_OK;
}

// Summarise a device trace on stderr: time spent before each event kind,
// measured from the previous event of the same team leader.
static void dump_trace(lra_ctx* ctx, const uint64_t* tr, int cap)
{
    static const char* names[] = {"?", "step_begin", "warm_lu", "gathered", "basis", "swap_g",
                                  "step_end", "final_begin", "final_end", "task_begin", "task_end",
                                  "pivot", "swap_upd+red", "swap_xchg", "phase_end", "dispatch"};
    const uint64_t n = std::min<uint64_t>(tr[0], (uint64_t)cap);
    double tot[16] = {0};
    int64_t cnt[16] = {0};
    const double us_per_tick = 1000.0 / (double)ctx->wall_rate_khz;
    for (uint64_t i = 1; i < n; ++i) {
        const int ev = (int)(tr[1 + 2 * i] >> 56);
        const double dt = (double)(tr[2 + 2 * i] - tr[2 + 2 * (i - 1)]) * us_per_tick;
        if (ev > 0 && ev < 16) { tot[ev] += dt; cnt[ev] += 1; }
        if (ctx->trace >= 2 && ev > 0 && ev < 16)
            std::fprintf(stderr, "[lra trace] %5llu %-12s arg %6lld  +%8.2f us\n", (unsigned long long)i, names[ev],
                         (long long)(tr[1 + 2 * i] & 0x00FFFFFFFFFFFFFFull), dt);
    }
    std::fprintf(stderr, "[lra trace] %llu events\n", (unsigned long long)n);
    for (int e = 1; e < 16; ++e)
        if (cnt[e])
            std::fprintf(stderr, "[lra trace] %-12s n=%6lld total %9.1f us  mean %7.2f us\n", names[e],
                         (long long)cnt[e], tot[e], tot[e] / (double)cnt[e]);
}

// ----------------------------------------------------------------------------
// control image of one launch
// ----------------------------------------------------------------------------

struct CtlImage {
    int64_t tasks = 0, items = 0, qoff = 0, qlen = 0, teams = 0, wgteam = 0;  // uploaded
    int64_t ctl = 0, qhead = 0;                                             // zero-filled
    int64_t ctl_stride = 0;
    int nq = 0;
};

static void lay_ctl_upload(Layout& L, CtlImage& c, size_t ntasks, const Plan& pl)
{
    int64_t nitems = 0;
    for (auto& q : pl.queues) nitems += (int64_t)q.size();
    c.nq = (int)pl.queues.size();
    c.tasks = L.add(sizeof(TaskDesc) * ntasks);
    c.items = L.add(4 * std::max<int64_t>(1, nitems));
    c.qoff = L.add(4 * c.nq);
    c.qlen = L.add(4 * c.nq);
    c.teams = L.add(sizeof(TeamInfo) * pl.teams.size());
    c.wgteam = L.add(4 * (int64_t)pl.wg_team.size());
}

static void lay_ctl_zero(Layout& L, CtlImage& c, const Plan& pl)
{
    c.ctl_stride = align_up(team_ctl_bytes(pl.max_team), 256);
    c.ctl = L.add(c.ctl_stride * (int64_t)pl.teams.size());
    c.qhead = L.add(4 * (int64_t)c.nq);
}

static void write_ctl(uint8_t* h, const CtlImage& c, const Plan& pl)
{
    int32_t* items = (int32_t*)(h + c.items);
    int32_t* qoff = (int32_t*)(h + c.qoff);
    int32_t* qlen = (int32_t*)(h + c.qlen);
    int64_t pos = 0;
    for (int q = 0; q < c.nq; ++q) {
        qoff[q] = (int32_t)pos;
        qlen[q] = (int32_t)pl.queues[q].size();
        for (int32_t t : pl.queues[q]) items[pos++] = t;
    }
    std::memcpy(h + c.teams, pl.teams.data(), sizeof(TeamInfo) * pl.teams.size());
    std::memcpy(h + c.wgteam, pl.wg_team.data(), 4 * pl.wg_team.size());
}

static EngineArgs engine_args(lra_ctx* ctx, uint8_t* d, const CtlImage& c, const LaunchPlan& lp, int phase_budget,
                              uint32_t* err, uint64_t* trace, int trace_cap)
{
    EngineArgs ea;
    ea.tasks = (TaskDesc*)(d + c.tasks);
    ea.queue_items = (const int32_t*)(d + c.items);
    ea.queue_off = (const int32_t*)(d + c.qoff);
    ea.queue_len = (const int32_t*)(d + c.qlen);
    ea.queue_head = (uint32_t*)(d + c.qhead);
    ea.teams = (const TeamInfo*)(d + c.teams);
    ea.wg_team = (const int32_t*)(d + c.wgteam);
    ea.team_ctl = d + c.ctl;
    ea.team_ctl_stride = c.ctl_stride;
    ea.phase_budget = phase_budget;
    for (int v = 0; v < NVARIANT; ++v) ea.lds_b[v] = lp.lds_b[v];
    ea.error_flag = err;
    ea.timeout_ticks = (int64_t)(ctx->timeout_s * (double)ctx->wall_rate_khz * 1000.0);
    ea.trace = trace;
    ea.trace_cap = trace_cap;
    return ea;
}

static lra_status launch(lra_ctx* ctx, const LaunchPlan& lp, const EngineArgs& ea, hipStream_t stream)
{
    const int prec64 = lp.prec64;
    LRA_LOG(2, "launch: grid %d, teams %zu (max %d), smem %zu, coop %d", lp.grid, lp.pl.teams.size(),
            lp.pl.max_team, lp.smem, (int)lp.coop);
    HIP_TRY(launch_engine(prec64, lp.kmx, lp.grid, lp.smem, lp.coop, ea, stream));
    ctx->stats.launches += 1;
    ctx->stats.last_grid = lp.grid;
    ctx->stats.last_teams = (int32_t)lp.pl.teams.size();
    return LRA_OK;
}

// ----------------------------------------------------------------------------
// results
// ----------------------------------------------------------------------------

static lra_status status_of(const TaskState& st)
{
    if (st.status < 0) return (lra_status)st.status;
    if (st.warn & W_TOL) return LRA_TOL_NOT_MET;
    if (st.warn & W_NUMRANK) return LRA_NUMERICAL_RANK;
    if (st.warn & W_CAP) return LRA_MAXVOL_CAP;
    return LRA_OK;
}

static void deliver(const TaskState& st, const int64_t* I, const int64_t* J, const double* G, const double* U,
                    lra_result* res)
{
    const int k = st.k;
    res->k = k;
    res->status = (int32_t)status_of(st);
    res->sweeps_done = st.sweeps_done;
    res->swaps_total = st.swaps_total;
    res->entries_read = st.entries_read;
    res->err_est_rel = st.est_rel;
    res->err_est_abs = st.est_abs;
    res->err_mean = st.mean;
    res->err_var = st.var;
    res->nucleus_cond1 = st.cond1;
    if (res->I && I) std::memcpy(res->I, I, 8 * (size_t)k);
    if (res->J && J) std::memcpy(res->J, J, 8 * (size_t)k);
    if (res->G && G) std::memcpy(res->G, G, 8 * (size_t)k * k);
    if (res->U && U) std::memcpy(res->U, U, 8 * (size_t)k * k);
}

static int severity(lra_status s)
{
    if (s < 0) return 100 - (int)s;
    return (int)s;
}

// ----------------------------------------------------------------------------
// blocking runs: a set of problems of one precision in one launch
// ----------------------------------------------------------------------------

// Image layout (one workspace buffer):
//   upload    : control | inputs (cand, Q, S) | states | I | J | error word
//   read back : states | I | J | error word, then G | U when asked for
//   zeroed    : team control blocks, queue heads, trace
//   scratch   : prevI, prevJ, final-phase work, global strips
// Caller-provided buffers of a run (the allocation-free entry point): the
// device workspace and the host staging, with their capacities.
struct FixedBuffers {
    uint8_t* dev;
    int64_t dev_bytes;
    uint8_t* host;
    int64_t host_bytes;
};

static lra_status run_batch(lra_ctx* ctx, std::vector<Prob>& probs, int prec64, int phase_budget,
                            lra_result* const* res, const FixedBuffers* fixed = nullptr)
{
    const size_t np = probs.size();
    if (np == 0) return LRA_OK;
    int kcap_all = 1;
    for (auto& p : probs) kcap_all = std::max(kcap_all, p.kcap);
    std::vector<Prob*> pp;
    for (auto& p : probs) {
        p.prec64 = prec64;
        p.kmx = kmax_bucket(kcap_all);
        pp.push_back(&p);
    }
    const double t_plan0 = now_us();
    LaunchPlan lp;
    lra_status rs = plan_launch(ctx, pp, prec64, kmax_bucket(kcap_all), false, lp);
    if (rs != LRA_OK) return rs;
    const double t_plan1 = now_us();
    bool want_G = false, want_U = false;
    for (size_t i = 0; i < np; ++i) {
        want_G = want_G || res[i]->G;
        want_U = want_U || res[i]->U;
    }

    Layout L;
    CtlImage c;
    lay_ctl_upload(L, c, np, lp.pl);
    std::vector<ProbRegions> regs(np);
    for (size_t i = 0; i < np; ++i) {
        regs[i].cand = L.add(8 * (int64_t)probs[i].cand.size(), 8);
        regs[i].Q = L.add(8 * (int64_t)probs[i].q, 8);
        regs[i].S = L.add(8 * (int64_t)probs[i].s, 8);
    }
    // many problems with G or U wanted: their k x k factors are packed on the
    // device and only sum k^2 entries read back (not the kcap^2 regions)
    int64_t kk_all = 0;
    for (size_t i = 0; i < np; ++i) kk_all += (int64_t)probs[i].kcap * probs[i].kcap;
    bool pack = !fixed && (want_G || want_U) && np >= 32;
    const int64_t off_pack = pack ? L.add(24 * (int64_t)np, 8) : -1;
    const int64_t rb0 = L.add(0);
    for (size_t i = 0; i < np; ++i) regs[i].st = L.add(sizeof(TaskState), 8);
    for (size_t i = 0; i < np; ++i) regs[i].I = L.add(8 * (int64_t)probs[i].kcap, 8);
    for (size_t i = 0; i < np; ++i) regs[i].J = L.add(8 * (int64_t)probs[i].kcap, 8);
    const int64_t off_err = L.add(8, 8);
    const int64_t up_end = L.size;
    for (size_t i = 0; i < np; ++i) regs[i].G = L.add(8 * (int64_t)probs[i].kcap * probs[i].kcap, 8);
    const int64_t u0 = L.add(0, 8);
    for (size_t i = 0; i < np; ++i) regs[i].U = L.add(8 * (int64_t)probs[i].kcap * probs[i].kcap, 8);
    const int64_t u1 = L.size;
    const int64_t z0 = L.add(0);
    lay_ctl_zero(L, c, lp.pl);
    const int trace_cap = ctx->trace ? 1 << 16 : 0;
    const int64_t off_trace = L.add(8 * (1 + 2 * (int64_t)trace_cap));
    const int64_t z1 = L.size;
    for (size_t i = 0; i < np; ++i) {
        regs[i].prevI = L.add(8 * (int64_t)probs[i].kcap);
        regs[i].prevJ = L.add(8 * (int64_t)probs[i].kcap);
        regs[i].work = L.add(work_bytes(probs[i]));
        regs[i].strip = probs[i].need_strip ? L.add(strip_bytes(probs[i], prec64)) : -1;
    }
    int64_t packed = -1;
    if (pack) {
        const int64_t room = ctx->budget ? (int64_t)ctx->budget - (ctx->dev_in_use - ctx->dev.bytes) : INT64_MAX;
        if (L.size + 16 * kk_all + 256 <= room) packed = L.add(16 * kk_all, 256);
        else pack = false;
    }
    const int64_t total = L.size;

    uint8_t* h = nullptr;
    uint8_t* d = nullptr;
    if (fixed) {
        if (total > fixed->dev_bytes || u1 > fixed->host_bytes) {
            LRA_LOG(1, "workspace of %lld device bytes (%lld staged) exceeds the fixed scratch of %lld (%lld)",
                    (long long)total, (long long)u1, (long long)fixed->dev_bytes, (long long)fixed->host_bytes);
            return LRA_ESCRATCH;
        }
        d = fixed->dev;
        h = fixed->host;
    } else {
        rs = ensure(ctx->dev, total, false, ctx);
        if (rs != LRA_OK) return rs;
        rs = ensure(ctx->host, u1, true, ctx);
        if (rs != LRA_OK) return rs;
        h = (uint8_t*)ctx->host.p;
        d = (uint8_t*)ctx->dev.p;
    }

    write_ctl(h, c, lp.pl);
    TaskDesc* htasks = (TaskDesc*)(h + c.tasks);
    for (size_t i = 0; i < np; ++i) {
        init_inputs(h, probs[i], regs[i]);
        init_state(h + regs[i].st, h + regs[i].I, h + regs[i].J, probs[i]);
        fill_task(htasks[i], probs[i], d, regs[i]);
    }
    *(uint64_t*)(h + off_err) = 0;
    if (pack) {
        int64_t* po = (int64_t*)(h + off_pack);
        for (size_t i = 0; i < np; ++i) {
            po[3 * i] = regs[i].st;
            po[3 * i + 1] = regs[i].G;
            po[3 * i + 2] = regs[i].U;
        }
    }

    const double t_image = now_us();
    HIP_TRY(hipMemcpyAsync(d, h, (size_t)up_end, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(launch_zero(d + z0, z1 - z0, ctx->stream));
    EngineArgs ea = engine_args(ctx, d, c, lp, phase_budget, (uint32_t*)(d + off_err),
                                trace_cap ? (uint64_t*)(d + off_trace) : nullptr, trace_cap);
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev0, ctx->stream));
    rs = launch(ctx, lp, ea, ctx->stream);
    if (rs != LRA_OK) return rs;
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev1, ctx->stream));

    if (pack)
        HIP_TRY(launch_pack_factors(d, (const int64_t*)(d + off_pack), (int)np, (double*)(d + packed),
                                    (double*)(d + packed) + kk_all, ctx->stream));
    const int64_t rb1 = pack ? up_end : want_U ? u1 : want_G ? u0 : up_end;
    HIP_TRY(hipMemcpyAsync(h + rb0, d + rb0, (size_t)(rb1 - rb0), hipMemcpyDeviceToHost, ctx->stream));
    std::vector<uint64_t> trace_host;
    if (trace_cap) {
        trace_host.resize(1 + 2 * (size_t)trace_cap);
        HIP_TRY(hipMemcpyAsync(trace_host.data(), d + off_trace, 8 * trace_host.size(), hipMemcpyDeviceToHost,
                               ctx->stream));
    }
    const double t_enq = now_us();
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    const double t_wait = now_us();
    if (trace_cap) dump_trace(ctx, trace_host.data(), trace_cap);
    if (ctx->timing) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        ctx->stats.last_engine_ms = ms;
        ctx->stats.engine_ms_total += ms;
    }
    if (*(uint32_t*)(h + off_err)) {
        LRA_LOG(1, "device-side team barrier timed out");
        return LRA_EDEVICE;
    }
    if (pack) {
        // the packed factors, at the offsets the pack kernel formed from the
        // same final ranks, into the (unused) G and U staging regions
        std::vector<int64_t> pb(np + 1, 0);
        for (size_t i = 0; i < np; ++i) {
            const int64_t k = ((const TaskState*)(h + regs[i].st))->k;
            pb[i + 1] = pb[i] + k * k;
        }
        const int64_t hg = regs[0].G;
        if (pb[np] > 0) {
            if (want_G)
                HIP_TRY(hipMemcpyAsync(h + hg, d + packed, 8 * (size_t)pb[np], hipMemcpyDeviceToHost, ctx->stream));
            if (want_U)
                HIP_TRY(hipMemcpyAsync(h + u0, d + packed + 8 * kk_all, 8 * (size_t)pb[np], hipMemcpyDeviceToHost,
                                       ctx->stream));
            HIP_TRY(hipStreamSynchronize(ctx->stream));
        }
        for (size_t i = 0; i < np; ++i) {
            const ProbRegions& r = regs[i];
            deliver(*(const TaskState*)(h + r.st), (const int64_t*)(h + r.I), (const int64_t*)(h + r.J),
                    want_G ? (const double*)(h + hg) + pb[i] : nullptr, want_U ? (const double*)(h + u0) + pb[i] : nullptr,
                    res[i]);
        }
    } else {
        for (size_t i = 0; i < np; ++i) {
            const ProbRegions& r = regs[i];
            deliver(*(const TaskState*)(h + r.st), (const int64_t*)(h + r.I), (const int64_t*)(h + r.J),
                    want_G ? (const double*)(h + r.G) : nullptr, want_U ? (const double*)(h + r.U) : nullptr, res[i]);
        }
    }
    LRA_LOG(2, "%zu problem(s): plan %.0f us, host image %.0f us, upload + launch %.0f us, wait %.0f us, "
            "results %.0f us", np, t_plan1 - t_plan0, t_image - t_plan1, t_enq - t_image, t_wait - t_enq,
            now_us() - t_wait);
    return LRA_OK;
}

// ----------------------------------------------------------------------------
// public entry points
// ----------------------------------------------------------------------------

static lra_status ca_cur_one(lra_ctx* ctx, const lra_source* src, int64_t m, int64_t n, int k, int sweeps,
                             double tol, const lra_options* opts, lra_result* result, const FixedBuffers* fixed)
{
    if (!ctx || !result) return LRA_EINVAL;
    lra_options o;
    if (opts) o = *opts;
    else lra_default_options(&o);
    std::vector<Prob> probs(1);
    lra_status rs = make_prob(src, m, n, k, sweeps, tol, &o, probs[0], 0);
    if (rs != LRA_OK) return rs;
    const int prec64 = o.precision == LRA_PREC_FP64;
    probs[0].team = o.team_wgs > 0 ? std::min(o.team_wgs, NT) : auto_team(ctx, probs[0], prec64);
    probs[0].C_out = result->C_out;
    probs[0].R_out = result->R_out;
    lra_result* rp = result;
    rs = run_batch(ctx, probs, prec64, 1 << 30, &rp, fixed);
    if (rs != LRA_OK) return rs;
    return (lra_status)result->status;
}

extern "C" lra_status lra_ca_cur(lra_ctx* ctx, const lra_source* src, int64_t m, int64_t n, int k, int sweeps,
                                 double tol, const lra_options* opts, lra_result* result)
{
    return ca_cur_one(ctx, src, m, n, k, sweeps, tol, opts, result, nullptr);
}

// Host staging of the allocation-free entry point; the lock serialises its
// calls (they share this array and the device's scratch array).
namespace {
std::mutex noalloc_mu;
alignas(256) uint8_t noalloc_host[NOALLOC_HOST_BYTES];
}  // namespace

extern "C" lra_status lra_ca_cur_noalloc(lra_ctx* ctx, const lra_source* src, int64_t m, int64_t n, int k,
                                         int sweeps, double tol, const lra_options* opts, lra_result* result)
{
    static_assert(LRA_NOALLOC_SCRATCH_BYTES == (size_t)NOALLOC_SCRATCH_BYTES, "scratch size");
    if (!ctx || !result) return LRA_EINVAL;
    uint8_t* dev = (uint8_t*)noalloc_scratch(ctx->device);
    if (!dev) return LRA_EDEVICE;  // lra_create looks the address up; never reached after it succeeded
    std::lock_guard<std::mutex> lk(noalloc_mu);
    const FixedBuffers fb{dev, NOALLOC_SCRATCH_BYTES, noalloc_host, NOALLOC_HOST_BYTES};
    return ca_cur_one(ctx, src, m, n, k, sweeps, tol, opts, result, &fb);
}

extern "C" lra_status lra_cur_factors(lra_ctx* ctx, const lra_source* src, int64_t m, int64_t n, int k,
                                      const int64_t* I, const int64_t* J, int32_t out_dtype, void* C_out,
                                      void* R_out)
{
    if (!ctx || !src_ok(src) || m < 1 || n < 1 || k < 1 || !I || !J) return LRA_EINVAL;
    if (out_dtype != LRA_F32 && out_dtype != LRA_F64) return LRA_EINVAL;
    if (m * (int64_t)k >= ((int64_t)1 << 31) || n * (int64_t)k >= ((int64_t)1 << 31)) return LRA_EINVAL;
    if ((src->kind == LRA_SRC_DENSE || src->kind == LRA_SRC_PREPROCESSED) && src->lda < (src->col_major ? m : n))
        return LRA_EINVAL;
    if (!shape_ok(src, m, n)) return LRA_EINVAL;
    for (int c = 0; c < k; ++c)
        if (I[c] < 0 || I[c] >= m || J[c] < 0 || J[c] >= n) return LRA_EINVAL;
    if (!C_out && !R_out) return LRA_OK;
    const int64_t bytes = 16 * (int64_t)k;
    lra_status rs = ensure(ctx->dev, bytes, false, ctx);
    if (rs != LRA_OK) return rs;
    rs = ensure(ctx->host, bytes, true, ctx);
    if (rs != LRA_OK) return rs;
    int64_t* h = (int64_t*)ctx->host.p;
    std::memcpy(h, I, 8 * (size_t)k);
    std::memcpy(h + k, J, 8 * (size_t)k);
    int64_t* d = (int64_t*)ctx->dev.p;
    const DevSource ds = dev_source(src, m, n);
    HIP_TRY(hipMemcpyAsync(d, h, (size_t)bytes, hipMemcpyHostToDevice, ctx->stream));
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev0, ctx->stream));
    HIP_TRY(launch_factors(ds, m, n, k, d, d + k, out_dtype == LRA_F64, C_out, R_out, ctx->stream));
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev1, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->stats.launches += 1;
    if (ctx->timing) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        ctx->stats.last_engine_ms = ms;
        ctx->stats.engine_ms_total += ms;
    }
    return LRA_OK;
}

// Rows of the next TSQR level: k rows per 256-row block of this one.
static int64_t tsqr_blocks(int64_t rows) { return (rows + 255) / 256; }

extern "C" lra_status lra_top_svd(lra_ctx* ctx, int64_t m, int64_t n, int k, int r, int32_t dtype, const void* C,
                                  int64_t ldc, const double* W, const void* R, int64_t ldr, double* S, int64_t lds,
                                  double* sigma, double* Tt, int64_t ldt, int64_t* piv_c, int64_t* piv_r)
{
    if (!ctx || !C || !W || !R || !S || !sigma || !Tt) return LRA_EINVAL;
    if (k < 1 || k > 64 || r < 1 || r > k || m < k || n < k) return LRA_EINVAL;
    if (dtype != LRA_F32 && dtype != LRA_F64) return LRA_EINVAL;
    if (ldc < m || ldr < n || lds < m || ldt < n) return LRA_EINVAL;
    if (m * (int64_t)k >= ((int64_t)1 << 40) || n * (int64_t)k >= ((int64_t)1 << 40)) return LRA_EINVAL;
    for (int i = 0; i < k * k; ++i)
        if (!std::isfinite(W[i])) return LRA_ENONFINITE;
    // device workspace: two ping-pong level buffers per factor, W, the core block
    const int64_t lvl_c = tsqr_blocks(m) * k * k, lvl_r = tsqr_blocks(n) * k * k;
    const int64_t off_w = 2 * (lvl_c + lvl_r) * 8;
    const int64_t off_core = align_up(off_w + 8 * (int64_t)k * k, 256);
    const int64_t dev_bytes = off_core + (int64_t)core_out_bytes();
    lra_status rs = ensure(ctx->dev, dev_bytes, false, ctx);
    if (rs != LRA_OK) return rs;
    const int64_t host_bytes = std::max<int64_t>(8 * (int64_t)k * k, (int64_t)core_out_bytes());
    rs = ensure(ctx->host, host_bytes, true, ctx);
    if (rs != LRA_OK) return rs;
    double* d = (double*)ctx->dev.p;
    double* bc[2] = {d, d + lvl_c};
    double* br[2] = {d + 2 * lvl_c, d + 2 * lvl_c + lvl_r};
    double* dw = (double*)((uint8_t*)ctx->dev.p + off_w);
    void* dcore = (uint8_t*)ctx->dev.p + off_core;
    std::memcpy(ctx->host.p, W, 8 * (size_t)k * k);
    HIP_TRY(hipMemcpyAsync(dw, ctx->host.p, 8 * (size_t)k * k, hipMemcpyHostToDevice, ctx->stream));
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev0, ctx->stream));
    // TSQR of C and of R^T (R row-major k x n is R^T column-major, ld ldr)
    const void* xc = C;
    const void* xr = R;
    int64_t rc = m, rr = n, ldxc = ldc, ldxr = ldr;
    int dtc = dtype, dtr = dtype;
    int lc = 0, lr = 0;       // ping-pong index of the next output
    bool done_c = false, done_r = false;
    const double* RC = nullptr;
    const double* RR = nullptr;
    int launches = 0;
    while (!done_c || !done_r) {
        const int nbc = done_c ? 0 : (int)tsqr_blocks(rc);
        const int nbr = done_r ? 0 : (int)tsqr_blocks(rr);
        double* oc = bc[lc];
        double* orr = br[lr];
        HIP_TRY(launch_tsqr(xc, rc, ldxc, dtc, nbc, oc, xr, rr, ldxr, dtr, nbr, orr, k, ctx->stream));
        ++launches;
        if (!done_c) {
            if (nbc == 1) {
                done_c = true;
                RC = oc;
            } else {
                xc = oc;
                rc = (int64_t)nbc * k;
                ldxc = rc;
                dtc = LRA_F64;
                lc ^= 1;
            }
        }
        if (!done_r) {
            if (nbr == 1) {
                done_r = true;
                RR = orr;
            } else {
                xr = orr;
                rr = (int64_t)nbr * k;
                ldxr = rr;
                dtr = LRA_F64;
                lr ^= 1;
            }
        }
    }
    HIP_TRY(launch_topsvd_core(RC, RR, dw, k, r, (double)std::max(m, n) * 0x1p-53, dcore, ctx->stream));
    // the apply kernel leaves S and T^T alone when the core reports rank loss
    HIP_TRY(launch_topsvd_apply(C, ldc, R, ldr, dtype, m, n, r, dcore, S, lds, Tt, ldt, ctx->stream));
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev1, ctx->stream));
    HIP_TRY(hipMemcpyAsync(ctx->host.p, dcore, core_out_bytes(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    int32_t st = 0, sweeps = 0;
    const int32_t* pc = nullptr;
    const int32_t* pr = nullptr;
    const double* sg = nullptr;
    const int64_t* tk = nullptr;
    topsvd_core_fields(ctx->host.p, &st, &sweeps, &pc, &pr, &sg, &tk);
    if (piv_c && st != LRA_ENONFINITE)
        for (int j = 0; j < k; ++j) piv_c[j] = pc[j];
    if (piv_r && st != LRA_ENONFINITE)
        for (int j = 0; j < k; ++j) piv_r[j] = pr[j];
    ctx->stats.launches += launches + 2;
    if (ctx->timing) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        ctx->stats.last_engine_ms = ms;
        ctx->stats.engine_ms_total += ms;
    }
    LRA_LOG(2, "top SVD: m %lld n %lld k %d r %d, %d TSQR launches, %d Jacobi sweeps, status %d", (long long)m,
            (long long)n, k, r, launches, sweeps, st);
    if (st == 0) {
        const double us = 1e3 / (double)ctx->wall_rate_khz;
        LRA_LOG(2, "top SVD core: QR %.1f us, middle %.1f us, Jacobi %.1f us, sort %.1f us, solves %.1f us",
                (tk[1] - tk[0]) * us, (tk[2] - tk[1]) * us, (tk[3] - tk[2]) * us, (tk[4] - tk[3]) * us,
                (tk[5] - tk[4]) * us);
    }
    if (st != 0) return (lra_status)st;
    for (int j = 0; j < r; ++j) sigma[j] = sg[j];
    return LRA_OK;
}

extern "C" lra_status lra_maxvol(lra_ctx* ctx, const void* strip, int32_t dtype, int64_t m, int64_t ld, int k,
                                 double tau, int max_swaps, const int64_t* init, int64_t* I, int* swaps, int* k_eff)
{
    if (!ctx || !strip || !I || k < 1 || k > 64 || m < k || ld < m || !(tau >= 0.0)) return LRA_EINVAL;
    if (dtype != LRA_F32 && dtype != LRA_F64) return LRA_EINVAL;
    lra_source s;
    std::memset(&s, 0, sizeof(s));
    s.kind = LRA_SRC_DENSE;
    s.dtype = dtype;
    s.a = strip;
    s.lda = ld;
    s.col_major = 1;
    lra_options o;
    lra_default_options(&o);
    o.tau = tau;
    o.max_swaps = max_swaps;
    o.precision = dtype == LRA_F64 ? LRA_PREC_FP64 : LRA_PREC_MIXED;
    std::vector<int64_t> cols(k);
    for (int c = 0; c < k; ++c) cols[c] = c;
    o.init_cols = cols.data();
    o.n_init_cols = k;
    o.sample_q = 1;
    o.sample_s = 1;
    std::vector<Prob> probs(1);
    lra_status rs = make_prob(&s, m, k, k, 1, 0.0, &o, probs[0], 0);
    if (rs != LRA_OK) return rs;
    if (init) {
        probs[0].have_init_I = true;
        probs[0].init_I.assign(init, init + k);
        for (int a = 0; a < k; ++a) {
            if (init[a] < 0 || init[a] >= m) return LRA_EINVAL;
            for (int b = a + 1; b < k; ++b)
                if (init[a] == init[b]) return LRA_EINVAL;
        }
    }
    const int prec64 = dtype == LRA_F64;
    probs[0].team = auto_team(ctx, probs[0], prec64);
    lra_result r;
    std::memset(&r, 0, sizeof(r));
    std::vector<int64_t> Iout(k);
    r.I = Iout.data();
    lra_result* rp = &r;
    rs = run_batch(ctx, probs, prec64, 1, &rp);
    if (rs != LRA_OK) return rs;
    if (r.status < 0) return (lra_status)r.status;
    for (int c = 0; c < r.k; ++c) I[c] = Iout[c];
    if (swaps) *swaps = r.swaps_total;
    if (k_eff) *k_eff = r.k;
    return (lra_status)r.status;
}

extern "C" lra_status lra_ca_cur_batched(lra_ctx* ctx, const lra_block* blocks, int nblocks, const lra_options* opts,
                                         lra_result* results)
{
    if (!ctx || nblocks < 0 || (nblocks > 0 && (!blocks || !results))) return LRA_EINVAL;
    if (nblocks == 0) return LRA_OK;
    lra_options o;
    if (opts) o = *opts;
    else lra_default_options(&o);
    if (o.init_cols || o.sample_rows || o.sample_cols || o.init_rows) return LRA_EINVAL;
    const int prec64 = o.precision == LRA_PREC_FP64;
    const double t0 = now_us();
    std::vector<Prob> probs(nblocks);
    std::vector<lra_result*> rp(nblocks);
    std::vector<lra_status> bst(nblocks, LRA_OK);
    // each block's description (validation, seeded candidate and sample draws)
    // is independent of the others: thousands of blocks are described on
    // several host threads
    const auto describe = [&](int b0, int b1) {
        for (int b = b0; b < b1; ++b) {
            const lra_block& bl = blocks[b];
            bst[b] = make_prob(&bl.src, bl.m, bl.n, bl.k, bl.sweeps, bl.tol, &o, probs[b], b);
            if (bst[b] != LRA_OK) continue;
            // power-of-two team sizes keep the number of size classes small
            probs[b].team = o.team_wgs > 0 ? std::min(o.team_wgs, NT)
                                           : std::min(NT, pow2_ceil(auto_team(ctx, probs[b], prec64)));
            probs[b].team_fixed = o.team_wgs > 0;
            probs[b].C_out = results[b].C_out;
            probs[b].R_out = results[b].R_out;
            rp[b] = &results[b];
        }
    };
    const int nthr = nblocks >= 256 ? std::max(1, std::min(8, (int)std::thread::hardware_concurrency())) : 1;
    if (nthr > 1) {
        std::vector<std::thread> pool;
        const int per = (nblocks + nthr - 1) / nthr;
        for (int t = 0; t < nthr; ++t)
            if (t * per < nblocks) pool.emplace_back(describe, t * per, std::min(nblocks, (t + 1) * per));
        for (auto& th : pool) th.join();
    } else {
        describe(0, nblocks);
    }
    for (int b = 0; b < nblocks; ++b)
        if (bst[b] != LRA_OK) return bst[b];
    LRA_LOG(2, "%d block(s) described in %.0f us", nblocks, now_us() - t0);
    lra_status rs = run_batch(ctx, probs, prec64, 1 << 30, rp.data());
    if (rs != LRA_OK) return rs;
    lra_status worst = LRA_OK;
    for (int b = 0; b < nblocks; ++b)
        if (severity((lra_status)results[b].status) > severity(worst)) worst = (lra_status)results[b].status;
    return worst;
}

// ----------------------------------------------------------------------------
// serving: continuous batching of independent requests
// ----------------------------------------------------------------------------
//
// Admitted requests own a region of a device arena (inputs, state, results,
// scratch, a global strip) and a slot of a state table at the arena's start.
// A tick launches the engine once per (precision, KMAX) group over every
// admitted request with a budget of a few phases each (a phase is one column
// step, one row step, or the nucleus + estimate); the engine leaves each
// request's resumable state in HBM.  When the tick has finished, the state
// table comes back in one copy; completed requests are delivered and release
// their region, waiting requests are admitted first come first served, and
// the next tick is launched.  lra_poll never waits for the device.

struct Request {
    uint64_t ticket = 0;
    lra_result* res = nullptr;
    Prob p;
    int prec64 = 1;
    int kmx = 8;
    int team = 1;
    int64_t footprint = 0;
    int64_t arena_off = -1;
    int slot = -1;
    ProbRegions r;      // offsets relative to the arena base
    double t_submit = 0.0, t_start = 0.0;
};

// First-fit allocator over [0, size).
struct FreeList {
    std::map<int64_t, int64_t> free;  // offset -> bytes
    void reset(int64_t size)
    {
        free.clear();
        if (size > 0) free[0] = size;
    }
    int64_t alloc(int64_t bytes)
    {
        for (auto it = free.begin(); it != free.end(); ++it) {
            if (it->second < bytes) continue;
            const int64_t off = it->first, left = it->second - bytes;
            free.erase(it);
            if (left > 0) free[off + bytes] = left;
            return off;
        }
        return -1;
    }
    void release(int64_t off, int64_t bytes)
    {
        auto it = free.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free.erase(nx);
        }
        if (it != free.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free.erase(it);
            }
        }
    }
};

struct Serve {
    Buffer arena;                 // device: state table, then request regions
    Buffer ctl_dev;               // device: control images of a tick
    Buffer host;                  // pinned: control images, admitted inputs, read-back
    int64_t arena_bytes = 0;      // 0: chosen at the first submit
    int64_t table_bytes = 0;
    int phases_per_tick = 4;
    int max_active = 1024;
    FreeList fl;
    std::vector<int> free_slots;
    std::deque<Request*> pending;
    std::vector<Request*> active;
    std::map<uint64_t, std::unique_ptr<Request>> live;
    std::map<uint64_t, lra_status> done;
    uint64_t next_ticket = 1;
    bool in_flight = false;
    bool failed = false;
    hipEvent_t ev = nullptr;
    int64_t tick_tbl_off = 0;       // host staging offsets of the in-flight tick's
    int64_t tick_err_off = 0;       // state table and error words
    int tick_groups = 0;
    int64_t ticks = 0;
    double tick_t0 = 0.0;           // host time of the in-flight tick's launch
    size_t tick_active = 0;
};

static int64_t request_footprint(const Prob& p, int prec64)
{
    Layout L;
    L.add(8 * (int64_t)p.cand.size(), 8);
    L.add(8 * (int64_t)p.q, 8);
    L.add(8 * (int64_t)p.s, 8);
    L.add(8 * (int64_t)p.kcap, 8);
    L.add(8 * (int64_t)p.kcap, 8);
    L.add(8 * (int64_t)p.kcap * p.kcap, 8);
    L.add(8 * (int64_t)p.kcap * p.kcap, 8);
    L.add(8 * (int64_t)p.kcap);
    L.add(8 * (int64_t)p.kcap);
    L.add(work_bytes(p));
    L.add(strip_bytes(p, prec64));
    return align_up(L.size, 256);
}

// Region of an admitted request: [cand | Q | S | I | J | G | U] then scratch;
// [cand .. J] is uploaded at admission, [I .. U] read back at completion.
static ProbRegions request_regions(const Prob& p, int prec64, int64_t base)
{
    Layout L;
    L.size = base;
    ProbRegions r;
    r.cand = L.add(8 * (int64_t)p.cand.size(), 8);
    r.Q = L.add(8 * (int64_t)p.q, 8);
    r.S = L.add(8 * (int64_t)p.s, 8);
    r.I = L.add(8 * (int64_t)p.kcap, 8);
    r.J = L.add(8 * (int64_t)p.kcap, 8);
    r.G = L.add(8 * (int64_t)p.kcap * p.kcap, 8);
    r.U = L.add(8 * (int64_t)p.kcap * p.kcap, 8);
    r.prevI = L.add(8 * (int64_t)p.kcap);
    r.prevJ = L.add(8 * (int64_t)p.kcap);
    r.work = L.add(work_bytes(p));
    r.strip = L.add(strip_bytes(p, prec64));
    return r;
}

static lra_status serve_init(lra_ctx* ctx)
{
    Serve& s = *ctx->srv;
    if (s.arena.p) return LRA_OK;
    if (s.arena_bytes <= 0) {
        const int64_t def = 4ll << 30;
        s.arena_bytes = ctx->budget ? std::min<int64_t>(def, (int64_t)ctx->budget / 2) : def;
    }
    s.table_bytes = align_up((int64_t)s.max_active * (int64_t)sizeof(TaskState), 256);
    if (s.arena_bytes <= s.table_bytes) return LRA_EBUDGET;
    if (ctx->budget && (size_t)(s.arena_bytes + ctx->dev_in_use) > ctx->budget) return LRA_EBUDGET;
    if (hipMalloc(&s.arena.p, (size_t)s.arena_bytes) != hipSuccess) {
        s.arena.p = nullptr;
        return LRA_ENOMEM;
    }
    s.arena.bytes = s.arena_bytes;
    ctx->dev_in_use += s.arena_bytes;
    ctx->dev_allocs += 1;
    s.fl.reset(s.arena_bytes - s.table_bytes);
    s.free_slots.clear();
    for (int i = s.max_active - 1; i >= 0; --i) s.free_slots.push_back(i);
    HIP_TRY(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
    return LRA_OK;
}

static void finish_request(lra_ctx* ctx, Request* q, lra_status st)
{
    Serve& s = *ctx->srv;
    q->res->status = (int32_t)st;
    q->res->t_submit_us = q->t_submit;
    q->res->t_start_us = q->t_start;
    q->res->t_end_us = now_us();
    if (q->arena_off >= 0) s.fl.release(q->arena_off, q->footprint);
    if (q->slot >= 0) s.free_slots.push_back(q->slot);
    s.done[q->ticket] = st;
    s.live.erase(q->ticket);
}

// Launch one tick: admit what fits, then one engine launch per group.
static lra_status serve_launch(lra_ctx* ctx)
{
    Serve& s = *ctx->srv;
    // admission, first come first served (the head of the queue blocks)
    std::vector<Request*> admitted;
    while (!s.pending.empty() && !s.free_slots.empty()) {
        Request* q = s.pending.front();
        const int64_t off = s.fl.alloc(q->footprint);
        if (off < 0) break;
        s.pending.pop_front();
        q->arena_off = off;
        q->slot = s.free_slots.back();
        s.free_slots.pop_back();
        q->r = request_regions(q->p, q->prec64, s.table_bytes + off);
        q->r.st = (int64_t)q->slot * (int64_t)sizeof(TaskState);
        q->t_start = now_us();
        s.active.push_back(q);
        admitted.push_back(q);
    }
    if (s.active.empty()) return LRA_OK;

    // one launch: the variant's own kernel when all requests share one, else
    // the all-variant kernel (key (0, 0))
    std::map<std::pair<int, int>, std::vector<Request*>> groups;
    for (Request* q : s.active) groups[{q->prec64, q->kmx}].push_back(q);
    if (groups.size() > 1) {
        std::vector<Request*> all = s.active;
        groups.clear();
        groups[{0, 0}] = all;
    }
    struct G {
        int prec64;
        LaunchPlan lp;
        CtlImage c;
        std::vector<Request*> reqs;
    };
    std::vector<G> gs;
    Layout L;   // control images, device and host alike
    for (auto& kv : groups) {
        G g;
        g.prec64 = kv.first.first;
        g.reqs = kv.second;
        std::vector<Prob*> pp;
        for (Request* q : g.reqs) {
            q->p.team = q->team;
            pp.push_back(&q->p);
        }
        lra_status rs = plan_launch(ctx, pp, g.prec64, kv.first.second, true, g.lp);
        if (rs != LRA_OK) return rs;
        lay_ctl_upload(L, g.c, g.reqs.size(), g.lp.pl);
        gs.push_back(std::move(g));
    }
    const int64_t ctl_up_end = L.size;
    const int64_t zero0 = L.add(0);
    for (auto& g : gs) lay_ctl_zero(L, g.c, g.lp.pl);
    const int64_t err_off = L.add(8 * (int64_t)gs.size(), 8);
    const int64_t zero1 = L.size;
    const int64_t dev_bytes = L.size;
    // host staging: control images, then admitted requests' uploads, then the state table read-back
    std::vector<int64_t> adm_off(admitted.size());
    for (size_t i = 0; i < admitted.size(); ++i) {
        Request* q = admitted[i];
        adm_off[i] = L.add(q->r.G - q->r.cand + sizeof(TaskState));
    }
    int max_slot = 0;
    for (Request* q : s.active) max_slot = std::max(max_slot, q->slot + 1);
    const int64_t tbl_off = L.add((int64_t)max_slot * (int64_t)sizeof(TaskState));
    const int64_t err_rb = L.add(8 * (int64_t)gs.size(), 8);
    lra_status rs = ensure(s.ctl_dev, dev_bytes, false, ctx);
    if (rs != LRA_OK) return rs;
    rs = ensure(s.host, L.size, true, ctx);
    if (rs != LRA_OK) return rs;
    uint8_t* h = (uint8_t*)s.host.p;
    uint8_t* dc = (uint8_t*)s.ctl_dev.p;
    uint8_t* da = (uint8_t*)s.arena.p;

    // uploads of admitted requests: [cand .. J] and the state slot
    for (size_t i = 0; i < admitted.size(); ++i) {
        Request* q = admitted[i];
        const ProbRegions& r = q->r;
        uint8_t* hb = h + adm_off[i] - r.cand;   // host image addressed like the arena
        init_inputs(hb, q->p, r);
        uint8_t* hst = h + adm_off[i] + (r.G - r.cand);
        init_state(hst, hb + r.I, hb + r.J, q->p);
        HIP_TRY(hipMemcpyAsync(da + r.cand, h + adm_off[i], (size_t)(r.G - r.cand), hipMemcpyHostToDevice,
                               ctx->stream));
        HIP_TRY(hipMemcpyAsync(da + r.st, hst, sizeof(TaskState), hipMemcpyHostToDevice, ctx->stream));
    }
    for (size_t gi = 0; gi < gs.size(); ++gi) {
        G& g = gs[gi];
        write_ctl(h, g.c, g.lp.pl);
        TaskDesc* td = (TaskDesc*)(h + g.c.tasks);
        for (size_t i = 0; i < g.reqs.size(); ++i) fill_task(td[i], g.reqs[i]->p, da, g.reqs[i]->r);
    }
    HIP_TRY(hipMemcpyAsync(dc, h, (size_t)ctl_up_end, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(launch_zero(dc + zero0, zero1 - zero0, ctx->stream));
    for (size_t gi = 0; gi < gs.size(); ++gi) {
        G& g = gs[gi];
        EngineArgs ea = engine_args(ctx, dc, g.c, g.lp, s.phases_per_tick, (uint32_t*)(dc + err_off + 8 * gi),
                                    nullptr, 0);
        rs = launch(ctx, g.lp, ea, ctx->stream);
        if (rs != LRA_OK) return rs;
    }
    HIP_TRY(hipMemcpyAsync(h + tbl_off, da, (size_t)max_slot * sizeof(TaskState), hipMemcpyDeviceToHost,
                           ctx->stream));
    HIP_TRY(hipMemcpyAsync(h + err_rb, dc + err_off, 8 * gs.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipEventRecord(s.ev, ctx->stream));
    s.in_flight = true;
    s.tick_t0 = now_us();
    s.tick_active = s.active.size();
    LRA_LOG(2, "tick %lld launched: %zu active (%zu admitted), %zu waiting, %zu launch(es)", (long long)s.ticks,
            s.active.size(), admitted.size(), s.pending.size(), gs.size());
    s.tick_tbl_off = tbl_off;
    s.tick_err_off = err_rb;
    s.tick_groups = (int)gs.size();
    s.ticks += 1;
    ctx->stats.ticks += 1;
    return LRA_OK;
}

static void serve_fail_all(lra_ctx* ctx, lra_status st)
{
    Serve& s = *ctx->srv;
    for (Request* q : s.active) finish_request(ctx, q, st);
    s.active.clear();
    while (!s.pending.empty()) {
        Request* q = s.pending.front();
        s.pending.pop_front();
        finish_request(ctx, q, st);
    }
}

// The in-flight tick has finished: deliver the completed requests.
static lra_status serve_complete(lra_ctx* ctx)
{
    Serve& s = *ctx->srv;
    s.in_flight = false;
    const uint8_t* h = (const uint8_t*)s.host.p;
    bool dev_err = false;
    for (int g = 0; g < s.tick_groups; ++g)
        if (*(const uint32_t*)(h + s.tick_err_off + 8 * g)) dev_err = true;
    if (dev_err) {
        LRA_LOG(1, "device-side team barrier timed out while serving");
        serve_fail_all(ctx, LRA_EDEVICE);
        return LRA_EDEVICE;
    }
    const TaskState* tbl = (const TaskState*)(h + s.tick_tbl_off);
    std::vector<Request*> fin, keep;
    std::vector<TaskState> fst;
    for (Request* q : s.active) {
        const TaskState& st = tbl[q->slot];
        if (st.phase == PH_DONE || st.status < 0) {
            fin.push_back(q);
            fst.push_back(st);
        } else {
            keep.push_back(q);
        }
    }
    s.active = keep;
    LRA_LOG(2, "tick done after %.3f ms: %zu of %zu finished", (now_us() - s.tick_t0) * 1e-3, fin.size(),
            s.tick_active);
    if (fin.empty()) return LRA_OK;
    // read back [I | J | G | U] of every completed request
    Layout L;
    std::vector<int64_t> off(fin.size());
    for (size_t i = 0; i < fin.size(); ++i) {
        const ProbRegions& r = fin[i]->r;
        off[i] = L.add(r.U + 8 * (int64_t)fin[i]->p.kcap * fin[i]->p.kcap - r.I);
    }
    lra_status rs = ensure(s.host, L.size, true, ctx);
    if (rs != LRA_OK) return rs;
    uint8_t* hh = (uint8_t*)s.host.p;
    const uint8_t* da = (const uint8_t*)s.arena.p;
    for (size_t i = 0; i < fin.size(); ++i) {
        const ProbRegions& r = fin[i]->r;
        const int64_t bytes = r.U + 8 * (int64_t)fin[i]->p.kcap * fin[i]->p.kcap - r.I;
        HIP_TRY(hipMemcpyAsync(hh + off[i], da + r.I, (size_t)bytes, hipMemcpyDeviceToHost, ctx->stream));
    }
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (size_t i = 0; i < fin.size(); ++i) {
        Request* q = fin[i];
        const ProbRegions& r = q->r;
        const uint8_t* b = hh + off[i] - r.I;
        deliver(fst[i], (const int64_t*)(b + r.I), (const int64_t*)(b + r.J), (const double*)(b + r.G),
                (const double*)(b + r.U), q->res);
        finish_request(ctx, q, status_of(fst[i]));
    }
    return LRA_OK;
}

// Advance the scheduler: finish the in-flight tick if it is done (or wait
// for it when `block`), then launch the next one when work remains.
static lra_status serve_progress(lra_ctx* ctx, bool block)
{
    Serve& s = *ctx->srv;
    if (s.in_flight) {
        if (!block) {
            const hipError_t q = hipEventQuery(s.ev);
            if (q == hipErrorNotReady) return LRA_OK;
            if (q != hipSuccess) {
                serve_fail_all(ctx, LRA_EDEVICE);
                return hip_fail(q, "hipEventQuery");
            }
        } else {
            const hipError_t q = hipEventSynchronize(s.ev);
            if (q != hipSuccess) {
                serve_fail_all(ctx, LRA_EDEVICE);
                return hip_fail(q, "hipEventSynchronize");
            }
        }
        lra_status rs = serve_complete(ctx);
        if (rs < 0) return rs;
    }
    if (!s.active.empty() || !s.pending.empty()) {
        lra_status rs = serve_launch(ctx);
        if (rs < 0) {
            (void)hipStreamSynchronize(ctx->stream);
            s.in_flight = false;
            serve_fail_all(ctx, rs);
            return rs;
        }
    }
    return LRA_OK;
}

extern "C" lra_status lra_serve_config(lra_ctx* ctx, size_t arena_bytes, int phases_per_tick, int max_active)
{
    if (!ctx || phases_per_tick < 0 || max_active < 0) return LRA_EINVAL;
    if (!ctx->srv) ctx->srv = new Serve();
    Serve& s = *ctx->srv;
    if (s.arena.p && ((arena_bytes && (int64_t)arena_bytes != s.arena_bytes) ||
                      (max_active && max_active != s.max_active)))
        return LRA_EINVAL;
    if (arena_bytes) s.arena_bytes = (int64_t)arena_bytes;
    if (max_active) s.max_active = max_active;
    if (phases_per_tick) s.phases_per_tick = phases_per_tick;
    return LRA_OK;
}

extern "C" lra_status lra_submit(lra_ctx* ctx, const lra_request* req, uint64_t* ticket)
{
    if (!ctx || !req || !ticket || !req->result) return LRA_EINVAL;
    if (!ctx->srv) ctx->srv = new Serve();
    Serve& s = *ctx->srv;
    if (s.failed) return LRA_EDEVICE;
    auto q = std::make_unique<Request>();
    lra_status rs = make_prob(&req->src, req->m, req->n, req->k, req->sweeps, req->tol, &req->opts, q->p, 0);
    if (rs != LRA_OK) return rs;
    q->prec64 = req->opts.precision == LRA_PREC_FP64;
    q->team = req->opts.team_wgs > 0 ? std::min(req->opts.team_wgs, NT)
                                     : std::min(NT, pow2_ceil(auto_team(ctx, q->p, q->prec64)));
    q->p.team_fixed = req->opts.team_wgs > 0;
    q->kmx = kmax_bucket(q->p.kcap);
    q->p.prec64 = q->prec64;
    q->p.kmx = q->kmx;
    q->p.need_strip = true;
    q->p.C_out = req->result->C_out;
    q->p.R_out = req->result->R_out;
    q->footprint = request_footprint(q->p, q->prec64);
    rs = serve_init(ctx);
    if (rs != LRA_OK) return rs;
    if (q->footprint > s.arena_bytes - s.table_bytes) return LRA_EBUDGET;
    q->ticket = s.next_ticket++;
    q->res = req->result;
    q->res->status = LRA_PENDING;
    q->t_submit = now_us();
    *ticket = q->ticket;
    s.pending.push_back(q.get());
    s.live[q->ticket] = std::move(q);
    rs = serve_progress(ctx, false);
    return rs < 0 ? rs : LRA_OK;
}

extern "C" lra_status lra_poll(lra_ctx* ctx, uint64_t ticket)
{
    if (!ctx || !ctx->srv) return LRA_EINVAL;
    Serve& s = *ctx->srv;
    auto d = s.done.find(ticket);
    if (d != s.done.end()) return d->second;
    if (!s.live.count(ticket)) return LRA_EINVAL;
    lra_status rs = serve_progress(ctx, false);
    d = s.done.find(ticket);
    if (d != s.done.end()) return d->second;
    return rs < 0 ? rs : LRA_PENDING;
}

extern "C" lra_status lra_wait(lra_ctx* ctx, uint64_t ticket)
{
    if (!ctx || !ctx->srv) return LRA_EINVAL;
    Serve& s = *ctx->srv;
    for (;;) {
        auto d = s.done.find(ticket);
        if (d != s.done.end()) return d->second;
        if (!s.live.count(ticket)) return LRA_EINVAL;
        const bool had_work = s.in_flight || !s.active.empty() || !s.pending.empty();
        lra_status rs = serve_progress(ctx, true);
        if (rs < 0) {
            d = s.done.find(ticket);
            return d != s.done.end() ? d->second : rs;
        }
        if (!had_work) return LRA_EDEVICE;  // nothing could advance the ticket
    }
}


// ----------------------------------------------------------------------------
// autotuning: time candidates with HIP events, keep the fastest in the context
// ----------------------------------------------------------------------------

// Median engine time of `reps` runs (after one warm-up) of a problem set.
static lra_status time_batch(lra_ctx* ctx, std::vector<Prob> probs, int prec64, int reps, double* ms)
{
    std::vector<lra_result> res(probs.size());
    std::vector<lra_result*> rp(probs.size());
    for (size_t i = 0; i < probs.size(); ++i) {
        std::memset(&res[i], 0, sizeof(lra_result));
        rp[i] = &res[i];
    }
    const bool was_timing = ctx->timing;
    const lra_stats saved = ctx->stats;
    if (!ctx->ev0) {
        HIP_TRY(hipEventCreate(&ctx->ev0));
        HIP_TRY(hipEventCreate(&ctx->ev1));
    }
    ctx->timing = true;
    std::vector<double> t;
    lra_status rs = LRA_OK;
    for (int r = 0; r <= reps && rs == LRA_OK; ++r) {
        std::vector<Prob> copy = probs;
        rs = run_batch(ctx, copy, prec64, 1 << 30, rp.data());
        if (r > 0) t.push_back(ctx->stats.last_engine_ms);
    }
    ctx->timing = was_timing;
    ctx->stats = saved;
    if (rs != LRA_OK) return rs;
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return LRA_OK;
}

extern "C" lra_status lra_autotune_team(lra_ctx* ctx, const lra_source* src, int64_t m, int64_t n, int k, int sweeps,
                                        double tol, const lra_options* opts, int* best_team, double* best_ms)
{
    if (!ctx) return LRA_EINVAL;
    lra_options o;
    if (opts) o = *opts;
    else lra_default_options(&o);
    std::vector<Prob> probs(1);
    lra_status rs = make_prob(src, m, n, k, sweeps, tol, &o, probs[0], 0);
    if (rs != LRA_OK) return rs;
    const int prec64 = o.precision == LRA_PREC_FP64;
    const int base = auto_team(ctx, probs[0], prec64, false);
    int occ = 0;
    const int kmx = kmax_bucket(probs[0].kcap);
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, engine_kernel_ptr(prec64, kmx), NT,
                                                         engine_smem_fixed(prec64, kmx) + strip_lds(ctx, prec64, kmx)));
    const int cap = std::min(NT, std::max(1, occ) * ctx->num_cu);
    std::vector<int> cand = {std::max(1, base / 4), std::max(1, base / 2), base, std::min(cap, base + base / 2),
                             std::min(cap, base * 2), std::min(cap, base * 4)};
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    int best = base;
    double bms = 1e300;
    for (int c : cand) {
        probs[0].team = c;
        probs[0].team_fixed = true;
        double ms = 0.0;
        rs = time_batch(ctx, probs, prec64, 3, &ms);
        if (rs != LRA_OK) return rs;
        LRA_LOG(1, "autotune team %d: %.3f ms", c, ms);
        if (ms < bms) {
            bms = ms;
            best = c;
        }
    }
    ctx->tuned[team_key(probs[0], prec64)] = best;
    if (best_team) *best_team = best;
    if (best_ms) *best_ms = bms;
    return LRA_OK;
}

extern "C" lra_status lra_autotune_batched(lra_ctx* ctx, const lra_block* blocks, int nblocks, const lra_options* opts,
                                           int64_t* best_floor_rows, double* best_ms)
{
    if (!ctx || nblocks < 1 || !blocks) return LRA_EINVAL;
    lra_options o;
    if (opts) o = *opts;
    else lra_default_options(&o);
    if (o.init_cols || o.sample_rows || o.sample_cols) return LRA_EINVAL;
    const int prec64 = o.precision == LRA_PREC_FP64;
    std::vector<Prob> probs(nblocks);
    for (int b = 0; b < nblocks; ++b) {
        const lra_block& bl = blocks[b];
        lra_status rs = make_prob(&bl.src, bl.m, bl.n, bl.k, bl.sweeps, bl.tol, &o, probs[b], b);
        if (rs != LRA_OK) return rs;
        probs[b].team = o.team_wgs > 0 ? std::min(o.team_wgs, NT)
                                       : std::min(NT, pow2_ceil(auto_team(ctx, probs[b], prec64)));
        probs[b].team_fixed = o.team_wgs > 0;
    }
    const int64_t saved = ctx->floor_rows;
    int64_t best = share_floor_rows();
    double bms = 1e300;
    for (int64_t f : {(int64_t)0, (int64_t)2048, (int64_t)4096, (int64_t)8192, (int64_t)16384, (int64_t)32768,
                      (int64_t)65536}) {
        ctx->floor_rows = f;
        double ms = 0.0;
        lra_status rs = time_batch(ctx, probs, prec64, 2, &ms);
        if (rs != LRA_OK) {
            ctx->floor_rows = saved;
            return rs;
        }
        LRA_LOG(1, "autotune floor %lld rows: %.3f ms", (long long)f, ms);
        if (ms < bms) {
            bms = ms;
            best = f;
        }
    }
    ctx->floor_rows = best;
    if (best_floor_rows) *best_floor_rows = best;
    if (best_ms) *best_ms = bms;
    return LRA_OK;
}

extern "C" lra_status lra_tuning_save(lra_ctx* ctx, const char* path)
{
    if (!ctx || !path) return LRA_EINVAL;
    FILE* f = std::fopen(path, "w");
    if (!f) return LRA_EINVAL;
    std::fprintf(f, "# lra tuning: team <precision/rank bucket/size bits> <workgroups>; floor <rows>\n");
    for (auto& kv : ctx->tuned) std::fprintf(f, "team %s %d\n", kv.first.c_str(), kv.second);
    if (ctx->floor_rows >= 0) std::fprintf(f, "floor %lld\n", (long long)ctx->floor_rows);
    std::fclose(f);
    return LRA_OK;
}

extern "C" lra_status lra_tuning_load(lra_ctx* ctx, const char* path)
{
    if (!ctx || !path) return LRA_EINVAL;
    FILE* f = std::fopen(path, "r");
    if (!f) return LRA_EINVAL;
    char line[256];
    lra_status rs = LRA_OK;
    while (std::fgets(line, sizeof(line), f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        char kind[16], key[96];
        long long v = 0;
        if (std::sscanf(line, "team %95s %lld", key, &v) == 2 && v >= 1 && v <= NT) ctx->tuned[key] = (int)v;
        else if (std::sscanf(line, "floor %lld", &v) == 1 && v >= 0) ctx->floor_rows = v;
        else if (std::sscanf(line, "%15s", kind) == 1) rs = LRA_EINVAL;
    }
    std::fclose(f);
    return rs;
}

extern "C" lra_status lra_set_timing(lra_ctx* ctx, int enable, int reset)
{
    if (!ctx) return LRA_EINVAL;
    if (enable && !ctx->ev0) {
        HIP_TRY(hipEventCreate(&ctx->ev0));
        HIP_TRY(hipEventCreate(&ctx->ev1));
    }
    ctx->timing = enable != 0;
    if (reset) ctx->stats = lra_stats{};
    return LRA_OK;
}

extern "C" lra_status lra_get_stats(lra_ctx* ctx, lra_stats* out)
{
    if (!ctx || !out) return LRA_EINVAL;
    *out = ctx->stats;
    out->device_allocs = ctx->dev_allocs;
    out->device_bytes = ctx->dev_in_use;
    return LRA_OK;
}

extern "C" void lra_destroy(lra_ctx* ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    if (Serve* s = ctx->srv) {
        if (s->ev) (void)hipEventDestroy(s->ev);
        if (s->arena.p) (void)hipFree(s->arena.p);
        if (s->ctl_dev.p) (void)hipFree(s->ctl_dev.p);
        if (s->host.p) (void)hipHostFree(s->host.p);
        delete s;
    }
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->dev.p) (void)hipFree(ctx->dev.p);
    if (ctx->host.p) (void)hipHostFree(ctx->host.p);
    delete ctx;
}
