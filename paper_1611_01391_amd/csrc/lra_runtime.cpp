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
#include <string>
#include <vector>

#include "../../include/lra.h"
#include "lra_internal.h"

namespace lra {
size_t engine_smem_fixed(int prec64, int kmax);
const void* engine_kernel_ptr(int prec64, int kmax);
hipError_t launch_engine(int prec64, int kmax, int grid, size_t smem, bool cooperative,
                         const EngineArgs& ea, hipStream_t stream);
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t stream);
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

// cnt distinct indices in [0, n) in draw order (floor(v n / 2^64), repeats skipped).
void draw_distinct(uint64_t seed, int64_t n, int64_t cnt, int64_t* out)
{
    std::vector<int64_t> seen;
    int64_t got = 0;
    for (uint64_t ctr = 0; got < cnt; ++ctr) {
        const uint64_t v = splitmix64(seed, ctr);
        const int64_t idx = (int64_t)(((unsigned __int128)v * (unsigned __int128)(uint64_t)n) >> 64);
        bool dup = false;
        for (int64_t e = 0; e < got; ++e)
            if (out[e] == idx) { dup = true; break; }
        if (!dup) out[got++] = idx;
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

struct Request;

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
    int64_t dev_in_use = 0;  // bytes held by the serving slots
    std::map<std::string, int> tuned;  // autotuned team sizes
    bool timing = false;
    bool trace = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    lra_stats stats{};
    // serving
    uint64_t next_ticket = 1;
    std::deque<Request*> pending;
    std::vector<Request*> active;
    std::map<uint64_t, std::unique_ptr<Request>> all;
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

static lra_status ensure(Buffer& b, int64_t bytes, bool pinned, lra_ctx* ctx)
{
    if (b.bytes >= bytes) return LRA_OK;
    if (!pinned && ctx->budget && (size_t)(bytes + ctx->dev_in_use) > ctx->budget) return LRA_EBUDGET;
    if (b.p) {
        if (pinned) (void)hipHostFree(b.p);
        else (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    int64_t want = std::max<int64_t>(bytes, 1 << 20);
    want = align_up(want + want / 4, 1 << 20);
    hipError_t e = pinned ? hipHostMalloc(&b.p, (size_t)want, hipHostMallocDefault) : hipMalloc(&b.p, (size_t)want);
    if (e != hipSuccess) {
        b.p = nullptr;
        LRA_LOG(1, "allocation of %lld bytes failed: %s", (long long)want, hipGetErrorString(e));
        return LRA_ENOMEM;
    }
    b.bytes = want;
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
    if (const char* t = std::getenv("LRA_TRACE")) c->trace = std::atoi(t) != 0;
    // LDS for strip rows: all the device leaves per workgroup after the fixed
    // part of each kernel variant (LRA_LDS_B_BYTES caps it)
    c->lds_cap = std::min(c->max_lds, 160 * 1024);
    if (const char* t = std::getenv("LRA_LDS_B_BYTES")) c->lds_b_bytes = std::atoi(t);
    for (int p = 0; p < 2; ++p)
        for (int km : {8, 16, 32, 64})
            (void)hipFuncSetAttribute(engine_kernel_ptr(p, km), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      c->lds_cap);
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
    if (s->kind == LRA_SRC_CAUCHY || s->kind == LRA_SRC_INVDIST) return s->x && s->y;
    return false;
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
    bool need_strip = false;
    void* C_out = nullptr;
    void* R_out = nullptr;
    bool have_init_I = false;
    std::vector<int64_t> init_I;
};

static lra_status make_prob(const lra_source* src, int64_t m, int64_t n, int k, int sweeps, double tol,
                            const lra_options* o, Prob& p, int64_t blk_index)
{
    if (!src_ok(src) || m < 1 || n < 1 || k < 1 || k > 64 || k > m || k > n || sweeps < 1) return LRA_EINVAL;
    if (!(o->tau >= 0.0) || o->k_step < 1 || o->k_max > 64) return LRA_EINVAL;
    if (src->kind == LRA_SRC_DENSE && src->lda < (src->col_major ? m : n)) return LRA_EINVAL;
    if (o->precision != LRA_PREC_FP64 && o->precision != LRA_PREC_MIXED) return LRA_EINVAL;
    p.src.kind = src->kind;
    p.src.dtype = src->dtype;
    p.src.a = src->a;
    p.src.lda = src->lda;
    p.src.col_major = src->col_major ? 1 : 0;
    p.src.pad = 0;
    p.src.x = src->x;
    p.src.y = src->y;
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

// Workgroups per problem: enough that each workgroup's rows fit its LDS,
// within the co-resident limit; an explicit or tuned choice overrides.
static int auto_team(lra_ctx* ctx, const Prob& p, int prec64)
{
    const int esz = prec64 ? 8 : 4;
    const int64_t M = std::max(p.m, p.n);
    char key[96];
    std::snprintf(key, sizeof(key), "%d/%d/%lld", prec64, kmax_bucket(p.kcap),
                  (long long)(64 - __builtin_clzll((unsigned long long)M)));
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) return it->second;
    int64_t rows_fit = strip_lds(ctx, prec64, kmax_bucket(p.kcap)) / ((int64_t)p.kcap * esz);
    // at most one row per thread keeps the swap loop register-resident
    rows_fit = std::max<int64_t>(64, std::min<int64_t>(rows_fit, NT));
    int64_t t = (M + rows_fit - 1) / rows_fit;
    t = std::min<int64_t>(t, std::min(ctx->num_cu, NT));
    return (int)std::max<int64_t>(1, t);
}

static void fill_task(TaskDesc& td, const Prob& p, uint8_t* dbase, const int64_t* offs)
{
    // offs: cand, Q, S, I, J, prevI, prevJ, G, U, work, strip, state
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
    td.cand = (const int64_t*)(dbase + offs[0]);
    td.n_cand = (int64_t)p.cand.size();
    td.Q = (const int64_t*)(dbase + offs[1]);
    td.S = (const int64_t*)(dbase + offs[2]);
    td.I = (int64_t*)(dbase + offs[3]);
    td.J = (int64_t*)(dbase + offs[4]);
    td.prevI = (int64_t*)(dbase + offs[5]);
    td.prevJ = (int64_t*)(dbase + offs[6]);
    td.G = (double*)(dbase + offs[7]);
    td.U = (double*)(dbase + offs[8]);
    td.work = (double*)(dbase + offs[9]);
    td.strip = offs[10] >= 0 ? (void*)(dbase + offs[10]) : nullptr;
    td.C_out = p.C_out;
    td.R_out = p.R_out;
    td.st = (TaskState*)(dbase + offs[11]);
}

// Offsets of one problem's device regions inside a layout.
struct ProbRegions {
    int64_t off[12];
};

static ProbRegions lay_prob(Layout& L, const Prob& p, int prec64)
{
    ProbRegions r;
    const int64_t kc = p.kcap;
    r.off[0] = L.add(8 * (int64_t)p.cand.size());
    r.off[1] = L.add(8 * (int64_t)p.q);
    r.off[2] = L.add(8 * (int64_t)p.s);
    r.off[3] = L.add(8 * kc);
    r.off[4] = L.add(8 * kc);
    r.off[5] = L.add(8 * kc);
    r.off[6] = L.add(8 * kc);
    r.off[7] = L.add(8 * kc * kc);
    r.off[8] = L.add(8 * kc * kc);
    {
        // final phase scratch: [G | I | A[I,S]] (row stride 2 KMAX + 64) and the sample blocks
        const int64_t kb = kmax_bucket(p.kcap);
        r.off[9] = L.add(8 * (kb * (2 * kb + 64) + (int64_t)p.q * kc + (int64_t)p.q * p.s));
    }
    r.off[10] = p.need_strip ? L.add(std::max(p.m, p.n) * kc * (prec64 ? 8 : 4)) : -1;
    r.off[11] = L.add(sizeof(TaskState));
    return r;
}

static void init_host_image(uint8_t* h, const Prob& p, const ProbRegions& r)
{
    std::memcpy(h + r.off[0], p.cand.data(), 8 * p.cand.size());
    std::memcpy(h + r.off[1], p.Q.data(), 8 * (size_t)p.q);
    std::memcpy(h + r.off[2], p.S.data(), 8 * (size_t)p.s);
    int64_t* I = (int64_t*)(h + r.off[3]);
    int64_t* J = (int64_t*)(h + r.off[4]);
    int64_t* pI = (int64_t*)(h + r.off[5]);
    int64_t* pJ = (int64_t*)(h + r.off[6]);
    for (int c = 0; c < p.kcap; ++c) {
        I[c] = (p.have_init_I && c < p.k) ? p.init_I[c] : 0;
        J[c] = c < p.k ? p.cand[c] : 0;
        pI[c] = 0;
        pJ[c] = 0;
    }
    TaskState* st = (TaskState*)(h + r.off[11]);
    std::memset(st, 0, sizeof(*st));
    st->phase = PH_COL;
    st->k = p.k;
    st->have_I = p.have_init_I ? 1 : 0;
    st->cand_next = p.k;
}

// ----------------------------------------------------------------------------
// running a set of problems in one launch
// ----------------------------------------------------------------------------

struct Plan {
    std::vector<TeamInfo> teams;
    std::vector<int32_t> wg_team;
    std::vector<std::vector<int32_t>> queues;
    int max_team = 1;
};

// Teams by size class: each class gets teams in proportion to its work,
// problems in a class are pulled largest first.
static Plan plan_teams(lra_ctx* ctx, const std::vector<Prob>& probs, int max_wgs)
{
    Plan pl;
    std::map<int, std::vector<int32_t>> cls;
    for (int i = 0; i < (int)probs.size(); ++i) cls[probs[i].team].push_back(i);
    double total = 0.0;
    std::map<int, double> cost;
    for (auto& kv : cls) {
        double c = 0.0;
        for (int i : kv.second) c += (double)(probs[i].m + probs[i].n) * probs[i].kcap * probs[i].sweeps;
        cost[kv.first] = c;
        total += c;
    }
    int used = 0;
    int qi = 0;
    for (auto& kv : cls) {
        const int tsz = kv.first;
        auto items = kv.second;
        std::stable_sort(items.begin(), items.end(), [&](int a, int b) {
            return (probs[a].m + probs[a].n) * (int64_t)probs[a].kcap > (probs[b].m + probs[b].n) * (int64_t)probs[b].kcap;
        });
        int want = (int)std::floor((double)max_wgs * cost[kv.first] / std::max(total, 1.0) / tsz);
        want = std::max(1, std::min<int>(want, (int)items.size()));
        const int room = std::max(0, max_wgs - used) / tsz;
        int nteam = std::max(1, std::min(want, room));
        for (int t = 0; t < nteam; ++t) {
            TeamInfo ti;
            ti.first_wg = used;
            ti.size = tsz;
            ti.queue = qi;
            ti.pad = 0;
            pl.teams.push_back(ti);
            for (int w = 0; w < tsz; ++w) pl.wg_team.push_back((int32_t)pl.teams.size() - 1);
            used += tsz;
        }
        pl.queues.push_back(items);
        pl.max_team = std::max(pl.max_team, tsz);
        ++qi;
    }
    return pl;
}

// Summarise a device trace on stderr: time spent before each event kind,
// measured from the previous event of the same team leader.
static void dump_trace(lra_ctx* ctx, const uint64_t* tr, int cap)
{
    static const char* names[] = {"?", "step_begin", "warm_lu", "gathered", "basis", "swap_g",
                                  "step_end", "final_begin", "final_end", "task_begin", "task_end",
                                  "pivot", "swap_upd+red", "swap_xchg"};
    const uint64_t n = std::min<uint64_t>(tr[0], (uint64_t)cap);
    double tot[14] = {0};
    int64_t cnt[14] = {0};
    const double us_per_tick = 1000.0 / (double)ctx->wall_rate_khz;
    for (uint64_t i = 1; i < n; ++i) {
        const int ev = (int)(tr[1 + 2 * i] >> 56);
        const double dt = (double)(tr[2 + 2 * i] - tr[2 + 2 * (i - 1)]) * us_per_tick;
        if (ev > 0 && ev < 14) { tot[ev] += dt; cnt[ev] += 1; }
    }
    std::fprintf(stderr, "[lra trace] %llu events\n", (unsigned long long)n);
    for (int e = 1; e < 14; ++e)
        if (cnt[e])
            std::fprintf(stderr, "[lra trace] %-12s n=%6lld total %9.1f us  mean %7.2f us\n", names[e],
                         (long long)cnt[e], tot[e], tot[e] / (double)cnt[e]);
}

// Device workspace + upload + launch + download for a set of problems that
// share precision and KMAX.  st_out / ij_out receive per-problem results.
struct RunOut {
    TaskState st;
    std::vector<int64_t> I, J;
    std::vector<double> G, U;
};

static lra_status run_problems(lra_ctx* ctx, std::vector<Prob>& probs, int prec64, int phase_budget,
                               std::vector<RunOut>& outs)
{
    if (probs.empty()) return LRA_OK;
    int kcap_all = 1;
    for (auto& p : probs) kcap_all = std::max(kcap_all, p.kcap);
    const int kmx = kmax_bucket(kcap_all);
    const int lds_b = strip_lds(ctx, prec64, kmx);
    const size_t smem = engine_smem_fixed(prec64, kmx) + (size_t)lds_b;
    int occ = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, engine_kernel_ptr(prec64, kmx), NT, smem));
    if (occ < 1) return LRA_EDEVICE;
    const int max_wgs = occ * ctx->num_cu;
    for (auto& p : probs) {
        p.team = std::min(p.team, max_wgs);
        const int esz = prec64 ? 8 : 4;
        const int64_t R = (std::max(p.m, p.n) + p.team - 1) / p.team;
        p.need_strip = R * p.kcap * esz > lds_b;
    }
    Plan pl = plan_teams(ctx, probs, max_wgs);
    const int grid = (int)pl.wg_team.size();
    const bool coop = pl.max_team > 1;

    // layout: [upload: tasks | per-problem regions | queues | teams | wg_team]
    //         [zeroed: team ctl | queue heads | error flag]
    Layout L;
    const int64_t off_tasks = L.add(sizeof(TaskDesc) * probs.size());
    std::vector<ProbRegions> regs;
    regs.reserve(probs.size());
    for (auto& p : probs) regs.push_back(lay_prob(L, p, prec64));
    int64_t nitems = 0;
    for (auto& q : pl.queues) nitems += (int64_t)q.size();
    const int nq = (int)pl.queues.size();
    const int64_t off_items = L.add(4 * std::max<int64_t>(1, nitems));
    const int64_t off_qoff = L.add(4 * nq);
    const int64_t off_qlen = L.add(4 * nq);
    const int64_t off_teams = L.add(sizeof(TeamInfo) * pl.teams.size());
    const int64_t off_wgteam = L.add(4 * (int64_t)grid);
    const int64_t upload_end = L.size;
    const int64_t ctl_stride = align_up(team_ctl_bytes(pl.max_team), 256);
    const int64_t off_ctl = L.add(ctl_stride * (int64_t)pl.teams.size());
    const int64_t off_qhead = L.add(4 * nq);
    const int64_t off_err = L.add(4);
    const int trace_cap = ctx->trace ? 1 << 16 : 0;
    const int64_t off_trace = L.add(8 * (1 + 2 * (int64_t)trace_cap));
    const int64_t total = L.size;

    lra_status rs = ensure(ctx->dev, total, false, ctx);
    if (rs != LRA_OK) return rs;
    rs = ensure(ctx->host, total, true, ctx);
    if (rs != LRA_OK) return rs;
    uint8_t* h = (uint8_t*)ctx->host.p;
    uint8_t* d = (uint8_t*)ctx->dev.p;

    TaskDesc* htasks = (TaskDesc*)(h + off_tasks);
    for (size_t i = 0; i < probs.size(); ++i) {
        init_host_image(h, probs[i], regs[i]);
        fill_task(htasks[i], probs[i], d, regs[i].off);
    }
    int32_t* items = (int32_t*)(h + off_items);
    int32_t* qoff = (int32_t*)(h + off_qoff);
    int32_t* qlen = (int32_t*)(h + off_qlen);
    int64_t pos = 0;
    for (int q = 0; q < nq; ++q) {
        qoff[q] = (int32_t)pos;
        qlen[q] = (int32_t)pl.queues[q].size();
        for (int32_t t : pl.queues[q]) items[pos++] = t;
    }
    std::memcpy(h + off_teams, pl.teams.data(), sizeof(TeamInfo) * pl.teams.size());
    std::memcpy(h + off_wgteam, pl.wg_team.data(), 4 * (size_t)grid);

    HIP_TRY(hipMemcpyAsync(d, h, (size_t)upload_end, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(launch_zero(d + off_ctl, total - off_ctl, ctx->stream));

    EngineArgs ea;
    ea.tasks = (TaskDesc*)(d + off_tasks);
    ea.queue_items = (const int32_t*)(d + off_items);
    ea.queue_off = (const int32_t*)(d + off_qoff);
    ea.queue_len = (const int32_t*)(d + off_qlen);
    ea.queue_head = (uint32_t*)(d + off_qhead);
    ea.teams = (const TeamInfo*)(d + off_teams);
    ea.wg_team = (const int32_t*)(d + off_wgteam);
    ea.team_ctl = d + off_ctl;
    ea.team_ctl_stride = ctl_stride;
    ea.phase_budget = phase_budget;
    ea.lds_b_bytes = lds_b;
    ea.error_flag = (uint32_t*)(d + off_err);
    ea.timeout_ticks = (int64_t)(ctx->timeout_s * (double)ctx->wall_rate_khz * 1000.0);
    ea.trace = trace_cap ? (uint64_t*)(d + off_trace) : nullptr;
    ea.trace_cap = trace_cap;
    ea.pad2 = 0;
    LRA_LOG(2, "launch: %zu problems, grid %d, teams %zu (max %d), smem %zu, coop %d", probs.size(), grid,
            pl.teams.size(), pl.max_team, smem, (int)coop);
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev0, ctx->stream));
    HIP_TRY(launch_engine(prec64, kmx, grid, smem, coop, ea, ctx->stream));
    if (ctx->timing) HIP_TRY(hipEventRecord(ctx->ev1, ctx->stream));
    ctx->stats.launches += 1;
    ctx->stats.last_grid = grid;
    ctx->stats.last_teams = (int32_t)pl.teams.size();

    // download: states, index sets, G, U, error flag
    for (size_t i = 0; i < probs.size(); ++i) {
        const auto& r = regs[i];
        const int64_t kc = probs[i].kcap;
        HIP_TRY(hipMemcpyAsync(h + r.off[11], d + r.off[11], sizeof(TaskState), hipMemcpyDeviceToHost, ctx->stream));
        for (int j = 3; j <= 4; ++j)
            HIP_TRY(hipMemcpyAsync(h + r.off[j], d + r.off[j], 8 * kc, hipMemcpyDeviceToHost, ctx->stream));
        for (int j = 7; j <= 8; ++j)
            HIP_TRY(hipMemcpyAsync(h + r.off[j], d + r.off[j], 8 * kc * kc, hipMemcpyDeviceToHost, ctx->stream));
    }
    HIP_TRY(hipMemcpyAsync(h + off_err, d + off_err, 4, hipMemcpyDeviceToHost, ctx->stream));
    if (trace_cap)
        HIP_TRY(hipMemcpyAsync(h + off_trace, d + off_trace, 8 * (1 + 2 * (int64_t)trace_cap),
                               hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (trace_cap) dump_trace(ctx, (const uint64_t*)(h + off_trace), trace_cap);
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
    outs.resize(probs.size());
    for (size_t i = 0; i < probs.size(); ++i) {
        const auto& r = regs[i];
        RunOut& o = outs[i];
        o.st = *(TaskState*)(h + r.off[11]);
        const int k = o.st.k;
        o.I.assign((int64_t*)(h + r.off[3]), (int64_t*)(h + r.off[3]) + k);
        o.J.assign((int64_t*)(h + r.off[4]), (int64_t*)(h + r.off[4]) + k);
        o.G.assign((double*)(h + r.off[7]), (double*)(h + r.off[7]) + (int64_t)k * k);
        o.U.assign((double*)(h + r.off[8]), (double*)(h + r.off[8]) + (int64_t)k * k);
    }
    return LRA_OK;
}

static lra_status status_of(const TaskState& st)
{
    if (st.status < 0) return (lra_status)st.status;
    if (st.warn & W_TOL) return LRA_TOL_NOT_MET;
    if (st.warn & W_NUMRANK) return LRA_NUMERICAL_RANK;
    if (st.warn & W_CAP) return LRA_MAXVOL_CAP;
    return LRA_OK;
}

static void deliver(const RunOut& o, lra_result* res)
{
    res->k = o.st.k;
    res->status = (int32_t)status_of(o.st);
    res->sweeps_done = o.st.sweeps_done;
    res->swaps_total = o.st.swaps_total;
    res->entries_read = o.st.entries_read;
    res->err_est_rel = o.st.est_rel;
    res->err_est_abs = o.st.est_abs;
    res->err_mean = o.st.mean;
    res->err_var = o.st.var;
    res->nucleus_cond1 = o.st.cond1;
    if (res->I) std::memcpy(res->I, o.I.data(), 8 * o.I.size());
    if (res->J) std::memcpy(res->J, o.J.data(), 8 * o.J.size());
    if (res->G) std::memcpy(res->G, o.G.data(), 8 * o.G.size());
    if (res->U) std::memcpy(res->U, o.U.data(), 8 * o.U.size());
}

static int severity(lra_status s)
{
    if (s < 0) return 100 - (int)s;
    return (int)s;
}

// ----------------------------------------------------------------------------
// public entry points
// ----------------------------------------------------------------------------

extern "C" lra_status lra_ca_cur(lra_ctx* ctx, const lra_source* src, int64_t m, int64_t n, int k, int sweeps,
                                 double tol, const lra_options* opts, lra_result* result)
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
    std::vector<RunOut> outs;
    rs = run_problems(ctx, probs, prec64, 1 << 30, outs);
    if (rs != LRA_OK) return rs;
    deliver(outs[0], result);
    return (lra_status)result->status;
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
    std::vector<RunOut> outs;
    rs = run_problems(ctx, probs, prec64, 1, outs);
    if (rs != LRA_OK) return rs;
    const TaskState& st = outs[0].st;
    if (st.status < 0) return (lra_status)st.status;
    for (int c = 0; c < st.k; ++c) I[c] = outs[0].I[c];
    if (swaps) *swaps = st.swaps_total;
    if (k_eff) *k_eff = st.k;
    return status_of(st);
}

extern "C" lra_status lra_ca_cur_batched(lra_ctx* ctx, const lra_block* blocks, int nblocks, const lra_options* opts,
                                         lra_result* results)
{
    if (!ctx || nblocks < 0 || (nblocks > 0 && (!blocks || !results))) return LRA_EINVAL;
    if (nblocks == 0) return LRA_OK;
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
        probs[b].team = o.team_wgs > 0 ? std::min(o.team_wgs, NT) : auto_team(ctx, probs[b], prec64);
        probs[b].C_out = results[b].C_out;
        probs[b].R_out = results[b].R_out;
    }
    std::vector<RunOut> outs;
    lra_status rs = run_problems(ctx, probs, prec64, 1 << 30, outs);
    if (rs != LRA_OK) return rs;
    lra_status worst = LRA_OK;
    for (int b = 0; b < nblocks; ++b) {
        deliver(outs[b], &results[b]);
        if (severity((lra_status)results[b].status) > severity(worst)) worst = (lra_status)results[b].status;
    }
    return worst;
}

// ----------------------------------------------------------------------------
// serving (continuous batching) -- filled in by lra_serve.cpp
// ----------------------------------------------------------------------------

struct Request {
    uint64_t ticket;
    lra_request req;
    lra_result* res;
    lra_status status = LRA_PENDING;
};

extern "C" lra_status lra_submit(lra_ctx* ctx, const lra_request* req, uint64_t* ticket)
{
    (void)ctx; (void)req; (void)ticket;
    return LRA_EINVAL;
}

extern "C" lra_status lra_poll(lra_ctx* ctx, uint64_t ticket)
{
    (void)ctx; (void)ticket;
    return LRA_EINVAL;
}

extern "C" lra_status lra_wait(lra_ctx* ctx, uint64_t ticket)
{
    (void)ctx; (void)ticket;
    return LRA_EINVAL;
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
    return LRA_OK;
}

extern "C" void lra_destroy(lra_ctx* ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->dev.p) (void)hipFree(ctx->dev.p);
    if (ctx->host.p) (void)hipHostFree(ctx->host.p);
    delete ctx;
}
