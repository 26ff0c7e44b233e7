// Host-only checks of the runtime's planning and bookkeeping logic, built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_sanitized.py
// (no GPU: the engine's launch helpers are stubbed, nothing is launched).
//
// Covered: the default-draw generator (published SplitMix64 outputs, distinct
// in-range draws), problem validation (make_prob on fuzzed arguments), team
// planning (share_teams / plan_teams: every workgroup in exactly one team,
// every problem queued exactly once, the grid respected), the serving arena's
// first-fit allocator (FreeList against a byte map: no overlap, full
// coalescing), request regions inside their footprint, and the status
// strings.  Exit status 0 when every check holds.
#include "../../paper_1611_01391_amd/csrc/lra_runtime.cpp"

#include <random>
#include <set>

namespace lra {
size_t engine_smem_fixed(int, int) { return 40960; }
const void* engine_kernel_ptr(int, int)
{
    static int sym;
    return &sym;
}
hipError_t launch_engine(int, int, int, size_t, bool, const EngineArgs&, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_zero(void*, int64_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_pack_factors(const void*, const int64_t*, int, double*, double*, hipStream_t)
{
    return hipErrorNoDevice;
}
hipError_t launch_factors(const DevSource&, int64_t, int64_t, int, const int64_t*, const int64_t*, int, void*, void*,
                          hipStream_t)
{
    return hipErrorNoDevice;
}
hipError_t noalloc_scratch_init(int) { return hipErrorNoDevice; }
void* noalloc_scratch(int) { return nullptr; }
size_t core_out_bytes() { return 70000; }
hipError_t topsvd_set_attributes() { return hipErrorNoDevice; }
hipError_t launch_tsqr(const void*, int64_t, int64_t, int, int, double*, const void*, int64_t, int64_t, int, int,
                       double*, int, hipStream_t)
{
    return hipErrorNoDevice;
}
hipError_t launch_topsvd_core(const double*, const double*, const double*, int, int, double, void*, hipStream_t)
{
    return hipErrorNoDevice;
}
hipError_t launch_topsvd_apply(const void*, int64_t, const void*, int64_t, int, int64_t, int64_t, int, const void*,
                               double*, int64_t, double*, int64_t, hipStream_t)
{
    return hipErrorNoDevice;
}
void topsvd_core_fields(const void*, int32_t*, int32_t*, const int32_t**, const int32_t**, const double**,
                        const int64_t**)
{
}
}  // namespace lra

static int failures = 0;
#define CHECK(cond)                                                                 \
    do {                                                                            \
        if (!(cond)) {                                                              \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                             \
        }                                                                           \
    } while (0)

static void check_draws()
{
    // published first outputs of SplitMix64 from state 0
    CHECK(splitmix64(0, 0) == 0xe220a8397b1dcdafull);
    CHECK(splitmix64(0, 1) == 0x6e789e6aa1b965f4ull);
    CHECK(splitmix64(0, 2) == 0x06c45d188009454full);
    std::mt19937_64 g(7);
    for (int t = 0; t < 300; ++t) {
        const int64_t n = 1 + (int64_t)(g() % 5000);
        const int64_t cnt = 1 + (int64_t)(g() % (uint64_t)std::min<int64_t>(n, 300));
        std::vector<int64_t> out(cnt);
        draw_distinct(g(), n, cnt, out.data());
        std::set<int64_t> seen(out.begin(), out.end());
        CHECK((int64_t)seen.size() == cnt);
        CHECK(*seen.begin() >= 0 && *seen.rbegin() < n);
    }
}

static lra_source dense_src(int64_t lda)
{
    static double dummy;
    lra_source s;
    std::memset(&s, 0, sizeof(s));
    s.kind = LRA_SRC_DENSE;
    s.dtype = LRA_F64;
    s.a = &dummy;
    s.lda = lda;
    return s;
}

static void check_make_prob()
{
    std::mt19937_64 g(11);
    int ok = 0;
    for (int t = 0; t < 2000; ++t) {
        const int64_t m = 1 + (int64_t)(g() % 3000), n = 1 + (int64_t)(g() % 3000);
        const int k = (int)(g() % 70) - 2;
        const int sweeps = (int)(g() % 5) - 1;
        const double tol = (g() % 3 == 0) ? 1e-6 : 0.0;
        lra_options o;
        lra_default_options(&o);
        o.k_max = (int)(g() % 80) - 4;
        o.cur_rank = (int)(g() % 20) - 2;
        o.nucleus_rank = (int)(g() % 20) - 2;
        o.seed = g();
        lra_source s = dense_src(n);
        Prob p;
        const lra_status st = make_prob(&s, m, n, k, sweeps, tol, &o, p, (int64_t)(g() % 100));
        if (st != LRA_OK) continue;
        ++ok;
        CHECK(k >= 1 && k <= 64 && k <= m && k <= n && sweeps >= 0);
        CHECK(p.kcap >= p.k && p.kcap <= 64);
        CHECK((int64_t)p.cand.size() >= p.k && (int64_t)p.cand.size() <= n);
        std::set<int64_t> cs(p.cand.begin(), p.cand.end());
        CHECK(cs.size() == p.cand.size() && *cs.rbegin() < n);
        CHECK(p.q >= 1 && p.q <= 64 && p.s >= 1 && p.s <= 64 && (int64_t)p.Q.size() == p.q);
        for (size_t i = 1; i < p.Q.size(); ++i) CHECK(p.Q[i - 1] < p.Q[i]);
        CHECK(p.Q.back() < m && p.S.back() < n);
        if (sweeps == 0) {
            CHECK(p.have_init_I && (int)p.init_I.size() == p.k);
            std::set<int64_t> rs(p.init_I.begin(), p.init_I.end());
            CHECK((int)rs.size() == p.k && *rs.rbegin() < m);
            CHECK(!(tol > 0.0));
        }
        CHECK(p.cur_rank >= 0 && p.cur_rank < p.k + 1 && p.nucleus_rank >= 0 && p.nucleus_rank < p.k + 1);
        CHECK(work_bytes(p) >= 8 * (int64_t)p.kcap * p.kcap);
    }
    CHECK(ok > 100);
    // invalid arguments are rejected
    lra_options o;
    lra_default_options(&o);
    lra_source s = dense_src(100);
    Prob p;
    CHECK(make_prob(&s, 100, 100, 0, 1, 0.0, &o, p, 0) == LRA_EINVAL);
    CHECK(make_prob(&s, 100, 100, 65, 1, 0.0, &o, p, 0) == LRA_EINVAL);
    CHECK(make_prob(&s, 100, 100, 8, 0, 1e-6, &o, p, 0) == LRA_EINVAL);
    CHECK(make_prob(&s, 100, 150, 8, 1, 0.0, &o, p, 0) == LRA_EINVAL);  // lda < n
    o.cur_rank = 9;
    CHECK(make_prob(&s, 100, 100, 8, 1, 0.0, &o, p, 0) == LRA_EINVAL);
    // the pre-processed source: depth 1..8, 2^depth dividing both dimensions
    lra_default_options(&o);
    lra_source h = dense_src(128);
    h.kind = LRA_SRC_PREPROCESSED;
    h.pre_seed = 0x123456789abcdefull;
    for (int d = 0; d <= 9; ++d) {
        h.pre_depth = d;
        const lra_status want = (d >= 1 && d <= 7) ? LRA_OK : LRA_EINVAL;  // 2^8 does not divide 128
        CHECK(make_prob(&h, 256, 128, 8, 1, 0.0, &o, p, 0) == want);
        if (want == LRA_OK) {
            CHECK(p.src.kind == 3 && p.src.depth == d && p.src.seed == h.pre_seed);
            CHECK(p.src.pm == 256 && p.src.pn == 128 && p.src.lda == 128);
        }
    }
    h.pre_depth = 3;
    CHECK(make_prob(&h, 100, 128, 8, 1, 0.0, &o, p, 0) == LRA_EINVAL);  // 8 does not divide 100
    CHECK(make_prob(&h, 256, 129, 8, 1, 0.0, &o, p, 0) == LRA_EINVAL);  // lda < n
}

static void check_planning()
{
    std::mt19937_64 g(5);
    for (int t = 0; t < 300; ++t) {
        const int np = 1 + (int)(g() % 200);
        const int max_wgs = 1 + (int)(g() % 512);
        std::vector<Prob> probs(np);
        std::vector<Prob*> pp;
        for (auto& p : probs) {
            p.m = 1 + (int64_t)(g() % 300000);
            p.n = 1 + (int64_t)(g() % 300000);
            p.k = 1 + (int)(g() % 64);
            p.kcap = p.k;
            p.sweeps = 1 + (int)(g() % 4);
            p.team = std::min(max_wgs, 1 << (int)(g() % 7));
            pp.push_back(&p);
        }
        share_teams(pp, max_wgs, (g() % 2) ? 8192 : 0);
        // the size classes take at most half the grid together (as plan_launch ensures)
        for (;;) {
            std::set<int> sizes;
            for (auto* p : pp) sizes.insert(p->team);
            int64_t sum = 0;
            for (int sz : sizes) sum += sz;
            if (sum <= std::max(1, max_wgs / 2) || sizes.size() == 1) break;
            const int big = *sizes.rbegin();
            for (auto* p : pp)
                if (p->team == big) p->team = std::max(1, big / 2);
        }
        for (auto* p : pp) CHECK(p->team >= 1 && p->team <= max_wgs);
        const Plan pl = plan_teams(pp, max_wgs);
        CHECK((int)pl.wg_team.size() <= std::max(max_wgs, pl.max_team));
        int wg = 0;
        for (size_t ti = 0; ti < pl.teams.size(); ++ti) {
            const TeamInfo& tinfo = pl.teams[ti];
            CHECK(tinfo.first_wg == wg && tinfo.size >= 1);
            for (int w = 0; w < tinfo.size; ++w) CHECK(pl.wg_team[wg + w] == (int32_t)ti);
            CHECK(tinfo.queue >= 0 && tinfo.queue < (int)pl.queues.size());
            wg += tinfo.size;
        }
        CHECK(wg == (int)pl.wg_team.size());
        std::vector<int> seen(np, 0);
        for (auto& q : pl.queues)
            for (int32_t i : q) {
                CHECK(i >= 0 && i < np);
                if (i >= 0 && i < np) seen[i]++;
            }
        for (int i = 0; i < np; ++i) CHECK(seen[i] == 1);
    }
}

static void check_freelist()
{
    std::mt19937_64 g(3);
    const int64_t size = 1 << 16;
    FreeList fl;
    fl.reset(size);
    std::vector<uint8_t> used(size, 0);
    std::vector<std::pair<int64_t, int64_t>> live;
    for (int t = 0; t < 20000; ++t) {
        if (!live.empty() && (g() % 2)) {
            const size_t i = g() % live.size();
            fl.release(live[i].first, live[i].second);
            for (int64_t b = 0; b < live[i].second; ++b) used[live[i].first + b] = 0;
            live.erase(live.begin() + (long)i);
        } else {
            const int64_t bytes = 1 + (int64_t)(g() % 3000);
            const int64_t off = fl.alloc(bytes);
            if (off < 0) continue;
            CHECK(off + bytes <= size);
            for (int64_t b = 0; b < bytes && off + b < size; ++b) {
                CHECK(!used[off + b]);
                used[off + b] = 1;
            }
            live.push_back({off, bytes});
        }
    }
    for (auto& l : live) fl.release(l.first, l.second);
    CHECK(fl.free.size() == 1 && fl.free.begin()->first == 0 && fl.free.begin()->second == size);
}

static void check_regions()
{
    std::mt19937_64 g(9);
    for (int t = 0; t < 500; ++t) {
        lra_options o;
        lra_default_options(&o);
        o.k_max = (int)(g() % 65);
        const int64_t m = 64 + (int64_t)(g() % 100000), n = 64 + (int64_t)(g() % 100000);
        const int k = 1 + (int)(g() % 64);
        lra_source s = dense_src(n);
        Prob p;
        if (make_prob(&s, m, n, k, 2, 0.0, &o, p, 0) != LRA_OK) continue;
        const int prec64 = (int)(g() % 2);
        const int64_t base = (int64_t)(g() % 4096) * 256;
        const int64_t fp = request_footprint(p, prec64);
        const ProbRegions r = request_regions(p, prec64, base);
        const int64_t ends[] = {r.Q, r.S, r.I, r.J, r.G, r.U, r.prevI, r.prevJ, r.work, r.strip};
        int64_t prev = r.cand;
        CHECK(r.cand >= base);
        for (int64_t e : ends) {
            CHECK(e >= prev);
            prev = e;
        }
        CHECK(r.strip + strip_bytes(p, prec64) <= base + fp);
    }
}

int main()
{
    check_draws();
    check_make_prob();
    check_planning();
    check_freelist();
    check_regions();
    for (int s = -7; s <= 4; ++s) CHECK(lra_status_str((lra_status)s) != nullptr);
    if (failures) std::fprintf(stderr, "%d checks failed\n", failures);
    else std::printf("runtime host checks: all passed\n");
    return failures ? 1 : 0;
}
