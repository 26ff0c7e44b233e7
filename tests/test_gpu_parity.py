"""GPU parity: the gfx950 library against the CPU oracle on the same seeded
inputs, through the C ABI.

Bar: index sets identical whenever the oracle's recorded decision margins
(LU pivot gaps, swap argmax gaps, stop-test and rank-threshold margins) are
clear of the arithmetic's rounding, gamma = 1e-9 on the binary64 path and
1e-3 on the binary32-selection path; otherwise only the errors are compared
and the GPU result is checked for validity (maxvol invariant).  Sampled
relative error within 1e-10 of the oracle's on the binary64 path; gathered
factors bit-exact.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GAMMA64 = 1e-9
GAMMA32 = 1e-3


@pytest.fixture(scope="module")
def ctx():
    os.environ.setdefault("LRA_TIMEOUT_S", "20")
    from paper_1611_01391_amd import lra
    c = lra.Context()
    yield c
    c.close()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _lra():
    from paper_1611_01391_amd import lra
    return lra


def _check_same(res, ref, gamma, what):
    assert res.status == ref.status, (what, res.status, ref.status)
    assert res.k == ref.k, (what, res.k, ref.k)
    if ref.min_gap() >= gamma:
        np.testing.assert_array_equal(res.I, ref.I, err_msg=what)
        np.testing.assert_array_equal(res.J, ref.J, err_msg=what)
        return True
    return False


def _true_rel_err(A, I, J):
    G = A[np.ix_(I, J)]
    E = A - A[:, J] @ np.linalg.solve(G, A[I, :])
    return np.linalg.norm(E) / np.linalg.norm(A)


# ---------------------------------------------------------------------------
# plain binary64 path, 512 x 512, k = 8, 3 sweeps
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_plain_fp64_512(ctx, seed):
    lra = _lra()
    _say(f"plain fp64 512 seed {seed}")
    A, d = synth.plain_fp64(seed)
    ref = oracle.ca_cur(oracle.dense(A), 8, 3, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    At = torch.from_numpy(A).cuda()
    res = ctx.ca_cur(lra.dense(At), 8, 3, 0.0, init_cols=d.cand_cols, sample_rows=d.sample_rows,
                     sample_cols=d.sample_cols, factors=True)
    torch.cuda.synchronize()
    same = _check_same(res, ref, GAMMA64, f"seed {seed}")
    assert abs(res.err_est_rel - ref.err_est_rel) <= 1e-10
    if same:
        assert abs(res.err_est_rel - ref.err_est_rel) <= 1e-9 * ref.err_est_rel + 1e-15
        np.testing.assert_allclose(res.U, ref.U, rtol=1e-9, atol=1e-9 * np.abs(ref.U).max())
        np.testing.assert_array_equal(res.G, ref.G)
    e_gpu = _true_rel_err(A, res.I, res.J)
    e_ref = _true_rel_err(A, ref.I, ref.J)
    assert abs(e_gpu - e_ref) <= 1e-10
    # gathered factors are exact copies
    np.testing.assert_array_equal(res.C.cpu().numpy(), A[:, res.J])
    np.testing.assert_array_equal(res.R.cpu().numpy(), A[res.I, :])
    assert res.sweeps_done == 3


@pytest.mark.parametrize("team", [1, 2, 3, 8])
@pytest.mark.parametrize("shape", [(1000, 777, 5), (777, 1000, 12), (300, 2049, 16)])
def test_teams_ragged(ctx, team, shape):
    """Several workgroups per problem (team barrier path) on ragged shapes."""
    lra = _lra()
    m, n, k = shape
    _say(f"teams ragged {shape} team {team}")
    A, d = synth.rect_factor_gaussian(7 + k, m, n, k, 1e-6, k)
    ref = oracle.ca_cur(oracle.dense(A), k, 2, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    res = ctx.ca_cur(lra.dense(torch.from_numpy(A).cuda()), k, 2, 0.0, init_cols=d.cand_cols,
                     sample_rows=d.sample_rows, sample_cols=d.sample_cols, team_wgs=team)
    _check_same(res, ref, GAMMA64, f"{shape} team {team}")
    assert abs(res.err_est_rel - ref.err_est_rel) <= 1e-10


def test_col_major_and_fp32_dense(ctx):
    lra = _lra()
    _say("col-major fp64 and fp32 dense")
    A, d = synth.plain_fp64(3)
    ref = oracle.ca_cur(oracle.dense(A), 8, 3, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    Acm = torch.from_numpy(np.asfortranarray(A)).cuda()
    Acm = torch.as_strided(torch.from_numpy(A.T.copy()).cuda(), (512, 512), (1, 512))
    res = ctx.ca_cur(lra.dense(Acm, col_major=True), 8, 3, 0.0, init_cols=d.cand_cols,
                     sample_rows=d.sample_rows, sample_cols=d.sample_cols)
    _check_same(res, ref, GAMMA64, "col-major")
    A32 = A.astype(np.float32)
    ref32 = oracle.ca_cur(oracle.dense(A32), 8, 3, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    res32 = ctx.ca_cur(lra.dense(torch.from_numpy(A32).cuda()), 8, 3, 0.0, init_cols=d.cand_cols,
                       sample_rows=d.sample_rows, sample_cols=d.sample_cols)
    _check_same(res32, ref32, GAMMA64, "fp32 entries, fp64 path")
    assert abs(res32.err_est_rel - ref32.err_est_rel) <= 1e-10


# ---------------------------------------------------------------------------
# mixed path (binary32 strips / basis / selection), generated sources
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_mixed_dense(ctx, seed):
    lra = _lra()
    _say(f"mixed dense seed {seed}")
    A, d = synth.rect_factor_gaussian(seed, 1500, 1200, 16, 1e-4, 16)
    A32 = A.astype(np.float32)
    ref = oracle.ca_cur(oracle.dense(A32), 16, 3, 0.0, d.cand_cols, d.sample_rows, d.sample_cols,
                        precision="f32")
    ref64 = oracle.ca_cur(oracle.dense(A32), 16, 3, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    res = ctx.ca_cur(lra.dense(torch.from_numpy(A32).cuda()), 16, 3, 0.0, init_cols=d.cand_cols,
                     sample_rows=d.sample_rows, sample_cols=d.sample_cols,
                     precision=lra.PREC_MIXED)
    same = _check_same(res, ref, GAMMA32, f"mixed seed {seed}")
    if same:
        # same index sets: nucleus and residual are binary64 on both sides
        assert abs(res.err_est_rel - ref.err_est_rel) <= 1e-9 * ref.err_est_rel + 1e-15
    # the mixed path's error stays within a small factor of the binary64 path's
    assert res.err_est_rel <= 3.0 * ref64.err_est_rel + 1e-12


def test_cauchy_fp64_and_adaptive(ctx):
    lra = _lra()
    _say("cauchy fp64 adaptive")
    rng = np.random.default_rng(0)
    s = rng.uniform(0, 1, 3000)
    t = rng.uniform(1.01, 2.01, 2500)
    cand = rng.choice(2500, 80, replace=False)
    Q, S = synth.residual_sample(3000, 2500, 0)
    ref = oracle.ca_cur(oracle.cauchy(s, t), 8, 4, 1e-10, cand, Q, S, k_max=40)
    res = ctx.ca_cur(lra.cauchy(torch.from_numpy(s).cuda(), torch.from_numpy(t).cuda()), 8, 4, 1e-10,
                     init_cols=cand, sample_rows=Q, sample_cols=S, k_max=40, factors=True)
    assert res.status == ref.status and res.k == ref.k
    if ref.min_gap() >= GAMMA64:
        np.testing.assert_array_equal(res.I, ref.I)
        np.testing.assert_array_equal(res.J, ref.J)
    assert res.err_est_rel <= 1e-10
    # generated entries are bit-exact IEEE divisions
    Cg = res.C.cpu().numpy()
    np.testing.assert_array_equal(Cg, 1.0 / (s[:, None] - t[res.J][None, :]))


def test_invdist_mixed(ctx):
    lra = _lra()
    _say("invdist mixed")
    rng = np.random.default_rng(1)
    x = np.sort(rng.uniform(0.0, 0.25, 2000))
    y = np.sort(rng.uniform(0.5, 0.75, 1800))
    cand = rng.choice(1800, 96, replace=False)
    Q, S = synth.residual_sample(2000, 1800, 1)
    ref = oracle.ca_cur(oracle.invdist(x, y), 8, 3, 1e-8, cand, Q, S, k_max=48, precision="f32")
    res = ctx.ca_cur(lra.invdist(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()), 8, 3, 1e-8,
                     init_cols=cand, sample_rows=Q, sample_cols=S, k_max=48,
                     precision=lra.PREC_MIXED, factors=True)
    assert res.status == ref.status and res.k == ref.k, (res.status, ref.status, res.k, ref.k)
    if ref.min_gap() >= GAMMA32:
        np.testing.assert_array_equal(res.I, ref.I)
        np.testing.assert_array_equal(res.J, ref.J)
        assert abs(res.err_est_rel - ref.err_est_rel) <= 1e-9 * ref.err_est_rel + 1e-15
    Cg = res.C.cpu().numpy()
    exp = (np.float32(1.0) / np.abs(x[:, None] - y[res.J][None, :]).astype(np.float32))
    np.testing.assert_array_equal(Cg, exp)


U64 = 2.0 ** -53


@pytest.mark.parametrize("team", [0, 3])
@pytest.mark.parametrize("seed", range(4))
def test_adaptive_growth_clear_decisions(ctx, seed, team):
    """Rank growth checked decision by decision: a matrix with singular values
    10^(-j/8) and tol 1e-3 grows k 8 -> 16 -> 24 -> 32, and every decision of
    the oracle (LU pivots, swaps, stop tests, warm-start and rank tests, and
    the estimate against tol at each level) clears the rounding of the basis,
    so the index sets, ranks, sweep and swap counts must be identical."""
    lra = _lra()
    _say(f"adaptive growth seed {seed} team {team}")
    A, d = synth.spectrum_dense(seed, 3000, 2500, decay=8.0)
    ref = oracle.ca_cur(oracle.dense(A), 8, 4, 1e-3, d.cand_cols, d.sample_rows, d.sample_cols, k_max=40)
    assert ref.status == 0 and ref.k == 32
    assert ref.min_gap() >= max(GAMMA64, 1000.0 * ref.k * ref.nucleus_cond1 * U64), ref.trace
    kw = dict(init_cols=d.cand_cols, sample_rows=d.sample_rows, sample_cols=d.sample_cols, k_max=40)
    if team:
        kw["team_wgs"] = team
    res = ctx.ca_cur(lra.dense(torch.from_numpy(A).cuda()), 8, 4, 1e-3, **kw)
    assert (res.status, res.k, res.sweeps_done, res.swaps_total) == \
        (ref.status, ref.k, ref.sweeps_done, ref.swaps_total)
    np.testing.assert_array_equal(res.I, ref.I)
    np.testing.assert_array_equal(res.J, ref.J)
    np.testing.assert_array_equal(res.G, ref.G)
    np.testing.assert_allclose(res.U, ref.U, rtol=1e-8, atol=1e-8 * np.abs(ref.U).max())
    assert abs(res.err_est_rel - ref.err_est_rel) <= 1e-9 * ref.err_est_rel


@pytest.mark.parametrize("team", [64, 0])
def test_dense_16384_fp64_path(ctx, team):
    """The dense 16384 x 16384 float32 workload (rank-32 scaled factor-Gaussian
    + 1e-4 noise, k = 32, 4 sweeps) in the launch configuration the benchmark
    times (a team of 64 workgroups, register-resident swap rows, strips in
    LDS) and with the automatic team: the oracle's smallest decision margin is
    ~1.3e-3, far above gamma, so index sets must be identical."""
    lra = _lra()
    _say(f"dense 16384 fp64 path team {team}")
    A, d = _dense16384()
    ref = _dense16384_ref()
    assert ref.status == 0 and ref.min_gap() >= GAMMA64
    kw = dict(init_cols=d.cand_cols, sample_rows=d.sample_rows, sample_cols=d.sample_cols)
    if team:
        kw["team_wgs"] = team
    res = ctx.ca_cur(lra.dense(_dense16384_dev()), 32, 4, 0.0, **kw)
    assert (res.status, res.k, res.sweeps_done, res.swaps_total) == \
        (ref.status, ref.k, ref.sweeps_done, ref.swaps_total)
    np.testing.assert_array_equal(res.I, ref.I)
    np.testing.assert_array_equal(res.J, ref.J)
    np.testing.assert_array_equal(res.G, ref.G)
    assert abs(res.err_est_rel - ref.err_est_rel) <= 1e-9 * ref.err_est_rel
    assert res.entries_read == ref.entries_read


_D16 = {}


def _dense16384():
    if "A" not in _D16:
        _D16["A"], _D16["d"] = synth.dense_scaled(0)
    return _D16["A"], _D16["d"]


def _dense16384_ref():
    if "ref" not in _D16:
        A, d = _dense16384()
        _D16["ref"] = oracle.ca_cur(oracle.dense(A), 32, 4, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    return _D16["ref"]


def _dense16384_dev():
    if "dev" not in _D16:
        _D16["dev"] = torch.from_numpy(_dense16384()[0]).cuda()
    return _D16["dev"]


@pytest.mark.parametrize("team", [0, 4])
@pytest.mark.parametrize("shape", [(2000, 1500, 40), (1500, 2000, 64)])
def test_rank_above_32(ctx, team, shape):
    """Ranks past 32 take the LDS forms of the small solves (warm start, L1
    inverse, nucleus) and the general swap path (team 0: automatic size)."""
    lra = _lra()
    m, n, k = shape
    _say(f"rank above 32 {shape} team {team}")
    A, d = synth.rect_factor_gaussian(100 + k, m, n, k, 1e-6, k)
    ref = oracle.ca_cur(oracle.dense(A), k, 2, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    kw = dict(init_cols=d.cand_cols, sample_rows=d.sample_rows, sample_cols=d.sample_cols)
    if team:
        kw["team_wgs"] = team
    res = ctx.ca_cur(lra.dense(torch.from_numpy(A).cuda()), k, 2, 0.0, **kw)
    assert _check_same(res, ref, GAMMA64, f"{shape} team {team}")
    assert abs(res.err_est_rel - ref.err_est_rel) <= 1e-9 * ref.err_est_rel + 1e-15
    np.testing.assert_allclose(res.U, ref.U, rtol=1e-8, atol=1e-8 * np.abs(ref.U).max())
    np.testing.assert_array_equal(res.G, ref.G)


# ---------------------------------------------------------------------------
# maxvol alone
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(300, 10), (5000, 32), (70000, 8), (4000, 48), (3000, 64)])
def test_maxvol_alone(ctx, shape):
    _say(f"maxvol alone {shape}")
    m, k = shape
    rng = np.random.default_rng(m + k)
    Cs = rng.standard_normal((m, k)) * np.exp(rng.uniform(-2, 2, k))[None, :]
    ref = oracle.maxvol(Cs, tau=0.01)
    Ct = torch.from_numpy(np.asfortranarray(Cs)).cuda()
    Ct = torch.as_strided(torch.from_numpy(Cs.T.copy()).cuda(), (m, k), (1, m))
    out = ctx.maxvol(Ct, tau=0.01)
    sol = np.linalg.solve(Cs[out["I"], :].T, Cs.T).T
    assert np.abs(sol).max() <= 1.01 + 1e-9
    if ref["trace"].min_swap_gap >= GAMMA64 and ref["trace"].min_pivot_gap >= GAMMA64 and \
            ref["trace"].min_stop_margin >= GAMMA64:
        np.testing.assert_array_equal(out["I"], ref["I"])
        assert out["swaps"] == ref["swaps"]
    warm = ctx.maxvol(Ct, tau=0.01, init=out["I"])
    assert warm["swaps"] == 0
    np.testing.assert_array_equal(warm["I"], out["I"])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_maxvol_warm_fallback(ctx, prec):
    """A warm start from rows whose C[I,:] is singular (repeated strip rows)
    must fail the rank test of the warm elimination and restart from the
    partial-pivot LU: the result equals the cold start, on the GPU as in the
    oracle (which takes the same fallback)."""
    _say(f"maxvol warm fallback {prec}")
    rng = np.random.default_rng(21)
    m, k = 3000, 16
    dt = np.float64 if prec == "f64" else np.float32
    Cs = (rng.standard_normal((m, k)) * np.exp(rng.uniform(-1, 1, k))[None, :]).astype(dt)
    Cs[400] = Cs[170]
    Cs[1777] = Cs[23]
    init = [170, 400, 23, 1777] + list(range(600, 600 + k - 4))
    ref_cold = oracle.maxvol(Cs, tau=0.01, precision=prec)
    ref_warm = oracle.maxvol(Cs, tau=0.01, init=init, precision=prec)
    np.testing.assert_array_equal(ref_warm["I"], ref_cold["I"])
    assert ref_warm["trace"].min_rank_margin <= 1.0
    Ct = torch.as_strided(torch.from_numpy(np.ascontiguousarray(Cs.T)).cuda(), (m, k), (1, m))
    cold = ctx.maxvol(Ct, tau=0.01)
    warm = ctx.maxvol(Ct, tau=0.01, init=init)
    np.testing.assert_array_equal(warm["I"], cold["I"])
    assert warm["swaps"] == cold["swaps"] and warm["k_eff"] == k
    gamma = GAMMA64 if prec == "f64" else GAMMA32
    tr = ref_cold["trace"]
    if min(tr.min_pivot_gap, tr.min_swap_gap, tr.min_stop_margin) >= gamma:
        np.testing.assert_array_equal(warm["I"], ref_warm["I"])
        assert warm["swaps"] == ref_warm["swaps"]
    C64 = Cs.astype(np.float64)
    sol = np.linalg.solve(C64[warm["I"], :].T, C64.T).T
    assert np.abs(sol).max() <= 1.01 * (1 + (1e-9 if prec == "f64" else 1e-3))


# ---------------------------------------------------------------------------
# error paths and degenerate cases
# ---------------------------------------------------------------------------

def test_errors(ctx):
    lra = _lra()
    _say("error paths")
    A, d = synth.plain_fp64(1)
    bad = A.copy()
    bad[10, d.cand_cols[0]] = np.nan
    r = ctx.ca_cur(lra.dense(torch.from_numpy(bad).cuda()), 8, 1, 0.0, init_cols=d.cand_cols,
                   sample_rows=d.sample_rows, sample_cols=d.sample_cols, raise_on_error=False)
    assert r.status == lra.ENONFINITE
    Z = torch.zeros(64, 64, dtype=torch.float64, device="cuda")
    r = ctx.ca_cur(lra.dense(Z), 2, 1, 0.0, raise_on_error=False)
    assert r.status == lra.ERANK
    with pytest.raises(lra.LraError):
        ctx.ca_cur(lra.dense(torch.from_numpy(A).cuda()), 0, 1, 0.0)
    with pytest.raises(lra.LraError):
        ctx.ca_cur(lra.dense(torch.from_numpy(A).cuda()), 8, 1, 0.0, init_cols=[1, 1, 2, 3, 4, 5, 6, 7])
    # delta-matrix (Appendix E): the spike is missed, rank loss reported
    D = torch.zeros(512, 512, dtype=torch.float64, device="cuda")
    D[300, 17] = 1.0
    r = ctx.ca_cur(lra.dense(D), 2, 2, 0.0, init_cols=[5, 9], raise_on_error=False)
    assert r.status == lra.ERANK
    # a context usable after errors
    r = ctx.ca_cur(lra.dense(torch.from_numpy(A).cuda()), 8, 3, 0.0, init_cols=d.cand_cols,
                   sample_rows=d.sample_rows, sample_cols=d.sample_cols)
    assert r.status == 0


def test_k_equals_min_dim(ctx):
    lra = _lra()
    _say("k == n")
    rng = np.random.default_rng(2)
    A = rng.standard_normal((200, 6))
    ref = oracle.ca_cur(oracle.dense(A), 6, 2, 0.0, np.arange(6), np.arange(64), np.arange(6))
    res = ctx.ca_cur(lra.dense(torch.from_numpy(A).cuda()), 6, 2, 0.0, init_cols=np.arange(6),
                     sample_rows=np.arange(64), sample_cols=np.arange(6))
    assert res.status == ref.status == 0
    assert sorted(res.J.tolist()) == list(range(6))
    assert res.err_est_rel <= 1e-13


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_dependent_columns(ctx, prec):
    """A repeated / scaled column in the start set: rank loss, as the oracle."""
    lra = _lra()
    _say(f"dependent columns {prec}")
    rng = np.random.default_rng(4)
    A = rng.standard_normal((60, 40))
    A[:, 7] = A[:, 3]
    A[:, 11] = 2.0 * A[:, 5]
    A = A.astype(np.float64 if prec == "f64" else np.float32)
    for J0, kk in (([3, 5, 0, 7, 11], 3), ([3, 7, 5, 11, 0], 1)):
        ref = oracle.ca_cur(oracle.dense(A), 5, 1, 0.0, J0, np.arange(60), np.arange(40), precision=prec)
        res = ctx.ca_cur(lra.dense(torch.from_numpy(A).cuda()), 5, 1, 0.0, init_cols=J0,
                         sample_rows=np.arange(60), sample_cols=np.arange(40),
                         precision=lra.PREC_FP64 if prec == "f64" else lra.PREC_MIXED)
        assert res.status == ref.status == lra.NUMERICAL_RANK and res.k == ref.k == kk
        np.testing.assert_array_equal(res.J, ref.J)
        np.testing.assert_array_equal(res.I, ref.I)


def test_global_strip_path_matches_lds_path(ctx):
    """Slices that do not fit LDS live in a global strip: capping the LDS for
    strip rows (LRA_LDS_B_BYTES) forces that path; results are bit-identical."""
    lra = _lra()
    _say("global strip path")
    A, d = synth.rect_factor_gaussian(7, 3000, 2200, 16, 1e-6, 16, n_cand=32)
    At = torch.from_numpy(A).cuda()
    kw = dict(init_cols=d.cand_cols, sample_rows=d.sample_rows, sample_cols=d.sample_cols)
    ref = ctx.ca_cur(lra.dense(At), 16, 3, 0.0, **kw)
    old = os.environ.get("LRA_LDS_B_BYTES")
    os.environ["LRA_LDS_B_BYTES"] = "1024"
    try:
        c2 = lra.Context()
    finally:
        if old is None:
            del os.environ["LRA_LDS_B_BYTES"]
        else:
            os.environ["LRA_LDS_B_BYTES"] = old
    for team in (1, 4):
        r = c2.ca_cur(lra.dense(At), 16, 3, 0.0, team_wgs=team, **kw)
        assert r.status == ref.status and r.k == ref.k
        np.testing.assert_array_equal(r.I, ref.I)
        np.testing.assert_array_equal(r.J, ref.J)
        np.testing.assert_array_equal(r.U, ref.U)
        assert r.err_est_rel == ref.err_est_rel
    c2.close()


# ---------------------------------------------------------------------------
# nucleus and estimator on sample sizes off the 16 x 16 product tiles and on
# both sides of the 32-column split of the nucleus solve
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k,q,s", [(16, 37, 20), (32, 64, 48), (8, 50, 64), (32, 23, 31),
                                   (32, 64, 33), (40, 45, 50), (1, 1, 1)])
def test_nucleus_sample_shapes(ctx, k, q, s):
    lra = _lra()
    m, n = 900, 700
    _say(f"nucleus sample shapes k {k} q {q} s {s}")
    A, d = synth.rect_factor_gaussian(31 + k + q + s, m, n, k, 1e-6, k)
    Q, S = synth.residual_sample(m, n, 500 + q + s, q, s)
    assert len(Q) == q and len(S) == s
    ref = oracle.ca_cur(oracle.dense(A), k, 2, 0.0, d.cand_cols, Q, S)
    res = ctx.ca_cur(lra.dense(torch.from_numpy(A).cuda()), k, 2, 0.0, init_cols=d.cand_cols,
                     sample_rows=Q, sample_cols=S)
    torch.cuda.synchronize()
    same = _check_same(res, ref, GAMMA64, f"k {k} q {q} s {s}")
    assert abs(res.err_est_rel - ref.err_est_rel) <= 1e-10
    if same:
        assert abs(res.err_est_rel - ref.err_est_rel) <= 1e-9 * ref.err_est_rel + 1e-15
        np.testing.assert_allclose(res.U, ref.U, rtol=1e-8, atol=1e-8 * np.abs(ref.U).max())
        np.testing.assert_array_equal(res.G, ref.G)
