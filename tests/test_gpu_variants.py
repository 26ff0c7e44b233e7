"""GPU parity of the fixed-rank CUR algorithms that the paper's C-A tests
compare (Section 12.2) and of the Primitive algorithm's truncated nucleus
(Section 6.5), against the CPU oracle on the same seeded inputs, through
the C ABI:

* Tests 1 -- random I, J (sweeps = 0) and U = A[I,J]^{-1};
* Tests 3 -- Cynical: a random 4r x 4r submatrix, then an r x r generator of
  locally maximal volume inside it (sweeps = 0, cur_rank = r);
* Tests 4 -- one C-A loop at width 4r, then the Cynical step (sweeps = 1);
* Primitive with k = l > r and U = (A[I,J])_r^+ (nucleus_rank = r), from
  random sets or after C-A sweeps.

Bars as in the other parity tests: index sets identical when the oracle's
decision margins clear gamma (1e-9 binary64, 1e-3 binary32); generator
bit-exact; sampled relative error within 1e-10 on the binary64 path.  The
truncated nucleus comes from a Jacobi SVD whose rotation order differs
between the two sides (cyclic on the host, round-robin pairs on the GPU),
so U agrees to rounding: within 1e-9 sigma_1(G) / sigma_r(G) relative.
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


def _paper_input(seed, n=512, r=8, eps=1e-10, k=None):
    """W = G1 G2 + eps G3 (the random inputs of the C-A tests), with the
    candidate columns and random rows of width k."""
    A, d = synth.plain_fp64(seed, n=n, r=r, eps=eps, k=k or r)
    rng = np.random.default_rng(seed + 50)
    rows = rng.choice(n, k or r, replace=False).astype(np.int64)
    return A, d, rows


def _compare(res, ref, gamma, what, est_tol=1e-10):
    assert res.status == ref.status, (what, res.status, ref.status)
    assert res.k == ref.k, (what, res.k, ref.k)
    clear = ref.min_gap() >= gamma
    if clear:
        np.testing.assert_array_equal(res.I, ref.I, err_msg=what)
        np.testing.assert_array_equal(res.J, ref.J, err_msg=what)
        np.testing.assert_array_equal(res.G, ref.G, err_msg=what)
        assert res.swaps_total == ref.swaps_total, what
        assert res.entries_read == ref.entries_read, (what, res.entries_read, ref.entries_read)
        assert abs(res.err_est_rel - ref.err_est_rel) <= est_tol, (what, res.err_est_rel, ref.err_est_rel)
    return clear


@pytest.mark.parametrize("seed", range(4))
def test_tests1_random_sets(ctx, seed):
    from paper_1611_01391_amd import lra
    _say(f"Tests 1 (random sets) seed {seed}")
    A, d, rows = _paper_input(seed)
    ref = oracle.cur_variant(oracle.dense(A), 8, 0, d.cand_cols, d.sample_rows, d.sample_cols, init_rows=rows)
    res = ctx.ca_cur(lra.dense(torch.from_numpy(A).cuda()), 8, 0, 0.0, init_cols=d.cand_cols,
                     init_rows=rows, sample_rows=d.sample_rows, sample_cols=d.sample_cols)
    assert _compare(res, ref, GAMMA64, f"tests1 {seed}")
    np.testing.assert_array_equal(res.I, rows)
    np.testing.assert_allclose(res.U, ref.U, rtol=0, atol=1e-9 * np.abs(ref.U).max())
    assert res.sweeps_done == 0


@pytest.mark.parametrize("sweeps", [0, 1])
@pytest.mark.parametrize("seed", range(4))
def test_cynical_fp64(ctx, seed, sweeps):
    """Tests 3 (sweeps = 0) and Tests 4 (sweeps = 1), p = q = 4r = 32, r = 8."""
    from paper_1611_01391_amd import lra
    _say(f"Cynical fp64 seed {seed} sweeps {sweeps}")
    A, d, rows = _paper_input(seed, k=32)
    ref = oracle.cur_variant(oracle.dense(A), 32, sweeps, d.cand_cols, d.sample_rows, d.sample_cols,
                             init_rows=rows, cur_rank=8)
    res = ctx.ca_cur(lra.dense(torch.from_numpy(A).cuda()), 32, sweeps, 0.0, init_cols=d.cand_cols,
                     init_rows=rows, sample_rows=d.sample_rows, sample_cols=d.sample_cols, cur_rank=8)
    _compare(res, ref, GAMMA64, f"cynical {seed}/{sweeps}")
    assert abs(res.err_est_rel - ref.err_est_rel) <= 1e-10
    assert res.k == 8 and res.status == 0


@pytest.mark.parametrize("team", [0, 3])
def test_cynical_mixed_and_teams(ctx, team):
    """The binary32 path, and the outer C-A loop on a team of workgroups
    (the reduction runs on the team's first workgroup)."""
    from paper_1611_01391_amd import lra
    _say(f"Cynical mixed team {team}")
    A, d = synth.rect_factor_gaussian(11, 3000, 2500, 12, 1e-6, 48)
    A32 = A.astype(np.float32)
    rows = np.random.default_rng(3).choice(3000, 48, replace=False).astype(np.int64)
    for prec, gamma in (("f32", GAMMA32), ("f64", GAMMA64)):
        ref = oracle.cur_variant(oracle.dense(A32), 48, 1, d.cand_cols, d.sample_rows, d.sample_cols,
                                 init_rows=rows, cur_rank=12, precision=prec)
        res = ctx.ca_cur(lra.dense(torch.from_numpy(A32).cuda()), 48, 1, 0.0, init_cols=d.cand_cols,
                         init_rows=rows, sample_rows=d.sample_rows, sample_cols=d.sample_cols, cur_rank=12,
                         team_wgs=team, precision=lra.PREC_FP64 if prec == "f64" else lra.PREC_MIXED)
        _compare(res, ref, gamma, f"cynical {prec} team {team}")
        assert res.err_est_rel <= 10 * ref.err_est_rel + 1e-12


@pytest.mark.parametrize("sweeps", [0, 2])
@pytest.mark.parametrize("seed", range(3))
def test_primitive_truncated_nucleus(ctx, seed, sweeps):
    """k = l = 16 > r = 8 on W = G1 G2 + 1e-10 G3 (numerical rank 8): the
    rank-8 truncated pseudo-inverse of the generator."""
    from paper_1611_01391_amd import lra
    _say(f"Primitive seed {seed} sweeps {sweeps}")
    A, d, rows = _paper_input(seed, k=16)
    ref = oracle.cur_variant(oracle.dense(A), 16, sweeps, d.cand_cols, d.sample_rows, d.sample_cols,
                             init_rows=rows, nucleus_rank=8)
    res = ctx.ca_cur(lra.dense(torch.from_numpy(A).cuda()), 16, sweeps, 0.0, init_cols=d.cand_cols,
                     init_rows=rows, sample_rows=d.sample_rows, sample_cols=d.sample_cols, nucleus_rank=8)
    if sweeps == 0:
        assert _compare(res, ref, GAMMA64, f"primitive {seed}")
    else:
        _compare(res, ref, GAMMA64, f"primitive {seed} after sweeps")
    if np.array_equal(res.I, ref.I) and np.array_equal(res.J, ref.J):
        s = np.linalg.svd(ref.G, compute_uv=False)
        tol = 1e-9 * s[0] / s[7] * np.abs(ref.U).max()
        np.testing.assert_allclose(res.U, ref.U, rtol=0, atol=tol)
        assert abs(res.err_est_rel - ref.err_est_rel) <= 1e-10
    assert res.err_est_rel < 1e-7


def test_primitive_large_rank(ctx):
    """k = 64, r = 40 (a spread spectrum): the Jacobi SVD at the largest
    generator, from random sets."""
    from paper_1611_01391_amd import lra
    _say("Primitive k 64 r 40")
    A, d = synth.spectrum_dense(7, 700, 650, decay=12.0, r=100, n_cand=64)
    rows = np.random.default_rng(7).choice(700, 64, replace=False).astype(np.int64)
    ref = oracle.cur_variant(oracle.dense(A), 64, 0, d.cand_cols, d.sample_rows, d.sample_cols,
                             init_rows=rows, nucleus_rank=40)
    res = ctx.ca_cur(lra.dense(torch.from_numpy(A).cuda()), 64, 0, 0.0, init_cols=d.cand_cols,
                     init_rows=rows, sample_rows=d.sample_rows, sample_cols=d.sample_cols, nucleus_rank=40)
    assert _compare(res, ref, GAMMA64, "primitive 64/40")
    s = np.linalg.svd(ref.G, compute_uv=False)
    tol = 1e-9 * s[0] / s[39] * np.abs(ref.U).max()
    np.testing.assert_allclose(res.U, ref.U, rtol=0, atol=tol)
    assert abs(res.err_est_rel - ref.err_est_rel) <= 1e-10 + 1e-6 * ref.err_est_rel


@pytest.mark.parametrize("case", ["tests1", "tests3", "tests4", "primitive"])
def test_variants_dense_16384(ctx, case):
    """The dense 16384 x 16384 float32 workload in the benchmark's
    configuration: random 64-column and 64-row draws of seed 11, Tests 1 at
    k = 32, Tests 3 and 4 from 64 x 64 to 16 x 16, the Primitive CUR of a
    64 x 64 generator at nucleus rank 32."""
    from paper_1611_01391_amd import lra
    _say(f"variants dense 16384 {case}")
    A, d = synth.dense_scaled(0)
    n = A.shape[0]
    rng = np.random.default_rng(11)
    cols64 = rng.choice(n, 64, replace=False).astype(np.int64)
    rows64 = rng.choice(n, 64, replace=False).astype(np.int64)
    spec = {"tests1": (32, 0, dict(init_cols=cols64[:32], init_rows=rows64[:32])),
            "tests3": (64, 0, dict(init_cols=cols64, init_rows=rows64, cur_rank=16)),
            "tests4": (64, 1, dict(init_cols=cols64, cur_rank=16)),
            "primitive": (64, 0, dict(init_cols=cols64, init_rows=rows64, nucleus_rank=32))}[case]
    k, sw, kw = spec
    res = ctx.ca_cur(lra.dense(torch.from_numpy(A).cuda()), k, sw, 0.0, sample_rows=d.sample_rows,
                     sample_cols=d.sample_cols, **kw)
    ref = oracle.cur_variant(oracle.dense(A), k, sw, kw["init_cols"], d.sample_rows, d.sample_cols,
                             init_rows=kw.get("init_rows"), cur_rank=kw.get("cur_rank", 0),
                             nucleus_rank=kw.get("nucleus_rank", 0))
    assert _compare(res, ref, GAMMA64, f"dense 16384 {case}", est_tol=1e-10 * max(1.0, ref.err_est_rel))
    if case == "primitive":
        s = np.linalg.svd(ref.G, compute_uv=False)
        tol = 1e-9 * s[0] / s[31] * np.abs(ref.U).max()
        np.testing.assert_allclose(res.U, ref.U, rtol=0, atol=tol)


def test_variants_batched_equal_single(ctx):
    """Cynical and Primitive problems inside one batched launch return the
    same bits as alone (default draws: stream seed + block index, random
    rows from stream seed + 3)."""
    from paper_1611_01391_amd import lra
    _say("variants batched == single")
    x, blocks, _ = synth.multipole(0, 1 << 14, 256, 96)
    xd = torch.from_numpy(x).cuda()
    sel = [b for b in range(len(blocks)) if min(blocks[b][1] - blocks[b][0], blocks[b][3] - blocks[b][2]) >= 64]
    sel = sel[:24]
    for opts in (dict(cur_rank=6), dict(nucleus_rank=6)):
        jobs = [(lra.invdist(xd[blocks[b][0]:blocks[b][1]], xd[blocks[b][2]:blocks[b][3]]), 24, 0, 0.0)
                for b in sel]
        _, out = ctx.ca_cur_batched(jobs, raise_on_error=False, seed=5, **opts)
        for i, (src, k, sw, tol) in enumerate(jobs):
            one = ctx.ca_cur(src, k, sw, tol, raise_on_error=False, seed=synth.block_draws(5, i), **opts)
            assert (out[i].status, out[i].k) == (one.status, one.k), (opts, i)
            np.testing.assert_array_equal(out[i].I, one.I)
            np.testing.assert_array_equal(out[i].J, one.J)
            np.testing.assert_array_equal(out[i].U, one.U)
            assert out[i].err_est_rel == one.err_est_rel


def test_variant_argument_checks(ctx):
    from paper_1611_01391_amd import lra
    A, d, rows = _paper_input(0, k=16)
    At = torch.from_numpy(A).cuda()
    src = lra.dense(At)
    # a tolerance needs C-A sweeps and a plain nucleus
    for kw in (dict(cur_rank=8), dict(nucleus_rank=8)):
        r = ctx.ca_cur(src, 16, 1, 1e-6, raise_on_error=False, **kw)
        assert r.status == lra.EINVAL
    r = ctx.ca_cur(src, 16, 0, 1e-6, raise_on_error=False)
    assert r.status == lra.EINVAL
    r = ctx.ca_cur(src, 16, 1, 0.0, raise_on_error=False, cur_rank=17)
    assert r.status == lra.EINVAL
    r = ctx.ca_cur(src, 16, 0, 0.0, raise_on_error=False, init_rows=np.zeros(16, dtype=np.int64))
    assert r.status == lra.EINVAL  # repeated rows
    # cur_rank = k and nucleus_rank = k are the plain algorithm
    base = ctx.ca_cur(src, 16, 1, 0.0, init_cols=d.cand_cols, sample_rows=d.sample_rows,
                      sample_cols=d.sample_cols)
    for kw in (dict(cur_rank=16), dict(nucleus_rank=16)):
        r = ctx.ca_cur(src, 16, 1, 0.0, init_cols=d.cand_cols, sample_rows=d.sample_rows,
                       sample_cols=d.sample_cols, **kw)
        np.testing.assert_array_equal(r.I, base.I)
        np.testing.assert_array_equal(r.U, base.U)
        assert r.err_est_rel == base.err_est_rel
