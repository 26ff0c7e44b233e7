"""GPU parity of C-A on a pre-processed matrix (the source F A H of
d-abridged Hadamard multipliers with random sign scaling on both sides,
Section 8.3 family (i); recovery of an LRA of A, Section 6.6) against the
oracle's kind-3 source.

Each entry of F A H is the same binary64 sum on both sides (t outer, u inner,
exact sign and 2^-d factors), so the gathered entries and the generator are
bit-identical; index sets are compared where the oracle's decisions are
clear, as for the other sources.  Also: C = (F A H)[:, J] and R = (F A H)[I, :]
from lra_cur_factors bit-exact against the oracle's entries; the LRA of A
recovered from the GPU's factors, F^T C U R H^T, has the error of C U R
against F A H; a two-spike matrix that C-A from random columns cannot see is
reproduced after full-depth pre-processing; batched and served runs equal
the single-problem calls bit for bit; invalid depths are rejected.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
GAMMA64 = 1e-9


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_1611_01391_amd import lra
    c = lra.Context()
    yield c
    c.close()


def _sign(seed, i):
    return -1.0 if (oracle.splitmix64(seed, i) >> 63) else 1.0


def _multipliers(m, n, d, seed):
    """F and H written out densely from their definition."""
    def abridged(N):
        h = np.array([[(-1.0) ** bin(a & b).count("1") for b in range(1 << d)] for a in range(1 << d)])
        return np.kron(h, np.eye(N >> d))
    F = np.diag([_sign(seed, i) for i in range(m)]) @ abridged(m) / 2 ** (d / 2)
    H = abridged(n) @ np.diag([_sign(seed + 1, j) for j in range(n)]) / 2 ** (d / 2)
    return F, H


def _same_sets(res, ref, what):
    assert (res.status, res.k) == (ref.status, ref.k), (what, res.status, ref.status, res.k, ref.k)
    if ref.min_gap() >= GAMMA64:
        np.testing.assert_array_equal(res.I, ref.I, err_msg=what)
        np.testing.assert_array_equal(res.J, ref.J, err_msg=what)
        np.testing.assert_array_equal(res.G, ref.G, err_msg=what)
        # the generators are bit-identical: U differs by the rounding of its
        # inversion, relative k cond_1 u
        tol = max(1e-9, 100 * ref.k * ref.nucleus_cond1 * 2.0 ** -53)
        np.testing.assert_allclose(res.U, ref.U, rtol=tol, atol=tol * np.abs(ref.U).max(), err_msg=what)
        assert abs(res.err_est_rel - ref.err_est_rel) <= 1e-9 * ref.err_est_rel + 1e-15, what
        return True
    return False


@pytest.mark.parametrize("d", [1, 3, 5])
@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("col_major", [False, True])
def test_preprocessed_vs_oracle(ctx, d, seed, col_major):
    from paper_1611_01391_amd import lra
    _say(f"preprocessed d={d} seed={seed} col_major={col_major}")
    m, n, k = 512, 384, 8
    A, dr = synth.rect_factor_gaussian(seed, m, n, k, 1e-6, k)
    # a column-major m x n view: stride(0) == 1
    At = torch.from_numpy(A.T.copy()).cuda().t() if col_major else torch.from_numpy(A).cuda()
    ref = oracle.ca_cur(oracle.abridged(A, d, 40 + seed, col_major), k, 3, 0.0, dr.cand_cols, dr.sample_rows,
                        dr.sample_cols)
    res = ctx.ca_cur(lra.preprocessed(At, d, 40 + seed, col_major), k, 3, 0.0, init_cols=dr.cand_cols,
                     sample_rows=dr.sample_rows, sample_cols=dr.sample_cols)
    assert _same_sets(res, ref, f"d={d} seed={seed}")
    assert res.entries_read == ref.entries_read
    assert res.err_est_rel < 1e-4


@pytest.mark.parametrize("seed", [2, 3])
def test_preprocessed_binary32(ctx, seed):
    """float32 storage on the binary32 path: each entry is the binary64 sum
    rounded once to binary32 on both sides."""
    from paper_1611_01391_amd import lra
    _say(f"preprocessed binary32 seed={seed}")
    m, n, k, d = 640, 512, 8, 4
    A, dr = synth.rect_factor_gaussian(seed, m, n, k, 1e-4, k, dtype=np.float32)
    ref = oracle.ca_cur(oracle.abridged(A, d, seed), k, 3, 0.0, dr.cand_cols, dr.sample_rows, dr.sample_cols,
                        precision="f32")
    res = ctx.ca_cur(lra.preprocessed(torch.from_numpy(A).cuda(), d, seed), k, 3, 0.0, init_cols=dr.cand_cols,
                     sample_rows=dr.sample_rows, sample_cols=dr.sample_cols, precision=lra.PREC_MIXED)
    assert (res.status, res.k) == (ref.status, ref.k)
    if ref.min_gap() >= 1e-3:
        np.testing.assert_array_equal(res.I, ref.I)
        np.testing.assert_array_equal(res.J, ref.J)
        assert abs(res.err_est_rel - ref.err_est_rel) <= 1e-9 * ref.err_est_rel + 1e-15


def test_preprocessed_dense_16384(ctx):
    """The dense 16384 x 16384 float32 workload through depth-3 multipliers
    (seed 5), k = 32, 4 sweeps, in the benchmark's configuration."""
    from paper_1611_01391_amd import lra
    _say("preprocessed dense 16384 depth 3")
    A, d = synth.dense_scaled(0)
    res = ctx.ca_cur(lra.preprocessed(torch.from_numpy(A).cuda(), 3, 5), 32, 4, 0.0, init_cols=d.cand_cols,
                     sample_rows=d.sample_rows, sample_cols=d.sample_cols)
    ref = oracle.ca_cur(oracle.abridged(A, 3, 5), 32, 4, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    assert _same_sets(res, ref, "dense 16384 depth 3")
    assert res.entries_read == ref.entries_read


def test_factors_bitwise_and_recovery(ctx):
    from paper_1611_01391_amd import lra
    _say("preprocessed factors and recovery")
    m, n, k, d, seed = 256, 192, 8, 3, 77
    A, dr = synth.rect_factor_gaussian(4, m, n, k, 1e-5, k)
    src = lra.preprocessed(torch.from_numpy(A).cuda(), d, seed)
    res = ctx.ca_cur(src, k, 3, 0.0, init_cols=dr.cand_cols, sample_rows=dr.sample_rows, sample_cols=dr.sample_cols)
    assert res.status == 0
    C, R = ctx.cur_factors(src, res.I, res.J)
    C, R = C.cpu().numpy(), R.cpu().numpy()
    hs = oracle.abridged(A, d, seed)
    Cref = np.array([[oracle.entry(hs, i, j) for j in res.J] for i in range(m)])
    Rref = np.array([[oracle.entry(hs, i, j) for j in range(n)] for i in res.I])
    np.testing.assert_array_equal(C, Cref)
    np.testing.assert_array_equal(R, Rref)
    F, H = _multipliers(m, n, d, seed)
    Mb = F @ A @ H
    cur = C @ res.U @ R
    e_pre = np.linalg.norm(Mb - cur)
    rec = F.T @ cur @ H.T
    assert np.linalg.norm(A - rec) == pytest.approx(e_pre, rel=1e-9)
    assert e_pre / np.linalg.norm(A) < 1e-3


def test_spikes_need_preprocessing(ctx):
    """Two spikes: from columns that miss them C-A loses rank; after
    full-depth pre-processing it reproduces A."""
    from paper_1611_01391_amd import lra
    _say("preprocessed spikes")
    m = n = 64
    A = np.zeros((m, n))
    A[10, 20] = 5.0
    A[40, 50] = 3.0
    cand = np.array([1, 2], dtype=np.int64)
    Q, S = synth.residual_sample(m, n, 0)
    At = torch.from_numpy(A).cuda()
    plain = ctx.ca_cur(lra.dense(At), 2, 2, 0.0, init_cols=cand, sample_rows=Q, sample_cols=S,
                       raise_on_error=False)
    assert plain.status == lra.ERANK
    src = lra.preprocessed(At, 6, 4)
    pre = ctx.ca_cur(src, 2, 2, 0.0, init_cols=cand, sample_rows=Q, sample_cols=S)
    ref = oracle.ca_cur(oracle.abridged(A, 6, 4), 2, 2, 0.0, cand, Q, S)
    assert pre.status == ref.status == 0
    C, R = ctx.cur_factors(src, pre.I, pre.J)
    F, H = _multipliers(m, n, 6, 4)
    rec = F.T @ (C.cpu().numpy() @ pre.U @ R.cpu().numpy()) @ H.T
    np.testing.assert_allclose(rec, A, atol=1e-12)


def _same(a, b, what):
    assert a.status == b.status, (what, a.status, b.status)
    np.testing.assert_array_equal(a.I, b.I, err_msg=what)
    np.testing.assert_array_equal(a.J, b.J, err_msg=what)
    np.testing.assert_array_equal(a.U, b.U, err_msg=what)
    assert a.err_est_rel == b.err_est_rel, what


def test_preprocessed_batched_and_served(ctx):
    """Pre-processed and plain blocks, adaptive rank, in one batched launch
    and as served requests: the same bits as the single-problem calls, and
    the single-problem calls identical to the oracle where its decisions are
    clear."""
    from paper_1611_01391_amd import lra
    _say("preprocessed batched and served")
    jobs, hosts = [], []
    for s in range(6):
        A, _ = synth.rect_factor_gaussian(10 + s, 256 + 64 * s, 192, 12, 1e-7, 8)
        At = torch.from_numpy(A).cuda()
        d = 1 + s % 4
        if s % 3:
            jobs.append((lra.preprocessed(At, d, 1000 + s), 8, 3, 1e-5))
            hosts.append(oracle.abridged(A, d, 1000 + s))
        else:
            jobs.append((lra.dense(At), 8, 3, 1e-5))
            hosts.append(oracle.dense(A))
    _, batched = ctx.ca_cur_batched(jobs, raise_on_error=False, k_max=24, seed=5)
    alone = [ctx.ca_cur(src, k, sw, tol, raise_on_error=False, k_max=24, seed=synth.block_draws(5, b))
             for b, (src, k, sw, tol) in enumerate(jobs)]
    sctx = lra.Context()
    tk = [sctx.submit(src, k, sw, tol, k_max=24, seed=synth.block_draws(5, b))
          for b, (src, k, sw, tol) in enumerate(jobs)]
    served = [sctx.wait(t) for t in tk]
    sctx.close()
    for b in range(len(jobs)):
        _same(batched[b], alone[b], f"batched block {b}")
        _same(served[b], alone[b], f"served block {b}")
    clear = 0
    for b, (src, k, sw, tol) in enumerate(jobs):
        m, n = src.m, src.n
        sd = synth.block_draws(5, b)
        cand = oracle.draw_distinct(sd, n, min(n, 2 * max(k, min(24, m, n))))
        Q = np.sort(oracle.draw_distinct(sd + 1, m, min(64, m)))
        S = np.sort(oracle.draw_distinct(sd + 2, n, min(64, n)))
        ref = oracle.ca_cur(hosts[b], k, sw, tol, cand, Q, S, k_max=24)
        clear += _same_sets(alone[b], ref, f"block {b}")
    assert clear >= 4, clear


def test_invalid_depth_rejected(ctx):
    from paper_1611_01391_amd import lra
    _say("preprocessed invalid depth")
    At = torch.zeros((96, 64), dtype=torch.float64, device="cuda")
    for d in (0, 9):
        with pytest.raises(lra.LraError):
            ctx.ca_cur(lra.preprocessed(At, d, 0), 4, 1, 0.0)
    with pytest.raises(lra.LraError):  # 2^6 does not divide 96
        ctx.ca_cur(lra.preprocessed(At, 6, 0), 4, 1, 0.0)
