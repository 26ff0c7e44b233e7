"""GPU parity of the BF16-shortlist selection (LRA_PREC_BF16SEL): binary32
strips, each swap's candidates shortlisted from a bfloat16 MFMA product with
binary32 accumulation and rechecked in binary32; nucleus and estimate in
binary64.

Reference: the binary32 oracle, whose argmax is exact in binary32.  With
entrywise error d of the bfloat16 product, the shortlist holds the binary32
argmax whenever it leads by more than 2 d, so index sets are asserted
identical when the oracle's decision margins are at least gamma = 5e-2
(bfloat16 unit roundoff 2^-9 per operand, k-term sums).  Always asserted:
the same status and rank, the estimate within a small factor of the binary64
oracle's (the error of this path against binary64, stated in the bench), and
the stopping invariant of the last row step recomputed in binary64 on the
host, max |A[I,:]^T A[I,J]^{-T}| <= 1 + tau + 2 d + 1e-3 with d bounded by
2^-8 max_i sum_a |R_ia| |W_aj|.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GAMMA_BF16 = 5e-2
TAU = 0.01


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_1611_01391_amd import lra
    c = lra.Context()
    yield c
    c.close()


def _scaled(seed, m=800, n=700, r=4):
    """Rank-r product with log-uniform row and column scales over three
    decades (clear maxvol decisions), plus 1e-6 relative noise, float32."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    A *= np.exp(rng.uniform(np.log(1e-3), 0, m))[:, None]
    A *= np.exp(rng.uniform(np.log(1e-3), 0, n))[None, :]
    A += 1e-6 * rng.standard_normal((m, n)) * np.abs(A).max()
    A = A.astype(np.float32)
    cand = rng.choice(n, r, replace=False).astype(np.int64)
    Q, S = synth.residual_sample(m, n, seed)
    return A, cand, Q, S


def _row_invariant(A, I, J):
    """max over columns outside J of |B| for the last row step's basis
    B = A[I,:]^T A[I,J]^{-T}, and the bfloat16 error bound d of its product."""
    A64 = A.astype(np.float64)
    Rt = A64[I, :].T                      # n x k strip of the row step
    W = np.linalg.inv(Rt[J, :])           # C[X,:]^{-1}
    B = Rt @ W
    mask = np.ones(A.shape[1], dtype=bool)
    mask[J] = False
    d = 2.0 ** -8 * (np.abs(Rt) @ np.abs(W)).max()
    return np.abs(B[mask]).max(), d


@pytest.mark.parametrize("seed", [23, 1, 26, 10, 0, 44])
def test_bf16_select_vs_binary32_oracle(ctx, seed):
    from paper_1611_01391_amd import lra
    _say(f"bf16 select seed {seed}")
    A, cand, Q, S = _scaled(seed)
    src = oracle.dense(A)
    ref = oracle.ca_cur(src, 4, 3, 0.0, cand, Q, S, precision="f32")
    ref64 = oracle.ca_cur(src, 4, 3, 0.0, cand, Q, S)
    res = ctx.ca_cur(lra.dense(torch.from_numpy(A).cuda()), 4, 3, 0.0, init_cols=cand, sample_rows=Q,
                     sample_cols=S, precision=lra.PREC_BF16SEL)
    assert (res.status, res.k) == (ref.status, ref.k), (res.status, ref.status, res.k, ref.k)
    if ref.min_gap() >= GAMMA_BF16:
        np.testing.assert_array_equal(res.I, ref.I)
        np.testing.assert_array_equal(res.J, ref.J)
        assert abs(res.err_est_rel - ref.err_est_rel) <= 1e-9 * ref.err_est_rel + 1e-15
    assert res.err_est_rel <= 3.0 * ref64.err_est_rel + 1e-12
    inv, d = _row_invariant(A, res.I, res.J)
    assert inv <= 1 + TAU + 2 * d + 1e-3, (inv, d)


@pytest.mark.parametrize("team", [64, 0])
def test_bf16_select_dense_16384(ctx, team):
    """The dense 16384 x 16384 float32 workload (k = 32, 4 sweeps) in the
    benchmark's launch configuration."""
    from paper_1611_01391_amd import lra
    _say(f"bf16 select dense 16384 team {team}")
    A, d = synth.dense_scaled(0)
    At = torch.from_numpy(A).cuda()
    res = ctx.ca_cur(lra.dense(At), 32, 4, 0.0, init_cols=d.cand_cols, sample_rows=d.sample_rows,
                     sample_cols=d.sample_cols, precision=lra.PREC_BF16SEL, team_wgs=team)
    ref64 = oracle.ca_cur(oracle.dense(A), 32, 4, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    assert res.status == 0 and res.k == 32
    assert res.err_est_rel <= 1.5 * ref64.err_est_rel, (res.err_est_rel, ref64.err_est_rel)
    # the shortlist path ran: after the LU start of the first column step it
    # gathers that strip a second time, which the plain binary32 path does not
    mixed = ctx.ca_cur(lra.dense(At), 32, 4, 0.0, init_cols=d.cand_cols, sample_rows=d.sample_rows,
                       sample_cols=d.sample_cols, precision=lra.PREC_MIXED, team_wgs=team)
    assert res.entries_read == mixed.entries_read + 16384 * 32, (res.entries_read, mixed.entries_read)
    # the estimate of the returned sets, recomputed by the oracle on the same sample
    chk = oracle.residual(oracle.dense(A), res.I, res.J, d.sample_rows, d.sample_cols)
    assert abs(chk["est_rel"] - res.err_est_rel) <= 1e-10
    inv, dd = _row_invariant(A, res.I, res.J)
    assert inv <= 1 + TAU + 2 * dd + 1e-3, (inv, dd)


def test_bf16_select_served_equals_alone(ctx):
    """The flag travels with each request: served and batched runs of
    BF16-select problems return the same bits as alone."""
    from paper_1611_01391_amd import lra
    _say("bf16 select served == alone")
    probs = [_scaled(s, m=900 + 50 * s, n=700) for s in range(6)]
    tens = [torch.from_numpy(A).cuda() for (A, _, _, _) in probs]
    alone = [ctx.ca_cur(lra.dense(t), 4, 3, 0.0, init_cols=c, sample_rows=Q, sample_cols=S,
                        precision=lra.PREC_BF16SEL) for t, (_, c, Q, S) in zip(tens, probs)]
    sctx = lra.Context()
    tk = [sctx.submit(lra.dense(t), 4, 3, 0.0, init_cols=c, sample_rows=Q, sample_cols=S,
                      precision=lra.PREC_BF16SEL) for t, (_, c, Q, S) in zip(tens, probs)]
    served = [sctx.wait(t) for t in tk]
    sctx.close()
    for a, b in zip(alone, served):
        assert a.status == b.status
        np.testing.assert_array_equal(a.I, b.I)
        np.testing.assert_array_equal(a.J, b.J)
        assert a.err_est_rel == b.err_est_rel
