"""Pins for the oracle's pre-processed source (kind 3): C-A on F A H with
d-abridged Hadamard multipliers and random sign scaling on both sides
(the paper's Section 8.3, family (i); recovery of an LRA of A after
orthogonal multipliers, Section 6.6).

* entries equal (F A H)_ij with F and H built densely from their definition
  (Kronecker Sylvester-Hadamard blocks, sign diagonals from SplitMix64) and
  multiplied by LAPACK-backed numpy; F and H are orthogonal;
* bitwise: each entry equals the same sum written out in Python in the same
  order (t outer, u inner);
* the CUR of F A H gives an LRA of A with the same error,
  ||A - F^T C U R H^T||_F = ||F A H - C U R||_F (orthogonal invariance), and a
  rank-r A is reproduced exactly;
* the point of pre-processing: a sum of two spikes (rank 2, Appendix E's hard
  inputs) defeats C-A from random columns, while after full-depth
  pre-processing C-A reproduces it exactly.
"""
import numpy as np
import pytest

import oracle
import synth


def _sign(seed, i):
    return -1.0 if (oracle.splitmix64(seed, i) >> 63) else 1.0


def _multipliers(m, n, d, seed):
    def abridged(N):
        h = np.array([[(-1.0) ** bin(a & b).count("1") for b in range(1 << d)] for a in range(1 << d)])
        return np.kron(h, np.eye(N >> d))
    F = np.diag([_sign(seed, i) for i in range(m)]) @ abridged(m) / 2 ** (d / 2)
    H = abridged(n) @ np.diag([_sign(seed + 1, j) for j in range(n)]) / 2 ** (d / 2)
    return F, H


@pytest.mark.parametrize("m,n,d", [(64, 48, 1), (96, 80, 3), (128, 64, 6)])
def test_entries_against_dense_multipliers(m, n, d):
    rng = np.random.default_rng(m + d)
    A = rng.standard_normal((m, n))
    F, H = _multipliers(m, n, d, 7)
    np.testing.assert_allclose(F @ F.T, np.eye(m), atol=1e-14)
    np.testing.assert_allclose(H.T @ H, np.eye(n), atol=1e-14)
    Mb = F @ A @ H
    src = oracle.abridged(A, d, 7)
    for (i, j) in [(0, 0), (m - 1, n - 1), (m // 3, n // 2), (5, n - 7)]:
        assert oracle.entry(src, i, j) == pytest.approx(Mb[i, j], abs=1e-12 * np.abs(A).max())
    # column-major storage of the same matrix
    srcc = oracle.abridged(A, d, 7, col_major=True)
    assert oracle.entry(srcc, 3, 4) == oracle.entry(src, 3, 4)


def test_entry_bitwise_against_the_written_out_sum():
    rng = np.random.default_rng(2)
    m, n, d, seed = 40, 24, 3, 123
    A = rng.standard_normal((m, n))
    src = oracle.abridged(A, d, seed)
    bm, bn = m >> d, n >> d
    for (i, j) in [(0, 0), (17, 9), (39, 23)]:
        ib, ir, jb, jr = i // bm, i % bm, j // bn, j % bn
        acc = 0.0
        for t in range(1 << d):
            for u in range(1 << d):
                v = float(A[ir + t * bm, jr + u * bn])
                neg = (bin(ib & t).count("1") + bin(u & jb).count("1")) & 1
                acc += -v if neg else v
        ref = acc * _sign(seed, i) * _sign(seed + 1, j) * 2.0 ** -d
        assert oracle.entry(src, i, j) == ref
        assert oracle.entry(src, i, j, "f32") == np.float32(ref)


@pytest.mark.parametrize("seed", range(3))
def test_recovered_lra_has_the_same_error(seed):
    m, n, d, k = 256, 192, 3, 8
    A, _ = synth.rect_factor_gaussian(seed, m, n, k, 1e-5, k)
    src = oracle.abridged(A, d, 99 + seed)
    rng = np.random.default_rng(seed)
    cand = rng.choice(n, k, replace=False)
    Q, S = synth.residual_sample(m, n, seed)
    res = oracle.ca_cur(src, k, 3, 0.0, cand, Q, S)
    assert res.status == 0
    F, H = _multipliers(m, n, d, 99 + seed)
    Mb = F @ A @ H
    cur = Mb[:, res.J] @ res.U @ Mb[res.I, :]
    rec = F.T @ cur @ H.T
    e_pre = np.linalg.norm(Mb - cur)
    assert np.linalg.norm(A - rec) == pytest.approx(e_pre, rel=1e-9)
    assert e_pre / np.linalg.norm(A) < 1e-3
    # the estimator samples F A H: it estimates the recovered error
    full = oracle.residual(src, res.I, res.J, np.arange(m), np.arange(n))
    assert full["norm_e"] == pytest.approx(e_pre, rel=1e-9)


def test_rank_r_reproduced_exactly():
    m, n, d, r = 128, 96, 2, 6
    rng = np.random.default_rng(5)
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    src = oracle.abridged(A, d, 1)
    cand = rng.choice(n, r, replace=False)
    Q, S = synth.residual_sample(m, n, 5)
    res = oracle.ca_cur(src, r, 2, 0.0, cand, Q, S)
    assert res.status == 0 and res.err_est_rel < 1e-12


def test_spikes_need_preprocessing():
    """A = 5 e_p e_q^T + 3 e_p' e_q'^T (Appendix E: C-A misses what its
    strips do not meet).  From random columns that miss q and q', plain C-A
    sees a zero strip (exact rank loss); after full-depth pre-processing
    every column of F A H carries both spikes and C-A reproduces A."""
    m = n = 64
    A = np.zeros((m, n))
    A[10, 20] = 5.0
    A[40, 50] = 3.0
    cand = np.array([1, 2, 3, 4, 5, 6, 7, 8, 9, 11])[:2]
    Q, S = synth.residual_sample(m, n, 0)
    plain = oracle.ca_cur(oracle.dense(A), 2, 2, 0.0, cand, Q, S)
    assert plain.status == -2
    src = oracle.abridged(A, 6, 4)
    pre = oracle.ca_cur(src, 2, 2, 0.0, cand, Q, S)
    assert pre.status == 0
    F, H = _multipliers(m, n, 6, 4)
    Mb = F @ A @ H
    rec = F.T @ (Mb[:, pre.J] @ pre.U @ Mb[pre.I, :]) @ H.T
    np.testing.assert_allclose(rec, A, atol=1e-12)
