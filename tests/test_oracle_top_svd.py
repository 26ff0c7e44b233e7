"""Pins for the oracle of the LRA -> top SVD transition (Appendix D,
Algorithm D.1; oracle/top_svd.py).

* the pivoted QR against LAPACK's (scipy.linalg.qr with pivoting, dgeqp3):
  the same pivots wherever the oracle's pivot margins are clear, |R| equal,
  Q R = X P and Q orthonormal;
* with r = k the output is an exact SVD of C W R: S diag(sigma) T^T = C W R
  and sigma equals numpy's singular values of the product, S and T
  orthonormal, sigma descending (columns of very different scales, so that a
  dropped or misapplied permutation fails);
* a product of rank r with k > r is reproduced exactly at rank r;
* with noise the rank-r output is exactly the two-sided projection of
  C W R on the kept column spaces of the pivoted QR factors (LAPACK's),
  and its error lies between sigma_{r+1} and the factors' truncation
  residuals carried through the product;
* a request above the rank of C is reported as rank loss;
* applied to the oracle's C-A result on a rank-r + noise matrix, the top
  SVD is an LRA of A with the CUR's error up to the rank-r truncation.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle.top_svd import householder_qrp, top_svd

scipy_linalg = pytest.importorskip("scipy.linalg")


def _factors(seed, m, n, k, scales=True):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((m, k))
    R = rng.standard_normal((k, n))
    if scales:
        C *= np.exp(rng.uniform(-6, 0, k))[None, :]
        R *= np.exp(rng.uniform(-6, 0, k))[:, None]
    W = rng.standard_normal((k, k))
    return C, W, R


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("m,k", [(200, 8), (500, 32), (64, 64)])
def test_qrp_against_lapack(seed, m, k):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((m, k)) * np.exp(rng.uniform(-5, 0, k))[None, :]
    Q, R, piv, mg = householder_qrp(X)
    np.testing.assert_allclose(Q @ R, X[:, piv], atol=1e-13 * np.abs(X).max())
    np.testing.assert_allclose(Q.T @ Q, np.eye(k), atol=1e-13)
    assert np.allclose(np.tril(R, -1), 0.0)
    Ql, Rl, pl = scipy_linalg.qr(X, mode="economic", pivoting=True)
    clear = int(np.argmax(mg < 1e-9)) if (mg < 1e-9).any() else k
    np.testing.assert_array_equal(piv[:clear], pl[:clear])
    if clear == k:
        np.testing.assert_allclose(np.abs(R), np.abs(Rl), atol=1e-12 * np.abs(Rl).max())


def test_qrp_ties_take_the_lowest_index():
    X = np.eye(6)[:, ::-1] * 2.0
    _, R, piv, mg = householder_qrp(X)
    np.testing.assert_array_equal(piv, np.arange(6))
    assert mg[0] == 0.0
    np.testing.assert_allclose(np.abs(np.diag(R)), 2.0)


@pytest.mark.parametrize("seed", range(4))
def test_full_rank_is_an_exact_svd(seed):
    m, n, k = 300, 250, 12
    C, W, R = _factors(seed, m, n, k)
    out = top_svd(C, W, R, k)
    assert out.status == 0
    M = C @ W @ R
    sv = np.linalg.svd(M, compute_uv=False)
    np.testing.assert_allclose(out.sigma, sv[:k], rtol=1e-10, atol=1e-13 * sv[0])
    np.testing.assert_allclose(out.S @ np.diag(out.sigma) @ out.Tt, M, atol=1e-12 * sv[0])
    np.testing.assert_allclose(out.S.T @ out.S, np.eye(k), atol=1e-12)
    np.testing.assert_allclose(out.Tt @ out.Tt.T, np.eye(k), atol=1e-12)
    assert (np.diff(out.sigma) <= 0).all()
    # the pivots matter here: the middle factor built without them is wrong
    assert not np.array_equal(out.piv_c, np.arange(k)) and not np.array_equal(out.piv_r, np.arange(k))


@pytest.mark.parametrize("seed", range(3))
def test_rank_r_product_reproduced(seed):
    m, n, k, r = 240, 200, 16, 5
    rng = np.random.default_rng(100 + seed)
    C = rng.standard_normal((m, r)) @ rng.standard_normal((r, k))
    R = rng.standard_normal((k, r)) @ rng.standard_normal((r, n))
    W = rng.standard_normal((k, k))
    # C and R have rank r: a request of rank r is exact, one above is rank loss
    out = top_svd(C, W, R, r)
    assert out.status == 0
    M = C @ W @ R
    sv = np.linalg.svd(M, compute_uv=False)
    np.testing.assert_allclose(out.S @ np.diag(out.sigma) @ out.Tt, M, atol=1e-11 * sv[0])
    np.testing.assert_allclose(out.sigma, sv[:r], rtol=1e-9)
    assert top_svd(C, W, R, r + 1).status == -2


@pytest.mark.parametrize("seed", range(4))
def test_noisy_rank_r_is_the_two_sided_projection(seed):
    """With noise the rank-r output is exactly Pi_C C W R Pi_R, Pi_C and Pi_R
    the orthogonal projectors on the first r columns of the pivoted QR
    factors of C and R^T (here from LAPACK, independently of the oracle's own
    QR); its error is bounded by the truncation residuals of the two
    factors, ||R_C[r:,r:]|| ||W R|| + ||C W|| ||R_R[r:,r:]||, which is
    O(sigma_{r+1}) when C and R are themselves near rank r."""
    m, n, k, r = 400, 300, 16, 6
    rng = np.random.default_rng(200 + seed)
    eps = 1e-6
    C = rng.standard_normal((m, r)) @ rng.standard_normal((r, k)) + eps * rng.standard_normal((m, k))
    R = rng.standard_normal((k, r)) @ rng.standard_normal((r, n)) + eps * rng.standard_normal((k, n))
    W = rng.standard_normal((k, k))
    M = C @ W @ R
    sv = np.linalg.svd(M, compute_uv=False)
    out = top_svd(C, W, R, r)
    assert out.status == 0 and out.min_margin(r) > 1e-6
    Qc, Rc, _ = scipy_linalg.qr(C, mode="economic", pivoting=True)
    Qr, Rr, _ = scipy_linalg.qr(R.T, mode="economic", pivoting=True)
    Pc, Pr = Qc[:, :r] @ Qc[:, :r].T, Qr[:, :r] @ Qr[:, :r].T
    proj = Pc @ M @ Pr
    lra = out.S @ np.diag(out.sigma) @ out.Tt
    np.testing.assert_allclose(lra, proj, atol=1e-12 * sv[0])
    err = np.linalg.norm(M - lra, 2)
    bound = np.linalg.norm(Rc[r:, r:], 2) * np.linalg.norm(W @ R, 2) + \
        np.linalg.norm(C @ W, 2) * np.linalg.norm(Rr[r:, r:], 2)
    assert sv[r] * (1 - 1e-9) <= err <= bound * (1 + 1e-9), (sv[r], err, bound)
    np.testing.assert_allclose(out.sigma, np.linalg.svd(proj, compute_uv=False)[:r], rtol=1e-10)


def test_rank_loss_of_a_zero_column_block():
    C, W, R = _factors(7, 100, 90, 6, scales=False)
    C[:, 3:] = 0.0
    assert top_svd(C, W, R, 3).status == 0
    assert top_svd(C, W, R, 4).status == -2


@pytest.mark.parametrize("seed", range(2))
def test_after_ca_cur(seed):
    m, n, r = 512, 384, 8
    A, d = synth.rect_factor_gaussian(seed, m, n, r, 1e-7, r)
    res = oracle.ca_cur(oracle.dense(A), r, 3, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    assert res.status == 0
    C, R = A[:, res.J], A[res.I, :]
    cur = C @ res.U @ R
    out = top_svd(C, res.U, R, r)
    assert out.status == 0
    svd_lra = out.S @ np.diag(out.sigma) @ out.Tt
    e_cur, e_svd = np.linalg.norm(A - cur), np.linalg.norm(A - svd_lra)
    # r = k: the same LRA in another form
    assert e_svd == pytest.approx(e_cur, rel=1e-6)
    np.testing.assert_allclose(svd_lra, cur, atol=1e-10 * np.abs(A).max())
    np.testing.assert_allclose(out.sigma, np.linalg.svd(cur, compute_uv=False)[:r], rtol=1e-9)


@pytest.mark.parametrize("seed", range(3))
def test_oversampled_ca_cur_truncated(seed):
    """C-A at k = 10 on a rank-6 + noise matrix, then the rank-6 top SVD of
    its CUR: the truncation keeps the CUR's accuracy (an error within twice
    the CUR's plus a few sigma_7 of A)."""
    m, n, r, k = 512, 384, 6, 10
    A, d = synth.rect_factor_gaussian(seed, m, n, r, 1e-7, k)
    res = oracle.ca_cur(oracle.dense(A), k, 3, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    assert res.status == 0
    C, R = A[:, res.J], A[res.I, :]
    out = top_svd(C, res.U, R, r)
    assert out.status == 0
    sv = np.linalg.svd(A, compute_uv=False)
    e_cur = np.linalg.norm(A - C @ res.U @ R, 2)
    e_svd = np.linalg.norm(A - out.S @ np.diag(out.sigma) @ out.Tt, 2)
    assert sv[r] <= e_svd <= 2 * e_cur + 10 * sv[r], (e_svd, e_cur, sv[r])
    np.testing.assert_allclose(out.sigma, sv[:r], rtol=1e-3)
