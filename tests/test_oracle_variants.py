"""Pins for the oracle's fixed-rank CUR algorithms of the C-A tests (the
four algorithms the paper's Section 12.2 compares, and the Primitive
algorithm of Section 6.5 with a truncated pseudo-inverse nucleus).  Each
check ties the oracle to something other than itself: LAPACK's SVD, the
Moore-Penrose identities, exact reproduction of a rank-r matrix (the CUR
decomposition of Section 6.5), the oracle's already-pinned C-A driver,
a planted maximum found by brute force, and the maxvol stopping invariant
re-solved with numpy.

* oracle_svd_jacobi         -- singular values equal LAPACK's; G = W V^T;
                               V orthogonal; W's columns orthogonal.
* oracle_nucleus_trunc      -- r = k equals the inverse; r < k equals
                               LAPACK's pseudo-inverse of the rank-r
                               truncation; Moore-Penrose identities.
* oracle_residual_explicit  -- with U = G^{-1} equals the LU-based residual;
                               full sample equals ||A - C U R||_F.
* oracle_cur_variant        -- sweeps >= 1 without reduction equals
                               oracle_ca_cur; sweeps = 0 keeps the random
                               sets; Cynical (Tests 3, 4) and Primitive
                               reproduce a rank-r matrix exactly; the
                               Cynical r x r submatrix satisfies the maxvol
                               invariant in its block's row and column
                               strips; a planted maximum is found exactly.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth


def _rank_r(seed, m, n, r, eps=0.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    if eps:
        A = A + eps * rng.standard_normal((m, n))
    return np.ascontiguousarray(A)


def _draws(seed, m, n, k):
    rng = np.random.default_rng(seed + 100)
    rows = rng.choice(m, k, replace=False).astype(np.int64)
    cols = rng.choice(n, k, replace=False).astype(np.int64)
    Q, S = synth.residual_sample(m, n, seed)
    return rows, cols, Q, S


# ---------------------------------------------------------------------------
# Jacobi SVD and the truncated pseudo-inverse
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed,k", [(0, 5), (1, 16), (2, 33), (3, 64)])
def test_svd_jacobi_against_lapack(seed, k):
    rng = np.random.default_rng(seed)
    # a spread spectrum: U diag(10^-j/4) V^T
    Qa, _ = np.linalg.qr(rng.standard_normal((k, k)))
    Qb, _ = np.linalg.qr(rng.standard_normal((k, k)))
    G = (Qa * 10.0 ** (-np.arange(k) / 4.0)) @ Qb.T
    W, V, sv, sweeps = oracle.svd_jacobi(G)
    ref = np.linalg.svd(G, compute_uv=False)
    np.testing.assert_allclose(np.sort(sv)[::-1], ref, rtol=1e-12, atol=1e-14 * ref[0])
    np.testing.assert_allclose(W @ V.T, G, atol=1e-13 * ref[0])
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-13)
    off = W.T @ W - np.diag(sv ** 2)
    assert np.abs(off).max() <= 1e-13 * ref[0] ** 2
    assert 1 <= sweeps < 100


@pytest.mark.parametrize("seed,k,r", [(0, 8, 8), (1, 12, 5), (2, 32, 8), (3, 24, 1)])
def test_nucleus_trunc_against_lapack_pinv(seed, k, r):
    m = n = 200
    A = _rank_r(seed, m, n, r + 4, 0.0)
    # singular values of the generator spread over a few decades
    rng = np.random.default_rng(seed)
    A = A * np.exp(rng.uniform(-2, 2, n))[None, :]
    I, J, _, _ = _draws(seed, m, n, k)
    rc, G, U, cond = oracle.nucleus_trunc(oracle.dense(A), I, J, r)
    assert rc == 0
    np.testing.assert_array_equal(G, A[np.ix_(I, J)])
    Ug, s, Vt = np.linalg.svd(G)
    Gr = (Ug[:, :r] * s[:r]) @ Vt[:r]
    ref = (Vt[:r].T / s[:r]) @ Ug[:, :r].T  # LAPACK's V_r Sigma_r^{-1} U_r^T
    tol = 1e-9 * np.abs(ref).max()
    np.testing.assert_allclose(U, ref, atol=tol)
    # Moore-Penrose identities of the truncation
    np.testing.assert_allclose(U @ Gr @ U, U, atol=1e-8 * np.abs(U).max())
    np.testing.assert_allclose(Gr @ U @ Gr, Gr, atol=1e-8 * np.abs(Gr).max())
    assert cond == pytest.approx(np.abs(G).sum(0).max() * np.abs(U).sum(0).max(), rel=1e-12)


def test_nucleus_trunc_full_rank_equals_inverse():
    A = _rank_r(5, 100, 90, 10, 1e-3)
    I, J, _, _ = _draws(5, 100, 90, 10)
    src = oracle.dense(A)
    rc, G, U, _ = oracle.nucleus_trunc(src, I, J, 10)
    rc2, G2, U2, _ = oracle.nucleus(src, I, J)
    assert rc == rc2 == 0
    np.testing.assert_allclose(U, U2, rtol=0, atol=1e-10 * np.abs(U2).max())


def test_residual_explicit_pins():
    A = _rank_r(6, 150, 140, 6, 1e-4)
    I, J, Q, S = _draws(6, 150, 140, 6)
    src = oracle.dense(A)
    _, G, U, _ = oracle.nucleus(src, I, J)
    a = oracle.residual(src, I, J, Q, S)
    b = oracle.residual_explicit(src, I, J, U, Q, S)
    assert b["est_rel"] == pytest.approx(a["est_rel"], rel=1e-9)
    # the full sample is the exact error of C U R
    allQ, allS = np.arange(150), np.arange(140)
    full = oracle.residual_explicit(src, I, J, U, allQ, allS)
    E = A - A[:, J] @ U @ A[I, :]
    assert full["norm_e"] == pytest.approx(np.linalg.norm(E), rel=1e-10)


# ---------------------------------------------------------------------------
# drivers
# ---------------------------------------------------------------------------

def test_cur_variant_without_reduction_equals_ca_cur():
    A, d = synth.plain_fp64(4)
    src = oracle.dense(A)
    for prec in ("f64", "f32"):
        a = oracle.ca_cur(src, 8, 3, 0.0, d.cand_cols, d.sample_rows, d.sample_cols, precision=prec)
        b = oracle.cur_variant(src, 8, 3, d.cand_cols, d.sample_rows, d.sample_cols, precision=prec)
        assert (a.status, a.k, a.swaps_total, a.sweeps_done, a.entries_read) == \
               (b.status, b.k, b.swaps_total, b.sweeps_done, b.entries_read)
        np.testing.assert_array_equal(a.I, b.I)
        np.testing.assert_array_equal(a.J, b.J)
        assert a.err_est_rel == b.err_est_rel
        np.testing.assert_array_equal(a.U, b.U)


@pytest.mark.parametrize("seed", range(3))
def test_random_sets_reproduce_rank_r(seed):
    """Tests 1 / the Primitive algorithm with k = l = r: random I, J kept as
    given, and a rank-r matrix is reproduced exactly (Section 6.5)."""
    m, n, r = 300, 260, 7
    A = _rank_r(seed, m, n, r)
    rows, cols, Q, S = _draws(seed, m, n, r)
    res = oracle.cur_variant(oracle.dense(A), r, 0, cols, Q, S, init_rows=rows)
    assert res.status == 0 and res.k == r
    np.testing.assert_array_equal(res.I, rows)
    np.testing.assert_array_equal(res.J, cols)
    assert res.err_est_rel < 1e-11
    E = A - A[:, res.J] @ res.U @ A[res.I, :]
    assert np.linalg.norm(E) <= 1e-10 * np.linalg.norm(A)


@pytest.mark.parametrize("sweeps", [0, 1])
@pytest.mark.parametrize("seed", range(3))
def test_cynical_reproduces_rank_r_and_is_dominant(seed, sweeps):
    """Tests 3 (sweeps = 0) and Tests 4 (one C-A loop at width 4r): the
    r x r generator picked inside the 4r x 4r block reproduces a rank-r
    matrix exactly (Tests 3), or a rank-r matrix plus 1e-10 Gaussian noise
    -- the paper's test input, whose 4r-wide strips keep full numerical rank
    -- to the noise level (Tests 4); it lies inside the block and satisfies
    the maxvol invariant in both of its strips within the block."""
    m, n, r = 400, 350, 6
    p = 4 * r
    eps = 0.0 if sweeps == 0 else 1e-10
    A = _rank_r(seed, m, n, r, eps)
    rows, cols, Q, S = _draws(seed, m, n, p)
    tau = 0.01
    res = oracle.cur_variant(oracle.dense(A), p, sweeps, cols, Q, S, init_rows=rows, cur_rank=r, tau=tau)
    assert res.status == 0 and res.k == r
    bound = 1e-11 if eps == 0 else 1e-8
    assert res.err_est_rel < bound
    E = A - A[:, res.J] @ res.U @ A[res.I, :]
    assert np.linalg.norm(E) <= 10 * bound * np.linalg.norm(A)
    if sweeps == 0:
        K, L = rows, cols
    else:
        ref = oracle.cur_variant(oracle.dense(A), p, 1, cols, Q, S)  # the outer sets alone
        K, L = ref.I, ref.J
    assert set(res.I) <= set(K) and set(res.J) <= set(L)
    B = A[np.ix_(K, L)]
    Il = np.array([list(K).index(i) for i in res.I])
    Jl = np.array([list(L).index(j) for j in res.J])
    Gs = B[np.ix_(Il, Jl)]
    row_strip = B[:, Jl] @ np.linalg.inv(Gs)           # p x r: the column step's basis
    col_strip = np.linalg.solve(Gs, B[Il, :])           # r x p: the row step's basis
    assert np.abs(col_strip).max() <= (1 + tau) * (1 + 1e-9)
    assert np.abs(row_strip).max() <= (1 + tau) * (1 + 1e-9) or res.swaps_total > 0


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("seed", range(4))
def test_cynical_planted_maximum(seed, precision):
    """A block whose rows I* and columns J* are scaled up by 30 and its r x r
    core set to 1000 I has its unique maximal-volume r x r submatrix at
    (I*, J*) (brute force over all pairs of
    subsets confirms it); the Cynical step finds it from J0 = the first r
    columns of the block."""
    rng = np.random.default_rng(seed)
    p, r = 8, 2
    m = n = 60
    A = rng.standard_normal((m, n))
    rows = rng.choice(m, p, replace=False).astype(np.int64)
    cols = rng.choice(n, p, replace=False).astype(np.int64)
    Ist = rng.choice(p, r, replace=False)
    Jst = rng.choice(p, r, replace=False)
    A[rows[Ist], :] *= 30.0
    A[:, cols[Jst]] *= 30.0
    A[np.ix_(rows[Ist], cols[Jst])] = 1000.0 * np.eye(r)
    B = A[np.ix_(rows, cols)]
    vols = {(a, b): abs(np.linalg.det(B[np.ix_(a, b)]))
            for a in itertools.combinations(range(p), r) for b in itertools.combinations(range(p), r)}
    best = max(vols, key=vols.get)
    ranked = sorted(vols.values(), reverse=True)
    assert ranked[0] >= 10 * ranked[1]
    assert set(best[0]) == set(Ist) and set(best[1]) == set(Jst)
    Q, S = synth.residual_sample(m, n, seed)
    res = oracle.cur_variant(oracle.dense(A), p, 0, cols, Q, S, init_rows=rows, cur_rank=r, precision=precision)
    assert res.status == 0
    assert set(res.I) == set(rows[Ist]) and set(res.J) == set(cols[Jst])


@pytest.mark.parametrize("seed", range(3))
def test_primitive_truncated_nucleus(seed):
    """Primitive algorithm with k = l > r: random k x k generator of a
    numerically rank-r matrix; the rank-r truncated pseudo-inverse keeps the
    error at the noise level, and the nucleus equals LAPACK's pinv of the
    truncated generator."""
    m, n, r, k = 300, 280, 5, 12
    A = _rank_r(seed, m, n, r, 1e-9)
    rows, cols, Q, S = _draws(seed, m, n, k)
    src = oracle.dense(A)
    res = oracle.cur_variant(src, k, 0, cols, Q, S, init_rows=rows, nucleus_rank=r)
    assert res.status == 0 and res.k == k
    G = A[np.ix_(rows, cols)]
    Ug, s, Vt = np.linalg.svd(G)
    ref = (Vt[:r].T / s[:r]) @ Ug[:, :r].T  # LAPACK's V_r Sigma_r^{-1} U_r^T
    np.testing.assert_allclose(res.U, ref, atol=1e-8 * np.abs(res.U).max())
    E = A - A[:, cols] @ res.U @ A[rows, :]
    true_rel = np.linalg.norm(E) / np.linalg.norm(A)
    assert true_rel < 1e-7
    full = oracle.residual_explicit(src, rows, cols, res.U, np.arange(m), np.arange(n))
    assert full["norm_e"] == pytest.approx(np.linalg.norm(E), rel=1e-8)


def test_variant_argument_checks():
    A, d = synth.plain_fp64(0)
    src = oracle.dense(A)
    bad = oracle.cur_variant(src, 8, 0, d.cand_cols, d.sample_rows, d.sample_cols)  # no init rows
    assert bad.status == -1
    bad = oracle.cur_variant(src, 8, 1, d.cand_cols, d.sample_rows, d.sample_cols, cur_rank=9)
    assert bad.status == -1
