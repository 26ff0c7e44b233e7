"""Pins for the CPU oracle: each check ties the oracle to something other than
itself -- a library routine, a closed form, brute force, a bound proved in the
paper, or a value the paper (or a published generator) prints.

Coverage (every oracle function is pinned; none is "parity unpinned"):

* oracle_entry_f64 / _f32  -- bitwise against numpy IEEE division.
* oracle_gepp_basis        -- pivot rows equal LAPACK getrf's; basis equals a
                              LAPACK solve; B[I,:] = I exactly.
* oracle_maxvol            -- stopping invariant max|B| <= 1+tau; final basis
                              equals C C[I,:]^{-1} re-solved by LAPACK (pins
                              the swap update); every single swap changes the
                              volume by |B_ic| (determinants); brute force
                              over all subsets (Hadamard bound, planted
                              maximum, Cauchy closed form); bound (eqfuge);
                              warm start falling back to the LU start on a
                              singular or numerically singular C[I,:]
                              equals the cold start.
* oracle_nucleus           -- U G = I and G = A[I,J] against numpy.
* oracle_residual          -- full sample equals the exact ||A - CUR||_F;
                              subsampled estimate within [0.5, 2] of it.
* oracle_ca_cur            -- exact rank-k reproduction (Section 6.5, CUR
                              decomposition; Theorem commhfg (i)); Eckart-Young
                              lower bound (Lemma letrnc); nucleus bound
                              (eqsvdtocur); det monotone across steps; the
                              delta-matrices of Appendix E.
* oracle_splitmix64        -- the published SplitMix64 outputs.
"""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _vol(M):
    return abs(np.linalg.det(M))


# ---------------------------------------------------------------------------
# entries
# ---------------------------------------------------------------------------

def test_entries_bitwise():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, 50)
    y = rng.uniform(2, 3, 40)
    src = oracle.cauchy(x, y)
    for i, j in [(0, 0), (7, 13), (49, 39)]:
        assert oracle.entry(src, i, j) == 1.0 / (x[i] - y[j])
        assert oracle.entry(src, i, j, "f32") == np.float32(1.0) / np.float32(x[i] - y[j])
    src2 = oracle.invdist(x, x)
    assert oracle.entry(src2, 3, 3) == 0.0
    assert oracle.entry(src2, 3, 5) == 1.0 / abs(x[3] - x[5])
    A = rng.standard_normal((6, 9)).astype(np.float32)
    for cm in (False, True):
        s = oracle.dense(A, col_major=cm)
        assert oracle.entry(s, 4, 7) == float(A[4, 7])


# ---------------------------------------------------------------------------
# partial-pivot LU start
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(5))
def test_gepp_pivots_match_lapack(seed):
    rng = np.random.default_rng(seed)
    m, k = 200, 12
    C = rng.standard_normal((m, k))
    keff, I, B, _ = oracle.gepp_basis(C)
    assert keff == k
    lu, piv = sla.lu_factor(C)
    perm = np.arange(m)
    for t, p in enumerate(piv[:k]):
        perm[t], perm[p] = perm[p], perm[t]
    np.testing.assert_array_equal(I, perm[:k])
    np.testing.assert_array_equal(B[I, :], np.eye(k))
    ref = np.linalg.solve(C[I, :].T, C.T).T
    kappa = np.linalg.cond(C[I, :])
    assert np.abs(B - ref).max() <= 10 * k * kappa * 2.0 ** -53 * max(1.0, np.abs(ref).max())


def test_gepp_rank_deficient():
    rng = np.random.default_rng(1)
    G = rng.standard_normal((100, 3))
    C = G @ rng.standard_normal((3, 6))  # rank 3, six columns
    keff, I, B, _ = oracle.gepp_basis(C)
    assert keff == 3
    Z = np.zeros((50, 4))
    keff, _, _, _ = oracle.gepp_basis(Z)
    assert keff == -1


# ---------------------------------------------------------------------------
# maxvol
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_maxvol_invariant_and_basis(seed, precision):
    rng = np.random.default_rng(seed)
    m, k, tau = 300, 10, 0.01
    C = rng.standard_normal((m, k)) * np.exp(rng.uniform(-2, 2, k))[None, :]
    out = oracle.maxvol(C, tau=tau, precision=precision)
    I, B = out["I"], out["B"]
    assert out["k_eff"] == k and not out["capped"]
    assert len(set(I.tolist())) == k
    # the stopping invariant: every |C C[I,:]^{-1}| entry is at most 1 + tau
    ref = np.linalg.solve(C[I, :].T, C.T).T
    tol = 1e-9 if precision == "f64" else 2e-3
    assert np.abs(ref).max() <= 1 + tau + tol
    # the swap updates left exactly the basis of the final set
    assert np.abs(B - ref).max() <= tol
    assert (np.asarray(B[I, :]) == np.eye(k)).all()


@pytest.mark.parametrize("seed", range(4))
def test_maxvol_single_swap_volume_ratio(seed):
    """|det C[I',:]| / |det C[I,:]| = |B_ic| for I' = I with slot c replaced by
    row i, so no single swap raises the volume above 1 + tau at the end."""
    rng = np.random.default_rng(seed + 10)
    m, k, tau = 40, 4, 0.05
    C = rng.standard_normal((m, k))
    out = oracle.maxvol(C, tau=tau)
    I = out["I"]
    v0 = _vol(C[I, :])
    worst = 0.0
    for i in range(m):
        if i in I:
            continue
        for c in range(k):
            I2 = I.copy()
            I2[c] = i
            ratio = _vol(C[I2, :]) / v0
            assert abs(ratio - abs(out["B"][i, c])) <= 1e-9 * max(1.0, ratio)
            worst = max(worst, ratio)
    assert worst <= 1 + tau + 1e-9


@pytest.mark.parametrize("seed", range(8))
def test_maxvol_brute_force_hadamard(seed):
    """vol(maxvol) >= vol_max / ((1 + tau) sqrt(k))^k (Hadamard's inequality on
    B[S*,:], whose entries are bounded by 1 + tau)."""
    rng = np.random.default_rng(seed + 100)
    m, k, tau = 11, 3, 0.01
    C = rng.standard_normal((m, k))
    out = oracle.maxvol(C, tau=tau)
    vmax = max(_vol(C[list(S), :]) for S in itertools.combinations(range(m), k))
    v = _vol(C[out["I"], :])
    assert v >= vmax / ((1 + tau) * math.sqrt(k)) ** k * (1 - 1e-12)
    assert v <= vmax * (1 + 1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_maxvol_planted_maximum(seed):
    rng = np.random.default_rng(seed + 200)
    m, k = 12, 4
    C = rng.standard_normal((m, k))
    target = rng.choice(m, k, replace=False)
    C[target, :] *= 100.0
    vols = {S: _vol(C[list(S), :]) for S in itertools.combinations(range(m), k)}
    best = max(vols, key=vols.get)
    second = sorted(vols.values())[-2]
    if vols[best] < 5 * second or set(best) != set(target.tolist()):
        pytest.skip("planted subset is not a clear unique maximum for this draw")
    out = oracle.maxvol(C, tau=0.01)
    assert set(out["I"].tolist()) == set(best)


def test_maxvol_cauchy_closed_form():
    """Cauchy determinant det[1/(s_i - t_j)] = prod_{i<j}(s_j - s_i)(t_i - t_j) /
    prod_{i,j}(s_i - t_j) gives every subset's volume without factorising."""
    rng = np.random.default_rng(5)
    m, k, tau = 10, 3, 0.01
    s = np.sort(rng.uniform(0, 1, m))
    t = rng.uniform(2, 3, k)
    C = 1.0 / (s[:, None] - t[None, :])

    def cdet(rows):
        ss = s[list(rows)]
        num = 1.0
        for a in range(k):
            for b in range(a + 1, k):
                num *= (ss[b] - ss[a]) * (t[a] - t[b])
        den = np.prod(ss[:, None] - t[None, :])
        return abs(num / den)

    vols = {S: cdet(S) for S in itertools.combinations(range(m), k)}
    for S in list(vols)[:20]:
        assert abs(vols[S] - _vol(C[list(S), :])) <= 1e-9 * vols[S]
    out = oracle.maxvol(C, tau=tau)
    vmax = max(vols.values())
    v = cdet(tuple(sorted(out["I"].tolist())))
    assert v >= vmax / ((1 + tau) * math.sqrt(k)) ** k


@pytest.mark.parametrize("seed", range(4))
def test_maxvol_eqfuge_bound(seed):
    """(eqfuge), Theorem thst3 with t_{m,r,h} of (eqtqsh): for orthonormal Q
    spanning the strip, ||Q[I,:]^{-1}||^2 <= (m - k) k h^2 + 1, h = 1 + tau."""
    rng = np.random.default_rng(seed + 300)
    m, k, tau = 500, 8, 0.01
    C = rng.standard_normal((m, k)) @ rng.standard_normal((k, k))
    Q, _ = np.linalg.qr(C)
    out = oracle.maxvol(Q, tau=tau)
    nrm = np.linalg.norm(np.linalg.inv(Q[out["I"], :]), 2)
    assert nrm ** 2 <= (m - k) * k * (1 + tau) ** 2 + 1
    # basis invariance: same set from C and from Q when started from the same set
    out_c = oracle.maxvol(C, tau=tau, init=out["I"])
    assert out_c["swaps"] == 0
    np.testing.assert_array_equal(out_c["I"], out["I"])


def test_maxvol_warm_fixed_point_and_cap():
    rng = np.random.default_rng(9)
    C = rng.standard_normal((200, 6))
    out = oracle.maxvol(C, tau=0.01)
    again = oracle.maxvol(C, tau=0.01, init=out["I"])
    assert again["swaps"] == 0
    np.testing.assert_array_equal(again["I"], out["I"])
    if out["swaps"] > 1:
        capped = oracle.maxvol(C, tau=0.01, max_swaps=1)
        assert capped["capped"] and capped["swaps"] == 1


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_maxvol_warm_fallback_equals_cold_start(precision):
    """A warm start whose C[I,:] is singular (two equal strip rows in I) or
    numerically singular (rows equal up to far less than 64 u max|C|) fails the
    rank test of its elimination, so the step restarts from the partial-pivot
    LU of the whole strip: the result is exactly the cold start's.  The
    decision's margin |pivot - thresh| / thresh is recorded."""
    rng = np.random.default_rng(21)
    m, k = 150, 6
    C = rng.standard_normal((m, k))
    C[40] = C[17]
    u = 2.0 ** -53 if precision == "f64" else 2.0 ** -24
    C[77] = C[23]
    C[77, 2] += 1e-3 * u * np.abs(C).max()
    if precision == "f32":
        C = C.astype(np.float32).astype(np.float64)
        C[77] = C[23]
    cold = oracle.maxvol(C, tau=0.01, precision=precision)
    for init in ([17, 40, 3, 5, 8, 9], [23, 1, 77, 5, 8, 9]):
        warm = oracle.maxvol(C, tau=0.01, init=init, precision=precision)
        np.testing.assert_array_equal(warm["I"], cold["I"])
        np.testing.assert_array_equal(warm["B"], cold["B"])
        assert warm["swaps"] == cold["swaps"] and warm["k_eff"] == k
        assert warm["trace"].min_rank_margin <= 1.0
    # a well-conditioned start passes the test with a wide margin and no restart
    ok = oracle.maxvol(C, tau=0.01, init=cold["I"], precision=precision)
    assert ok["swaps"] == 0 and ok["trace"].min_rank_margin > 1e3
    np.testing.assert_array_equal(ok["I"], cold["I"])


def test_warm_start_margin_reaches_the_driver_trace():
    """In a whole run, warm starts happen from the second step on; their rank
    tests feed the same margin as the first step's LU, so the driver's
    min_rank_margin is the smaller of the two kinds."""
    A, d = synth.plain_fp64(6)
    cold_only = oracle.ca_cur(oracle.dense(A), 8, 1, 0.0, d.cand_cols, d.sample_rows, d.sample_cols,
                              warm_start=False)
    warm = oracle.ca_cur(oracle.dense(A), 8, 3, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    assert np.isfinite(warm.trace["min_rank_margin"])
    assert warm.trace["min_rank_margin"] <= cold_only.trace["min_rank_margin"]


def test_tol_margin_recorded():
    """The stop-or-grow decision of each rank level compares est_rel with tol;
    its margin |est_rel - tol| / tol is recorded (one level here)."""
    A, d = synth.plain_fp64(3)
    tol = 1e-6
    r = oracle.ca_cur(oracle.dense(A), 8, 3, tol, d.cand_cols, d.sample_rows, d.sample_cols, k_max=16)
    assert r.status == 0 and r.k == 8
    assert r.trace["min_tol_margin"] == abs(r.err_est_rel - tol) / tol
    r0 = oracle.ca_cur(oracle.dense(A), 8, 3, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    assert r0.trace["min_tol_margin"] == float("inf")


# ---------------------------------------------------------------------------
# nucleus and residual
# ---------------------------------------------------------------------------

def test_nucleus_against_numpy():
    A, d = synth.plain_fp64(4)
    src = oracle.dense(A)
    rng = np.random.default_rng(0)
    I = rng.choice(512, 8, replace=False)
    J = rng.choice(512, 8, replace=False)
    rc, G, U, cond = oracle.nucleus(src, I, J)
    assert rc == 0
    np.testing.assert_array_equal(G, A[np.ix_(I, J)])
    np.testing.assert_allclose(U @ G, np.eye(8), atol=1e-9 * np.linalg.cond(G) * 1e-3 + 1e-10)
    assert abs(cond - np.linalg.norm(G, 1) * np.linalg.norm(np.linalg.inv(G), 1)) <= 1e-6 * cond


def test_residual_full_sample_is_exact():
    A, d = synth.plain_fp64(2)
    src = oracle.dense(A)
    r = oracle.ca_cur(src, 8, 3, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    allr = np.arange(512)
    e = oracle.residual(src, r.I, r.J, allr, allr)
    E = A - A[:, r.J] @ r.U @ A[r.I, :]
    assert abs(e["norm_e"] - np.linalg.norm(E)) <= 1e-6 * np.linalg.norm(E)
    assert abs(e["est_abs"] - np.linalg.norm(E)) <= 1e-6 * np.linalg.norm(E)
    assert abs(e["norm_a"] - np.linalg.norm(A)) <= 1e-12 * np.linalg.norm(A)
    assert abs(e["mean"] - E.mean()) <= 1e-6 * np.abs(E).max()
    assert abs(e["var"] - E.var()) <= 1e-5 * E.var()


def test_residual_estimate_unbiased_range():
    ratios = []
    for seed in range(20):
        A, d = synth.plain_fp64(seed)
        src = oracle.dense(A)
        r = oracle.ca_cur(src, 8, 3, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
        E = A - A[:, r.J] @ r.U @ A[r.I, :]
        ratios.append(r.err_est_abs / np.linalg.norm(E))
    ratios = np.array(ratios)
    assert ((ratios > 0.5) & (ratios < 2.0)).all()
    assert 0.8 < np.mean(ratios ** 2) < 1.25


# ---------------------------------------------------------------------------
# whole C-A runs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(5))
def test_exact_rank_reproduction_and_nucleus_bound(seed):
    """A of rank k: CUR with a nonsingular generator is exact (Section 6.5 and
    Theorem commhfg (i)); ||U|| <= t_{m,k,h} t_{n,k,h} / sigma_k (eqsvdtocur)."""
    m, n, k, tau = 300, 260, 6, 0.01
    A, d = synth.rect_factor_gaussian(seed, m, n, k, 0.0, k)
    src = oracle.dense(A)
    r = oracle.ca_cur(src, k, 2, 0.0, d.cand_cols, d.sample_rows, d.sample_cols, tau=tau)
    assert r.status == 0 and r.k == k
    E = A - A[:, r.J] @ r.U @ A[r.I, :]
    assert np.linalg.norm(E) / np.linalg.norm(A) <= 1e-12
    sig = np.linalg.svd(A, compute_uv=False)
    h = 1 + tau
    t_m = math.sqrt((m - k) * k * h * h + 1)
    t_n = math.sqrt((n - k) * k * h * h + 1)
    assert np.linalg.norm(r.U, 2) <= t_m * t_n / sig[k - 1] * (1 + 1e-9)


@pytest.mark.parametrize("seed", range(10))
def test_eckart_young_lower_bound(seed):
    A, d = synth.plain_fp64(seed)
    src = oracle.dense(A)
    r = oracle.ca_cur(src, 8, 3, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    sig = np.linalg.svd(A, compute_uv=False)
    eps_svd = math.sqrt((sig[8:] ** 2).sum()) / np.linalg.norm(A)
    E = A - A[:, r.J] @ r.U @ A[r.I, :]
    eps_cur = np.linalg.norm(E) / np.linalg.norm(A)
    assert eps_cur >= eps_svd * (1 - 1e-9)
    assert eps_cur <= 20 * eps_svd
    assert r.status == 0 and r.sweeps_done == 3


def test_volume_monotone_across_steps():
    """Warm-started steps never decrease |det A[I,J]|."""
    A, d = synth.plain_fp64(11, eps=1e-3)
    J = d.cand_cols.copy()
    I = None
    vols = []
    for _ in range(4):
        out = oracle.maxvol(A[:, J], tau=0.01, init=I)
        I = out["I"]
        vols.append(_vol(A[np.ix_(I, J)]))
        out = oracle.maxvol(A[I, :].T, tau=0.01, init=J)
        J = out["I"]
        vols.append(_vol(A[np.ix_(I, J)]))
    for a, b in zip(vols[1:], vols[2:]):
        assert b >= a * (1 - 1e-12)


def test_ca_cur_matches_manual_steps():
    """The driver is the alternation of maxvol steps plus the nucleus."""
    A, d = synth.plain_fp64(12, eps=1e-4)
    src = oracle.dense(A)
    r = oracle.ca_cur(src, 8, 3, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    J = d.cand_cols.copy()
    I = None
    for _ in range(3):
        I = oracle.maxvol(A[:, J], tau=0.01, init=I)["I"]
        J = oracle.maxvol(A[I, :].T, tau=0.01, init=J)["I"]
    np.testing.assert_array_equal(r.I, I)
    np.testing.assert_array_equal(r.J, J)
    np.testing.assert_allclose(r.U, np.linalg.inv(A[np.ix_(I, J)]), rtol=1e-9, atol=1e-12)


def test_col_major_source_same_result():
    A, d = synth.plain_fp64(13)
    r1 = oracle.ca_cur(oracle.dense(A), 8, 3, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    r2 = oracle.ca_cur(oracle.dense(A, col_major=True), 8, 3, 0.0, d.cand_cols, d.sample_rows,
                       d.sample_cols)
    np.testing.assert_array_equal(r1.I, r2.I)
    np.testing.assert_array_equal(r1.J, r2.J)
    assert r1.err_est_rel == r2.err_est_rel


def test_adaptive_rank_cauchy():
    """Cauchy kernel on nearly touching intervals: the rank grows from 8 until
    the sampled relative error meets tol; the true error agrees."""
    rng = np.random.default_rng(0)
    s = rng.uniform(0, 1, 3000)
    t = rng.uniform(1.01, 2.01, 2500)
    cand = rng.choice(2500, 80, replace=False)
    Q, S = synth.residual_sample(3000, 2500, 0)
    src = oracle.cauchy(s, t)
    r = oracle.ca_cur(src, 8, 4, 1e-10, cand, Q, S, k_max=40)
    assert r.status in (0, 3)
    assert r.k > 8
    assert r.err_est_rel <= 1e-10
    A = 1.0 / (s[:, None] - t[None, :])
    G = A[np.ix_(r.I, r.J)]
    E = A - A[:, r.J] @ np.linalg.solve(G, A[r.I, :])
    assert np.linalg.norm(E) / np.linalg.norm(A) <= 1e-9
    r8 = oracle.ca_cur(src, 8, 4, 0.0, cand, Q, S)
    assert r8.err_est_rel > 1e-10  # rank 8 alone is not enough


@pytest.mark.parametrize("seed", range(2))
def test_adaptive_rank_known_spectrum(seed):
    """A = U diag(sigma) V^T with sigma_j = 10^(-j/8): the rank grows by whole
    steps of 8 until the sampled error meets tol, and at every level the true
    CUR error is bounded below by the Eckart-Young optimum, known here in
    closed form from sigma (Lemma letrnc), and above by a small multiple."""
    m, n = 3000, 2500
    A, d = synth.spectrum_dense(seed, m, n, decay=8.0)
    sig = 10.0 ** (-np.arange(160) / 8.0)
    tol = 1e-3
    r = oracle.ca_cur(oracle.dense(A), 8, 4, tol, d.cand_cols, d.sample_rows, d.sample_cols, k_max=40)
    assert r.status == 0 and r.k == 32 and r.err_est_rel <= tol
    for k in (8, 16, 24, 32):
        rk = oracle.ca_cur(oracle.dense(A), k, 4, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
        G = A[np.ix_(rk.I, rk.J)]
        E = A - A[:, rk.J] @ np.linalg.solve(G, A[rk.I, :])
        eps = np.linalg.norm(E) / np.linalg.norm(A)
        eps_svd = math.sqrt((sig[k:] ** 2).sum() / (sig ** 2).sum())
        assert eps_svd * (1 - 1e-6) <= eps <= 20 * eps_svd, (k, eps, eps_svd)
        # a level below 32 misses tol, which is why the rank grew past it
        assert (rk.err_est_rel > tol) == (k < 32), (k, rk.err_est_rel)


def test_tol_not_met_at_cap():
    A, d = synth.rect_factor_gaussian(1, 200, 200, 30, 1e-3, 8, n_cand=16)
    r = oracle.ca_cur(oracle.dense(A), 8, 2, 1e-12, d.cand_cols, d.sample_rows, d.sample_cols,
                      k_max=16)
    assert r.status == 1 and r.k == 16


def test_delta_matrices_appendix_e():
    """Appendix E: a superfast method sees a delta-matrix only if it samples
    its nonzero.  k = 1 from either start column: exact CUR or exact rank loss."""
    rows = np.loadtxt(os.path.join(GOLDEN, "delta_2x2.txt"))
    for row in rows:
        A = row.reshape(2, 2)
        for j0 in range(2):
            r = oracle.ca_cur(oracle.dense(A), 1, 1, 0.0, [j0], [0, 1], [0, 1])
            if A[:, j0].any():
                assert r.status == 0
                E = A - A[:, r.J] @ r.U @ A[r.I, :]
                assert np.abs(E).max() == 0.0
            else:
                assert r.status == -2
    # a large delta-matrix whose spike is never sampled: rank loss is reported
    A = np.zeros((512, 512))
    A[300, 17] = 1.0
    r = oracle.ca_cur(oracle.dense(A), 2, 2, 0.0, [5, 9], [0, 1], [0, 1])
    assert r.status == -2


def test_dependent_column_reduces_rank():
    """The first step's LU takes the strip's columns in slot order: a
    dependent column leaves no usable pivot, so the rank drops to the pivots
    before it with NUMERICAL_RANK, whether rounding leaves that column exactly
    zero or not; only a zero strip is FAILURE."""
    rng = np.random.default_rng(4)
    A = rng.standard_normal((60, 40))
    A[:, 7] = A[:, 3]
    A[:, 11] = 2.0 * A[:, 5]
    for prec in ("f64", "f32"):
        Ap = A.astype(np.float64 if prec == "f64" else np.float32)
        r = oracle.ca_cur(oracle.dense(Ap), 5, 1, 0.0, [3, 5, 0, 7, 11], np.arange(60), np.arange(40),
                          precision=prec)
        assert r.status == 3 and r.k == 3, (prec, r.status, r.k)
        # the three surviving columns are independent ones
        assert len({3, 7} & set(r.J.tolist())) <= 1 and len({5, 11} & set(r.J.tolist())) <= 1
        r = oracle.ca_cur(oracle.dense(Ap), 5, 1, 0.0, [3, 7, 5, 11, 0], np.arange(60), np.arange(40),
                          precision=prec)
        assert r.status == 3 and r.k == 1, (prec, r.status, r.k)


def test_nonfinite_entry_reported():
    A, d = synth.plain_fp64(1)
    A = A.copy()
    A[10, d.cand_cols[0]] = np.nan
    r = oracle.ca_cur(oracle.dense(A), 8, 1, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
    assert r.status == -6


def test_splitmix64_published_outputs():
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    assert [oracle.splitmix64(0, i) for i in range(3)] == vals
    dd = oracle.draw_distinct(5, 37, 37)
    assert sorted(dd.tolist()) == list(range(37))
