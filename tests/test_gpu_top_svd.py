"""GPU parity of lra_top_svd (Appendix D, Algorithm D.1) against the oracle
(oracle/top_svd.py: Householder QR with column pivoting on the tall factors
themselves, LAPACK's SVD of the middle factor).

The GPU reduces each tall factor to a triangle by a TSQR tree before the
pivoted QR and solves with the kept triangle instead of forming Q, so the
comparison is by what is unique: the pivots wherever the oracle's pivot
margins are clear; sigma; the rank-r matrix S diag(sigma) T^T (unique given
the pivots); the singular vectors up to sign where the singular values are
separated; S and T orthonormal within the conditioning of the kept triangle.
Tolerances: 1e-10 relative to sigma_1 for sigma and the product (binary64
QR and Jacobi SVD of well-conditioned factors), orthogonality within
1e-13 kappa(R_C[:r,:r]).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle.top_svd import top_svd as oracle_top_svd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MARGIN = 1e-9


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_1611_01391_amd import lra
    c = lra.Context()
    yield c
    c.close()


def _factors(seed, m, n, k, scales=6.0, dtype=np.float64):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((m, k)) * np.exp(rng.uniform(-scales, 0, k))[None, :]
    R = rng.standard_normal((k, n)) * np.exp(rng.uniform(-scales, 0, k))[:, None]
    W = rng.standard_normal((k, k))
    return C.astype(dtype), W, R.astype(dtype)


def _dev(C, R):
    """C as an m x k column-major device view, R as k x n row-major."""
    Cd = torch.from_numpy(np.ascontiguousarray(C.T)).cuda().t()
    Rd = torch.from_numpy(np.ascontiguousarray(R)).cuda()
    return Cd, Rd


def _compare(got, ref, r, what):
    S, sigma, Tt, pc, pr = got
    S, Tt = S.cpu().numpy(), Tt.cpu().numpy()
    assert ref.status == 0, what
    clear_c = ref.margins_c[:r].min() >= MARGIN
    clear_r = ref.margins_r[:r].min() >= MARGIN
    if clear_c:
        np.testing.assert_array_equal(pc[:r], ref.piv_c[:r], err_msg=what)
    if clear_r:
        np.testing.assert_array_equal(pr[:r], ref.piv_r[:r], err_msg=what)
    assert np.all(np.diff(sigma) <= 0), what
    s1 = ref.sigma[0]
    np.testing.assert_allclose(sigma, ref.sigma, rtol=0, atol=1e-10 * s1, err_msg=what)
    if clear_c and clear_r:
        got_lra = S @ np.diag(sigma) @ Tt
        ref_lra = ref.S @ np.diag(ref.sigma) @ ref.Tt
        np.testing.assert_allclose(got_lra, ref_lra, rtol=0, atol=1e-10 * s1, err_msg=what)
        # singular vectors up to sign where sigma is separated
        gaps = np.minimum(np.r_[np.inf, -np.diff(ref.sigma)], np.r_[-np.diff(ref.sigma), ref.sigma[-1]])
        for a in range(r):
            if gaps[a] > 1e-6 * s1:
                sg = np.sign(S[:, a] @ ref.S[:, a])
                np.testing.assert_allclose(sg * S[:, a], ref.S[:, a], atol=1e-8 * s1 / gaps[a], err_msg=what)
    kappa = ref.rdiag_c[0] / ref.rdiag_c[r - 1]
    kappa_r = ref.rdiag_r[0] / ref.rdiag_r[r - 1]
    np.testing.assert_allclose(S.T @ S, np.eye(r), atol=max(1e-12, 1e-13 * kappa), err_msg=what)
    np.testing.assert_allclose(Tt @ Tt.T, np.eye(r), atol=max(1e-12, 1e-13 * kappa_r), err_msg=what)


@pytest.mark.parametrize("m,n,k,r", [(300, 250, 12, 12), (1000, 700, 32, 32), (700, 1000, 32, 10),
                                     (256, 256, 64, 64), (257, 511, 16, 5), (64, 64, 64, 30), (5000, 40, 8, 8),
                                     (70000, 3000, 16, 16), (100, 100, 1, 1)])
@pytest.mark.parametrize("seed", [0, 1])
def test_top_svd_vs_oracle(ctx, m, n, k, r, seed):
    _say(f"top svd m={m} n={n} k={k} r={r} seed={seed}")
    C, W, R = _factors(seed + 17 * k, m, n, k, scales=3.0)
    Cd, Rd = _dev(C, R)
    got = ctx.top_svd(Cd, W, Rd, r)
    ref = oracle_top_svd(C, W, R, r)
    _compare(got, ref, r, f"m={m} n={n} k={k} r={r}")


@pytest.mark.parametrize("seed", range(3))
def test_rank_r_exact_and_rank_loss(ctx, seed):
    from paper_1611_01391_amd import lra
    _say(f"top svd rank r exact seed={seed}")
    m, n, k, r = 900, 600, 16, 5
    rng = np.random.default_rng(100 + seed)
    C = rng.standard_normal((m, r)) @ rng.standard_normal((r, k))
    R = rng.standard_normal((k, r)) @ rng.standard_normal((r, n))
    W = rng.standard_normal((k, k))
    Cd, Rd = _dev(C, R)
    S, sigma, Tt, _, _ = ctx.top_svd(Cd, W, Rd, r)
    M = C @ W @ R
    sv = np.linalg.svd(M, compute_uv=False)
    np.testing.assert_allclose(S.cpu().numpy() @ np.diag(sigma) @ Tt.cpu().numpy(), M, atol=1e-11 * sv[0])
    np.testing.assert_allclose(sigma, sv[:r], rtol=1e-9)
    assert oracle_top_svd(C, W, R, r + 1).status == -2
    with pytest.raises(lra.LraError) as e:
        ctx.top_svd(Cd, W, Rd, r + 1)
    assert e.value.args[0].endswith(f"({lra.ERANK})")


@pytest.mark.parametrize("seed", range(2))
def test_noisy_projection(ctx, seed):
    """Rank-6 factors plus 1e-6 noise at r = 6: the two-sided projection on
    the kept subspaces, compared with the oracle's."""
    _say(f"top svd noisy projection seed={seed}")
    m, n, k, r = 4000, 3000, 16, 6
    rng = np.random.default_rng(200 + seed)
    C = rng.standard_normal((m, r)) @ rng.standard_normal((r, k)) + 1e-6 * rng.standard_normal((m, k))
    R = rng.standard_normal((k, r)) @ rng.standard_normal((r, n)) + 1e-6 * rng.standard_normal((k, n))
    W = rng.standard_normal((k, k))
    Cd, Rd = _dev(C, R)
    got = ctx.top_svd(Cd, W, Rd, r)
    ref = oracle_top_svd(C, W, R, r)
    _compare(got, ref, r, f"noisy {seed}")


def test_binary32_factors(ctx):
    """float32 factors are read exactly and processed in binary64."""
    _say("top svd binary32 factors")
    C, W, R = _factors(5, 2000, 1500, 24, scales=3.0, dtype=np.float32)
    Cd, Rd = _dev(C, R)
    got = ctx.top_svd(Cd, W, Rd, 24)
    ref = oracle_top_svd(C.astype(np.float64), W, R.astype(np.float64), 24)
    _compare(got, ref, 24, "binary32")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_after_ca_cur_dense_16384(ctx, precision):
    """The dense 16384 x 16384 float32 workload (k = 32, 4 sweeps, team 64):
    C-A on the GPU, its factors by lra_cur_factors, then the top SVD at
    r = 32 and r = 16 against the oracle's on the same factors."""
    from paper_1611_01391_amd import lra
    _say(f"top svd after C-A dense 16384 {precision}")
    A, d = synth.dense_scaled(0)
    At = torch.from_numpy(A).cuda()
    src = lra.dense(At)
    prec = lra.PREC_FP64 if precision == "fp64" else lra.PREC_MIXED
    res = ctx.ca_cur(src, 32, 4, 0.0, init_cols=d.cand_cols, sample_rows=d.sample_rows, sample_cols=d.sample_cols,
                     precision=prec, team_wgs=64)
    assert res.status == 0
    Cd, Rd = ctx.cur_factors(src, res.I, res.J)
    Ch, Rh = Cd.cpu().numpy().astype(np.float64), Rd.cpu().numpy().astype(np.float64)
    for r in (32, 16):
        got = ctx.top_svd(Cd, res.U, Rd, r)
        ref = oracle_top_svd(Ch, res.U, Rh, r)
        _compare(got, ref, r, f"dense 16384 {precision} r={r}")
    # r = k: the same LRA as the CUR, on sampled entries
    S, sigma, Tt, _, _ = ctx.top_svd(Cd, res.U, Rd, 32)
    rng = np.random.default_rng(1)
    ii, jj = rng.integers(0, 16384, 200), rng.integers(0, 16384, 200)
    Sh, Th = S.cpu().numpy(), Tt.cpu().numpy()
    lra_v = np.einsum("ia,a,ai->i", Sh[ii], sigma, Th[:, jj])
    cur_v = np.einsum("ia,ab,bi->i", Ch[ii], res.U, Rh[:, jj])
    np.testing.assert_allclose(lra_v, cur_v, rtol=0, atol=1e-9 * np.abs(A).max())


def test_strided_factors_and_outputs(ctx):
    """Leading dimensions above the row counts, through the C ABI: C inside a
    taller column-major buffer (ldc = m + 7), R inside a wider row-major one
    (ldr = n + 5), S and T^T written with padding (lds = m + 3, ldt = n + 9):
    the same bits as the packed call, and the padding untouched."""
    from paper_1611_01391_amd import lra
    _say("top svd strided")
    m, n, k, r = 1200, 900, 16, 10
    Cm, W, Rm = _factors(9, m, n, k, scales=3.0)
    Cd, Rd = _dev(Cm, Rm)
    S0, sg0, T0, pc0, pr0 = ctx.top_svd(Cd, W, Rd, r)
    ldc, ldr, lds, ldt = m + 7, n + 5, m + 3, n + 9
    Cbig = torch.zeros(k, ldc, dtype=torch.float64, device="cuda")
    Cbig[:, :m] = torch.from_numpy(np.ascontiguousarray(Cm.T)).cuda()
    Rbig = torch.zeros(k, ldr, dtype=torch.float64, device="cuda")
    Rbig[:, :n] = torch.from_numpy(Rm).cuda()
    Sb = torch.full((r, lds), 5.0, dtype=torch.float64, device="cuda")
    Tb = torch.full((r, ldt), 5.0, dtype=torch.float64, device="cuda")
    Wh = np.ascontiguousarray(W)
    sg = np.zeros(r)
    pc = np.zeros(k, dtype=np.int64)
    pr = np.zeros(k, dtype=np.int64)
    torch.cuda.synchronize()
    st = lra.lib().lra_top_svd(ctx._h, m, n, k, r, lra.F64, Cbig.data_ptr(), ldc, Wh.ctypes.data, Rbig.data_ptr(),
                               ldr, Sb.data_ptr(), lds, sg.ctypes.data, Tb.data_ptr(), ldt, pc.ctypes.data,
                               pr.ctypes.data)
    assert st == 0, st
    np.testing.assert_array_equal(sg, sg0)
    np.testing.assert_array_equal(pc, pc0)
    np.testing.assert_array_equal(pr, pr0)
    np.testing.assert_array_equal(Sb[:, :m].cpu().numpy(), S0.t().cpu().numpy())
    np.testing.assert_array_equal(Tb[:, :n].cpu().numpy(), T0.cpu().numpy())
    assert bool((Sb[:, m:] == 5.0).all()) and bool((Tb[:, n:] == 5.0).all())
    # leading dimensions below the row counts are rejected
    st = lra.lib().lra_top_svd(ctx._h, m, n, k, r, lra.F64, Cbig.data_ptr(), m - 1, Wh.ctypes.data, Rbig.data_ptr(),
                               ldr, Sb.data_ptr(), lds, sg.ctypes.data, Tb.data_ptr(), ldt, None, None)
    assert st == lra.EINVAL


def test_invalid_arguments(ctx):
    from paper_1611_01391_amd import lra
    _say("top svd invalid arguments")
    C, W, R = _factors(0, 100, 90, 8)
    Cd, Rd = _dev(C, R)
    for r in (0, 9):
        with pytest.raises(lra.LraError):
            ctx.top_svd(Cd, W, Rd, r)
    Wn = W.copy()
    Wn[2, 3] = np.nan
    with pytest.raises(lra.LraError) as e:
        ctx.top_svd(Cd, Wn, Rd, 4)
    assert e.value.args[0].endswith(f"({lra.ENONFINITE})")
    # a NaN in C or an Inf in R: reported, outputs untouched
    for bad in ("C", "R"):
        C2, R2 = C.copy(), R.copy()
        if bad == "C":
            C2[57, 3] = np.nan
        else:
            R2[5, 80] = np.inf
        Cb, Rb = _dev(C2, R2)
        S0 = torch.full((4 * 100,), 7.0, dtype=torch.float64, device="cuda")
        with pytest.raises(lra.LraError) as e:
            ctx.top_svd(Cb, W, Rb, 4, S_out=S0)
        assert e.value.args[0].endswith(f"({lra.ENONFINITE})")
        assert bool((S0 == 7.0).all())
