"""GPU test of the allocation-free entry point lra_ca_cur_noalloc.

It runs the same kernels as lra_ca_cur on a fixed per-device scratch array,
so its results must be the same bits as lra_ca_cur's (which the parity
tests hold to the oracle).  Two calls in a row, the second with a smaller
input, check that nothing of the first call's contents in the shared array
leaks into the second; one larger call uses a global strip inside the array;
a problem whose workspace exceeds the array is rejected before any launch,
and the entry point still works afterwards.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _same(a, b, what):
    assert a.status == b.status, (what, a.status, b.status)
    assert a.k == b.k, (what, a.k, b.k)
    np.testing.assert_array_equal(a.I, b.I, err_msg=what)
    np.testing.assert_array_equal(a.J, b.J, err_msg=what)
    np.testing.assert_array_equal(a.G, b.G, err_msg=what)
    np.testing.assert_array_equal(a.U, b.U, err_msg=what)
    assert a.err_est_rel == b.err_est_rel and a.err_est_abs == b.err_est_abs, what
    assert (a.sweeps_done, a.swaps_total, a.entries_read) == (b.sweeps_done, b.swaps_total, b.entries_read), what


@pytest.fixture(scope="module")
def ctx():
    from paper_1611_01391_amd import lra
    c = lra.Context()
    yield c
    c.close()


def test_noalloc_matches_ca_cur_twice(ctx):
    from paper_1611_01391_amd import lra
    # first call: float32 4096 x 3000, k = 32, binary64 path
    A, d = synth.rect_factor_gaussian(3, 4096, 3000, 32, 1e-4, 32, dtype=np.float32)
    At = torch.from_numpy(A).cuda()
    kw = dict(init_cols=d.cand_cols, sample_rows=d.sample_rows, sample_cols=d.sample_cols)
    _say("noalloc: dense float32 4096x3000 k=32")
    ref = ctx.ca_cur(lra.dense(At), 32, 3, 0.0, **kw)
    got = ctx.ca_cur_noalloc(lra.dense(At), 32, 3, 0.0, **kw)
    _same(got, ref, "4096x3000")
    assert got.status == lra.OK
    # second call, smaller: binary64 512 x 512, k = 8
    B, e = synth.plain_fp64(1)
    Bt = torch.from_numpy(B).cuda()
    kw = dict(init_cols=e.cand_cols, sample_rows=e.sample_rows, sample_cols=e.sample_cols)
    _say("noalloc: dense binary64 512x512 k=8")
    got = ctx.ca_cur_noalloc(lra.dense(Bt), 8, 3, 0.0, **kw)
    ref = ctx.ca_cur(lra.dense(Bt), 8, 3, 0.0, **kw)
    _same(got, ref, "512x512")
    assert got.status == lra.OK


def test_noalloc_global_strip_and_adaptive(ctx):
    """A team of 4 workgroups on 20000 rows cannot keep its strip rows in LDS:
    the strip lives in the scratch array.  Adaptive rank 8 -> 24 on a Cauchy
    kernel, then a smaller fixed-rank call."""
    from paper_1611_01391_amd import lra
    s, t, d = synth.cauchy_points(5, m=20000, n=18000, k=8, k_max=24)
    t = t - 0.9  # t in [1.1, 2.1]: closer to s, so the rank grows past 8
    src = lra.cauchy(torch.from_numpy(s).cuda(), torch.from_numpy(t).cuda())
    kw = dict(init_cols=d.cand_cols, sample_rows=d.sample_rows, sample_cols=d.sample_cols, k_max=24,
              team_wgs=4, raise_on_error=False)
    _say("noalloc: Cauchy 20000x18000 adaptive 8..24, team 4 (global strip)")
    ref = ctx.ca_cur(src, 8, 4, 1e-12, **kw)
    got = ctx.ca_cur_noalloc(src, 8, 4, 1e-12, **kw)
    _same(got, ref, "cauchy adaptive")
    assert got.k > 8
    s2, t2, d2 = synth.cauchy_points(6, m=3000, n=2500, k=8, k_max=8)
    src2 = lra.cauchy(torch.from_numpy(s2).cuda(), torch.from_numpy(t2).cuda())
    kw2 = dict(init_cols=d2.cand_cols, sample_rows=d2.sample_rows, sample_cols=d2.sample_cols,
               raise_on_error=False)
    _say("noalloc: Cauchy 3000x2500 k=8")
    got = ctx.ca_cur_noalloc(src2, 8, 2, 0.0, **kw2)
    ref = ctx.ca_cur(src2, 8, 2, 0.0, **kw2)
    _same(got, ref, "cauchy small")


def test_noalloc_rejects_oversized_workspace(ctx):
    """2^20 rows at rank 64 on 256 workgroups need a 512 MiB global strip,
    beyond the fixed array: LRA_ESCRATCH before any launch; a later call
    still runs."""
    from paper_1611_01391_amd import lra
    m = 1 << 20
    x = torch.linspace(0.0, 1.0, m, dtype=torch.float64, device="cuda")
    y = torch.linspace(2.0, 3.0, m, dtype=torch.float64, device="cuda")
    _say("noalloc: oversized workspace is rejected")
    r = ctx.ca_cur_noalloc(lra.cauchy(x, y), 64, 1, 0.0, team_wgs=256, raise_on_error=False)
    assert r.status == lra.ESCRATCH
    B, e = synth.plain_fp64(2)
    Bt = torch.from_numpy(B).cuda()
    kw = dict(init_cols=e.cand_cols, sample_rows=e.sample_rows, sample_cols=e.sample_cols)
    _same(ctx.ca_cur_noalloc(lra.dense(Bt), 8, 3, 0.0, **kw), ctx.ca_cur(lra.dense(Bt), 8, 3, 0.0, **kw),
          "after rejection")
