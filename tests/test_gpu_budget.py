"""Device memory of a context: the workspace of the blocking calls, the
serving arena and its control images all count against hbm_budget_bytes,
the context never holds more than the budget, a problem that needs more is
refused with LRA_EBUDGET (and the context keeps working), and calls no
larger than an earlier one allocate nothing (steady state)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BUDGET = 96 << 20


def _say(msg):
    print(msg, flush=True)


def test_budget_and_steady_state():
    from paper_1611_01391_amd import lra
    _say("budget: blocking calls")
    ctx = lra.Context(hbm_budget_bytes=BUDGET)
    A, d = synth.rect_factor_gaussian(2, 6000, 5000, 16, 1e-6, 16)
    At = torch.from_numpy(A).cuda()
    kw = dict(init_cols=d.cand_cols, sample_rows=d.sample_rows, sample_cols=d.sample_cols)
    first = ctx.ca_cur(lra.dense(At), 16, 2, 0.0, **kw)
    s1 = ctx.stats()
    assert 0 < s1["device_bytes"] <= BUDGET and s1["device_allocs"] >= 1
    for _ in range(3):
        again = ctx.ca_cur(lra.dense(At), 16, 2, 0.0, **kw)
        np.testing.assert_array_equal(again.I, first.I)
    s2 = ctx.stats()
    assert s2["device_allocs"] == s1["device_allocs"], "steady-state calls must not allocate"
    # smaller problems reuse the workspace too
    ctx.ca_cur(lra.dense(At[:1000, :900]), 8, 2, 0.0)
    assert ctx.stats()["device_allocs"] == s1["device_allocs"]
    # 2^20 rows at rank 64 on 256 workgroups need a 512 MiB global strip: refused
    m = 1 << 20
    x = torch.linspace(0.0, 1.0, m, dtype=torch.float64, device="cuda")
    y = torch.linspace(2.0, 3.0, m, dtype=torch.float64, device="cuda")
    r = ctx.ca_cur(lra.cauchy(x, y), 64, 1, 0.0, team_wgs=256, raise_on_error=False)
    assert r.status == lra.EBUDGET
    assert ctx.stats()["device_bytes"] <= BUDGET
    # and the context still works
    again = ctx.ca_cur(lra.dense(At), 16, 2, 0.0, **kw)
    np.testing.assert_array_equal(again.I, first.I)
    assert ctx.stats()["device_bytes"] <= BUDGET

    _say("budget: serving arena inside the same budget")
    ctx.serve_config(arena_bytes=48 << 20)
    tickets = [ctx.submit(lra.dense(At), 16, 2, 0.0, seed=i) for i in range(12)]
    res = [ctx.wait(t) for t in tickets]
    assert all(r.status >= 0 for r in res)
    st = ctx.stats()
    assert st["device_bytes"] <= BUDGET, st
    ctx.close()


def test_serving_arena_over_budget_is_refused():
    from paper_1611_01391_amd import lra
    ctx = lra.Context(hbm_budget_bytes=BUDGET)
    ctx.serve_config(arena_bytes=BUDGET + (16 << 20))
    A, d = synth.rect_factor_gaussian(3, 800, 700, 8, 1e-6, 8)
    At = torch.from_numpy(A).cuda()
    with pytest.raises(lra.LraError) as e:
        ctx.submit(lra.dense(At), 8, 2, 0.0)
    assert e.value.status == lra.EBUDGET
    assert ctx.stats()["device_bytes"] <= BUDGET
    ctx.close()
