"""Host-side logic that needs no GPU: the seeded workload generators (their
shapes, ranges and structural invariants) and the benchmark's refusal of
more than one GPU."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_plain_fp64_is_rank8_plus_noise():
    A, d = synth.plain_fp64(0)
    assert A.shape == (512, 512) and A.dtype == np.float64
    s = np.linalg.svd(A, compute_uv=False)
    assert s[7] > 1e3 * s[8]          # a clear rank-8 gap at noise 1e-8
    assert len(set(d.cand_cols.tolist())) == 8
    assert np.all(np.diff(d.sample_rows) > 0) and np.all(np.diff(d.sample_cols) > 0)
    assert len(d.sample_rows) == 64 and len(d.sample_cols) == 64


def test_seeded_inputs_are_reproducible():
    a1, d1 = synth.plain_fp64(3)
    a2, d2 = synth.plain_fp64(3)
    np.testing.assert_array_equal(a1, a2)
    np.testing.assert_array_equal(d1.cand_cols, d2.cand_cols)
    s1, t1, _ = synth.cauchy_points(5, m=1000)
    s2, t2, _ = synth.cauchy_points(5, m=1000)
    np.testing.assert_array_equal(s1, s2)
    np.testing.assert_array_equal(t1, t2)


def test_dense_scaled_recipe():
    A, d = synth.dense_scaled(0, n=512, r=8, k=8, rel_noise=1e-4, chunk=100)
    assert A.dtype == np.float32 and A.shape == (512, 512)
    s = np.linalg.svd(A.astype(np.float64), compute_uv=False)
    # noise at 1e-4 of the rank-8 part's Frobenius norm
    assert np.sqrt((s[8:] ** 2).sum()) / np.sqrt((s[:8] ** 2).sum()) == pytest.approx(1e-4, rel=0.2)


def test_cauchy_points_ranges():
    s, t, d = synth.cauchy_points(1, m=5000, n=4000, k=8, k_max=40)
    assert s.min() >= 0 and s.max() <= 1 and t.min() >= 2 and t.max() <= 3
    assert len(d.cand_cols) == 80 and len(set(d.cand_cols.tolist())) == 80
    assert d.cand_cols.max() < 4000


def test_far_field_blocks_are_admissible_and_disjoint():
    x, blocks, dense = synth.multipole(0, 1 << 14, 256, 96)
    assert np.all(np.diff(x) >= 0) and x.min() >= 0 and x.max() <= 1
    root = synth.build_tree(x, 256)
    # boxes: leaves hold at most 256 points (or are depth-limited)
    def leaves(b):
        return [b] if not b.children else leaves(b.children[0]) + leaves(b.children[1])
    lv = leaves(root)
    assert sum(b.count for b in lv) == len(x)
    assert all(b.count <= 256 or b.width < 1e-15 for b in lv)
    seen = set()
    for (a0, a1, b0, b1) in blocks:
        assert a1 - a0 >= 96 and b1 - b0 >= 96
        assert a1 <= b0 or b1 <= a0                  # disjoint point ranges
        assert (a0, a1, b0, b1) not in seen and (b0, b1, a0, a1) not in seen
        seen.add((a0, a1, b0, b1))
    for (a0, a1, b0, b1) in dense:
        assert min(a1 - a0, b1 - b0) < 96
    assert len(blocks) > 50


def test_far_field_pairs_cover_every_far_interaction_once():
    """Brute force on a small tree: no pair of points is covered twice, and
    every pair of points in well-separated leaves is covered by exactly one
    admissible pair (blocks or dense), in one orientation."""
    x = synth.mixture_points(2, 3000)
    root = synth.build_tree(x, 64)
    blocks, dense = synth.far_field_blocks(root, 0)
    cover = np.zeros((len(x), len(x)), dtype=np.int32)
    for (a0, a1, b0, b1) in blocks + dense:
        cover[a0:a1, b0:b1] += 1
    sym = cover + cover.T
    assert sym.max() == 1

    def leaves(b):
        return [b] if not b.children else leaves(b.children[0]) + leaves(b.children[1])
    lv = [b for b in leaves(root) if b.count]
    for A in lv:
        for B in lv:
            if A is B:
                continue
            d = max(0.0, B.lo - A.hi, A.lo - B.hi)
            if d >= max(A.width, B.width):
                assert np.all(sym[A.start:A.end, B.start:B.end] == 1)


def test_request_stream_recipe():
    specs = synth.request_stream(0, 400, rate=100.0, lo=1024, hi=65536)
    ks = {s.k for s in specs}
    assert ks <= {8, 16, 32, 64}
    assert all(1024 <= s.m <= 65536 and 1024 <= s.n <= 65536 for s in specs)
    assert all(1e-10 <= s.tol <= 1e-4 for s in specs)
    arr = np.array([s.arrival for s in specs])
    assert np.all(np.diff(arr) >= 0)
    # Poisson at rate 100/s: mean gap 10 ms
    assert np.mean(np.diff(arr)) == pytest.approx(0.01, rel=0.2)
    kinds = [s.kind for s in specs]
    assert 0.35 < kinds.count("dense") / len(kinds) < 0.65
    # the request mix does not depend on the arrival rate
    same = synth.request_stream(0, 400, rate=0.0, lo=1024, hi=65536)
    assert [(s.kind, s.m, s.n, s.k, s.tol, s.dtype) for s in same] == \
        [(s.kind, s.m, s.n, s.k, s.tol, s.dtype) for s in specs]


def test_dense_pool_matrix_rank():
    A = synth.dense_pool_matrix(1, 300, 200, 5, 1e-6)
    s = np.linalg.svd(A, compute_uv=False)
    assert s[4] > 1e4 * s[5]


def test_bench_refuses_more_than_one_gpu():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    msg = json.loads(out.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]
