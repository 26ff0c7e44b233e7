"""Seeded synthetic inputs for the C-A / CUR workloads.

Shared by the tests, the smoke check and the benchmark.  This module holds no
arithmetic of the method itself: it only draws matrices, point sets, index
sets and request streams with numpy's PCG64 ``default_rng(seed)``, in a fixed
draw order, so that the CPU oracle and the GPU library see identical bits.

Workload recipes (the paper's own benchmark matrices -- the San Jose State
singular-matrix collection, the Toeplitz-derived Cauchy-like matrices of its
HSS tests, the finite-difference operator -- are not available, so these
seeded inputs stand in for them):

* ``plain_fp64`` -- W = G1 G2 + eps G3 with Gaussian factors, the perturbed
  factor-Gaussian family of Section 12.3 (the paper uses eps = 1e-10; the
  512 x 512, rank-8 workload here uses eps = 1e-8).
* ``dense_scaled`` -- A = G1 G2 D + noise, D log-uniform column scales in
  [0.1, 10], noise N(0,1) scaled to 1e-4 of ||G1 G2 D||_F, stored float32.
* ``cauchy_points`` -- s ~ U[0,1], t ~ U[2,3]: a_ij = 1/(s_i - t_j), the
  Cauchy-like kernel of the HSS experiments (Section 12.8).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Draws:
    """Index sets that the method consumes as random input."""
    cand_cols: np.ndarray   # J0 = cand_cols[:k]; rank growth takes the rest in order
    sample_rows: np.ndarray  # residual sample Q (sorted, distinct)
    sample_cols: np.ndarray  # residual sample S (sorted, distinct)


def residual_sample(m: int, n: int, seed: int, q: int = 64, s: int = 64):
    """Q, S for the a posteriori estimate: a fresh default_rng(seed + 1)."""
    rng = np.random.default_rng(seed + 1)
    q = min(q, m)
    s = min(s, n)
    Q = np.sort(rng.choice(m, q, replace=False)).astype(np.int64)
    S = np.sort(rng.choice(n, s, replace=False)).astype(np.int64)
    return Q, S


def plain_fp64(seed: int = 0, n: int = 512, r: int = 8, eps: float = 1e-8, k: int | None = None):
    """Perturbed factor-Gaussian W = G1 G2 + eps E (float64, row-major).

    Draw order: G1 (n x r), G2 (r x n), E (n x n), then J0 = choice(n, k)."""
    k = r if k is None else k
    rng = np.random.default_rng(seed)
    G1 = rng.standard_normal((n, r))
    G2 = rng.standard_normal((r, n))
    E = rng.standard_normal((n, n))
    A = G1 @ G2 + eps * E
    J0 = rng.choice(n, k, replace=False).astype(np.int64)
    Q, S = residual_sample(n, n, seed)
    return A, Draws(J0, Q, S)


def rect_factor_gaussian(seed: int, m: int, n: int, r: int, eps: float, k: int,
                         dtype=np.float64, n_cand: int | None = None):
    """Rectangular perturbed factor-Gaussian matrix, for parity sweeps."""
    rng = np.random.default_rng(seed)
    G1 = rng.standard_normal((m, r))
    G2 = rng.standard_normal((r, n))
    E = rng.standard_normal((m, n))
    A = (G1 @ G2 + eps * E).astype(dtype)
    cand = rng.choice(n, n_cand or k, replace=False).astype(np.int64)
    Q, S = residual_sample(m, n, seed)
    return A, Draws(cand, Q, S)


def spectrum_dense(seed: int, m: int, n: int, decay: float = 8.0, r: int = 160, n_cand: int = 80):
    """A = U diag(sigma) V^T with orthonormal U (m x r), V (n x r) from the QR
    factors of Gaussian matrices and sigma_j = 10^(-j / decay): a numerically
    low-rank matrix whose error at rank k falls by a factor 10^(8 / decay) per
    8 more columns, so that a tolerance between those levels makes the rank
    grow by whole steps.  Draw order: the m x r Gaussian, the n x r Gaussian,
    then the candidate columns choice(n, n_cand)."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n, r)))
    sig = 10.0 ** (-np.arange(r) / decay)
    A = (U * sig[None, :]) @ V.T
    cand = rng.choice(n, n_cand, replace=False).astype(np.int64)
    Q, S = residual_sample(m, n, seed)
    return np.ascontiguousarray(A), Draws(cand, Q, S)


def dense_scaled(seed: int = 0, n: int = 16384, r: int = 32, k: int = 32, rel_noise: float = 1e-4,
                 chunk: int = 2048):
    """A = G1 G2 D + rel_noise (||G1 G2 D||_F / ||E||_F) E, cast to float32.

    Draw order: G1 (n x r), G2 (r x n), the log-uniform column scales d
    (U[ln 0.1, ln 10], exponentiated), E (n x n, row-major), J0 = choice(n, k).
    Row chunks of E are drawn in sequence, which reproduces one n x n draw."""
    rng = np.random.default_rng(seed)
    G1 = rng.standard_normal((n, r))
    G2 = rng.standard_normal((r, n))
    d = np.exp(rng.uniform(np.log(0.1), np.log(10.0), n))
    G2d = G2 * d[None, :]
    # ||G1 G2 D||_F^2 = sum_j (G2d[:, j]^T (G1^T G1) G2d[:, j])
    M = G1.T @ G1
    norm_l = float(np.sqrt(np.einsum("ij,ik,kj->", G2d, M, G2d)))
    E = np.empty((n, n), dtype=np.float64)
    for r0 in range(0, n, chunk):
        E[r0:r0 + chunk] = rng.standard_normal((min(chunk, n - r0), n))
    norm_e = float(np.sqrt(np.einsum("ij,ij->", E, E)))
    c = rel_noise * norm_l / norm_e
    A = np.empty((n, n), dtype=np.float32)
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        A[r0:r1] = (G1[r0:r1] @ G2d + c * E[r0:r1]).astype(np.float32)
    del E
    J0 = rng.choice(n, k, replace=False).astype(np.int64)
    Q, S = residual_sample(n, n, seed)
    return A, Draws(J0, Q, S)


def cauchy_points(seed: int = 0, m: int = 1 << 20, n: int | None = None, k: int = 8,
                  k_max: int = 40, dtype=np.float64):
    """s ~ U[0,1]^m, t ~ U[2,3]^n (drawn in that order), then the candidate
    column list choice(n, min(n, 2 k_max)) whose first k entries are J0."""
    n = m if n is None else n
    rng = np.random.default_rng(seed)
    s = rng.uniform(0.0, 1.0, m)
    t = rng.uniform(2.0, 3.0, n)
    cand = rng.choice(n, min(n, 2 * max(k, k_max)), replace=False).astype(np.int64)
    Q, S = residual_sample(m, n, seed)
    return s.astype(dtype), t.astype(dtype), Draws(cand, Q, S)


# ---------------------------------------------------------------------------
# multipole-style workload: 1D points, adaptive binary tree, far-field blocks
# (the neutered-block-column generators of the multipole application)
# ---------------------------------------------------------------------------

MIX_MEANS = (0.2, 0.5, 0.8)
MIX_SDS = (0.01, 0.05, 0.1)


def mixture_points(seed: int = 0, N: int = 1 << 20) -> np.ndarray:
    """N points from the 3-component Gaussian mixture (equal weights, means
    0.2/0.5/0.8, sds 0.01/0.05/0.1), clipped to [0, 1], sorted (float64).
    Draw order: component labels, then the standard normals."""
    rng = np.random.default_rng(seed)
    comp = rng.integers(0, 3, N)
    z = rng.standard_normal(N)
    x = np.asarray(MIX_MEANS)[comp] + np.asarray(MIX_SDS)[comp] * z
    return np.sort(np.clip(x, 0.0, 1.0))


@dataclass
class Box:
    lo: float
    hi: float
    start: int
    end: int
    children: tuple = ()

    @property
    def count(self) -> int:
        return self.end - self.start

    @property
    def width(self) -> float:
        return self.hi - self.lo


def build_tree(x: np.ndarray, leaf_max: int = 4096, lo: float = 0.0, hi: float = 1.0) -> Box:
    """Adaptive binary tree on sorted points: a box [lo, hi) is split at its
    midpoint while it holds more than leaf_max points."""
    def make(lo, hi, start, end, depth):
        b = Box(lo, hi, start, end)
        if end - start > leaf_max and depth < 60:
            mid = 0.5 * (lo + hi)
            cut = start + int(np.searchsorted(x[start:end], mid, side="left"))
            b.children = (make(lo, mid, start, cut, depth + 1), make(mid, hi, cut, end, depth + 1))
        return b
    return make(lo, hi, 0, len(x), 0)


def far_field_blocks(root: Box, min_size: int = 96):
    """Admissible pairs by dual-tree traversal: boxes X, Y with
    dist(X, Y) >= max(width X, width Y).  Each unordered pair is listed once
    (X left of Y); pairs with fewer than min_size points on a side are
    returned separately as dense blocks.  Returns (blocks, dense) lists of
    (x_start, x_end, y_start, y_end)."""
    blocks, dense = [], []

    def dist(a, b):
        return max(0.0, b.lo - a.hi, a.lo - b.hi)

    def visit(a, b):
        if a.count == 0 or b.count == 0:
            return
        if a is b:
            if not a.children:
                return  # diagonal leaf: near field
            c = a.children
            visit(c[0], c[0])
            visit(c[1], c[1])
            visit(c[0], c[1])
            return
        if dist(a, b) >= max(a.width, b.width):
            rec = (a.start, a.end, b.start, b.end)
            if min(a.count, b.count) < min_size:
                dense.append(rec)
            else:
                blocks.append(rec)
            return
        if not a.children and not b.children:
            return  # near field
        if a.children and (not b.children or a.width >= b.width):
            for c in a.children:
                visit(c, b)
        else:
            for c in b.children:
                visit(a, c)

    visit(root, root)
    return blocks, dense


def multipole(seed: int = 0, N: int = 1 << 20, leaf_max: int = 4096, min_size: int = 96):
    """The batched far-field workload: sorted mixture points, the adaptive
    tree, and its admissible blocks (x_start, x_end, y_start, y_end) with
    min(|X|, |Y|) >= min_size; the smaller pairs stay dense."""
    x = mixture_points(seed, N)
    root = build_tree(x, leaf_max)
    blocks, dense = far_field_blocks(root, min_size)
    return x, blocks, dense


def block_draws(seed: int, index: int):
    """Stream seed of block `index` in a batched call (the library's default
    draws use SplitMix64 stream seed + index * 0x1000003)."""
    return (seed + index * 0x1000003) & 0xFFFFFFFFFFFFFFFF


# ---------------------------------------------------------------------------
# served stream: request specifications
# ---------------------------------------------------------------------------

@dataclass
class RequestSpec:
    kind: str          # "dense" or "cauchy"
    m: int
    n: int
    k: int
    tol: float
    dtype: str         # "f32" or "f64"
    arrival: float     # seconds after the stream starts
    pool: int          # dense: index of the pool matrix (rank k, dtype); cauchy: point-set seed


def request_stream(seed: int = 0, count: int = 2000, rate: float = 0.0, lo: int = 1024, hi: int = 65536,
                   ks=(8, 16, 32, 64), tol_lo: float = 1e-10, tol_hi: float = 1e-4):
    """Poisson arrivals at `rate` requests/s (rate 0: all arrive at t = 0).
    Draw order per request: kind (p = 1/2), m, n (log-uniform [lo, hi]), k
    (uniform over ks, capped at min(m, n)), tol (log-uniform), dtype (p = 1/2);
    the exponential inter-arrival gaps are drawn afterwards."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        kind = "dense" if rng.random() < 0.5 else "cauchy"
        m = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        n = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        k = int(min(ks[int(rng.integers(0, len(ks)))], m, n))
        tol = float(np.exp(rng.uniform(np.log(tol_lo), np.log(tol_hi))))
        dtype = "f32" if rng.random() < 0.5 else "f64"
        specs.append(RequestSpec(kind, m, n, k, tol, dtype, 0.0, 0))
    gaps = rng.exponential(1.0 / rate, count) if rate > 0 else np.zeros(count)
    t = np.cumsum(gaps)
    for i, s in enumerate(specs):
        s.arrival = float(t[i]) if rate > 0 else 0.0
        s.pool = ks.index(s.k) if s.k in ks else 0
        if s.kind == "cauchy":
            s.pool = i
    return specs


def dense_pool_matrix(seed: int, m: int, n: int, r: int, rel_noise: float, dtype=np.float64):
    """Gaussian rank-r product plus Gaussian noise scaled to rel_noise of its
    Frobenius norm (host, for test-sized pools).  Draw order: G1, G2, E."""
    rng = np.random.default_rng(seed)
    G1 = rng.standard_normal((m, r))
    G2 = rng.standard_normal((r, n))
    E = rng.standard_normal((m, n))
    L = G1 @ G2
    A = L + rel_noise * (np.linalg.norm(L) / np.linalg.norm(E)) * E
    return A.astype(dtype)
