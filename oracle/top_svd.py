"""CPU oracle of the transition from an LRA to its top SVD (Appendix D,
Algorithm D.1), binary64, numpy.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use this module; the product library never
does, and this module never imports the product package.

Given the three factors of an LRA M ~ C W R (C m x k, W k x k, R k x n with
k much smaller than m and n) and a target rank r <= k, Algorithm D.1:

1. factors C and B = R by column-pivoted (rank-revealing) QR: C P = Q R_C
   and R^T P' = Q' R_R, keeping the first r columns of Q and Q'; then
   M ~ Q [R_C]_{r,:} P^T W P' [R_R]_{r,:}^T Q'^T with an r x r middle factor;
2. takes the SVD of that middle factor, U = S_bar Sigma T_bar^T;
3. returns S = Q[:, :r] S_bar, Sigma and T^T = T_bar^T Q'[:, :r]^T.

The pivoted QR is the textbook Householder QR with column pivoting
(Businger and Golub): at step j the remaining column of largest norm over
rows j.. is moved to position j (lowest index among equals), with the norms
recomputed from the current matrix at every step; the recorded margin of a
step is the relative gap between the largest and the second largest of those
norms.  The SVD of the small factor is LAPACK's (numpy.linalg.svd).  A
requested rank above the numerical rank of C or R (|R_C[j,j]| or |R_R[j,j]|
at most max(m, n) u |R[0,0]| for some j < r: the level of the rounding errors
of a Householder QR of the tall factor) is reported as rank loss, status -2.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

U64 = 2.0 ** -53


def householder_qrp(X: np.ndarray):
    """Householder QR with column pivoting of a tall m x k matrix (m >= k):
    X[:, piv] = Q R with Q m x k orthonormal, R k x k upper triangular.
    Returns (Q, R, piv, margins); margins[j] is (first - second) / first of
    the column norms compared at step j (inf with one column left)."""
    A = np.array(X, dtype=np.float64, copy=True)
    m, k = A.shape
    if m < k:
        raise ValueError("householder_qrp needs m >= k")
    piv = np.arange(k)
    margins = np.full(k, np.inf)
    vs, betas = [], []
    for j in range(k):
        norms = np.linalg.norm(A[j:, j:], axis=0)
        p = int(np.argmax(norms))  # first index among equal maxima
        if k - j > 1:
            rest = np.delete(norms, p)
            top = norms[p]
            margins[j] = (top - rest.max()) / top if top > 0 else 0.0
        if p:
            A[:, [j, j + p]] = A[:, [j + p, j]]
            piv[[j, j + p]] = piv[[j + p, j]]
        x = A[j:, j].copy()
        nx = np.linalg.norm(x)
        v = x
        if nx == 0.0:
            vs.append(None)
            betas.append(0.0)
            continue
        alpha = -nx if x[0] >= 0 else nx
        v[0] = x[0] - alpha
        beta = 2.0 / np.dot(v, v)
        A[j:, j:] -= beta * np.outer(v, v @ A[j:, j:])
        A[j, j] = alpha
        A[j + 1:, j] = 0.0
        vs.append(v)
        betas.append(beta)
    R = np.triu(A[:k, :])
    # Q = H_0 H_1 ... H_{k-1} applied to the first k columns of the identity
    Q = np.zeros((m, k))
    Q[:k, :k] = np.eye(k)
    for j in range(k - 1, -1, -1):
        if vs[j] is None:
            continue
        Q[j:, :] -= betas[j] * np.outer(vs[j], vs[j] @ Q[j:, :])
    return Q, R, piv, margins


@dataclass
class TopSVD:
    status: int
    S: np.ndarray           # m x r, orthonormal columns
    sigma: np.ndarray       # r, descending
    Tt: np.ndarray          # r x n, orthonormal rows
    piv_c: np.ndarray       # column pivots of C
    piv_r: np.ndarray       # column pivots of R^T (rows of R)
    margins_c: np.ndarray
    margins_r: np.ndarray
    rdiag_c: np.ndarray     # |R_C[j,j]|
    rdiag_r: np.ndarray

    def min_margin(self, r: int) -> float:
        """Smallest pivot margin among the first r steps of either factor:
        the decisions that fix the kept subspaces."""
        return float(min(self.margins_c[:r].min(), self.margins_r[:r].min()))


def top_svd(C: np.ndarray, W: np.ndarray, R: np.ndarray, r: int) -> TopSVD:
    """Algorithm D.1 on M ~ C W R, target rank r (1 <= r <= k)."""
    C = np.asarray(C, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    m, k = C.shape
    k2, n = R.shape
    if W.shape != (k, k2) or k2 != k or not (1 <= r <= k) or m < k or n < k:
        raise ValueError("need C m x k, W k x k, R k x n, k <= m, n and 1 <= r <= k")
    # step 1: rank-revealing QR of C and of R^T
    Qc, Rc, pc, mc = householder_qrp(C)
    Qr, Rr, pr, mr = householder_qrp(R.T)
    dc, dr = np.abs(np.diag(Rc)), np.abs(np.diag(Rr))
    lim = max(m, n) * U64
    bad = (dc[:r] <= lim * dc[0]).any() or (dr[:r] <= lim * dr[0]).any()
    if bad:
        z = np.zeros((0,))
        return TopSVD(-2, np.zeros((m, 0)), z, np.zeros((0, n)), pc, pr, mc, mr, dc, dr)
    # C = Qc Rc P^T and R = P' Rr^T Qr^T, so C W R = Qc (Rc P^T W P' Rr^T) Qr^T;
    # (P^T W P')[a, b] = W[pc[a], pr[b]]
    middle = Rc[:r, :] @ W[np.ix_(pc, pr)] @ Rr[:r, :].T
    # step 2: SVD of the r x r middle factor
    Sb, sigma, Tbt = np.linalg.svd(middle)
    # step 3: the orthonormal factors
    S = Qc[:, :r] @ Sb
    Tt = Tbt @ Qr[:, :r].T
    return TopSVD(0, S, sigma, Tt, pc, pr, mc, mr, dc, dr)
