"""Python view of the CPU oracle (plain C, binary64) for C-A / CUR.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark import this module; the product library never
does, and this module never imports the product package.

Every function marshals numpy arrays into the C library built from
``oracle.c`` / ``oracle_core.inc`` and returns numpy arrays.  Paper passages
are cited in those C sources.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["oracle.c", "oracle_core.inc", "oracle.h"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (no fast-math, no BLAS)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-o", tmp,
                    os.path.join(_HERE, "oracle.c"), "-lm"], check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dtype", C.c_int32), ("a", C.c_void_p),
                ("lda", C.c_int64), ("col_major", C.c_int32), ("pad_", C.c_int32),
                ("x", C.c_void_p), ("y", C.c_void_p), ("depth", C.c_int32), ("pad2_", C.c_int32),
                ("seed", C.c_uint64), ("pm", C.c_int64), ("pn", C.c_int64)]


class Trace(C.Structure):
    _fields_ = [("min_pivot_gap", C.c_double), ("min_swap_gap", C.c_double),
                ("min_stop_margin", C.c_double), ("min_rank_margin", C.c_double),
                ("min_tol_margin", C.c_double)]


class Options(C.Structure):
    _fields_ = [("tau", C.c_double), ("k_max", C.c_int32), ("k_step", C.c_int32),
                ("max_swaps", C.c_int32), ("warm_start", C.c_int32),
                ("cand_cols", C.c_void_p), ("n_cand", C.c_int64),
                ("sample_rows", C.c_void_p), ("q", C.c_int32),
                ("sample_cols", C.c_void_p), ("s", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("k", C.c_int32), ("status", C.c_int32), ("sweeps_done", C.c_int32),
                ("swaps_total", C.c_int32), ("entries_read", C.c_int64),
                ("err_est_rel", C.c_double), ("err_est_abs", C.c_double),
                ("err_mean", C.c_double), ("err_var", C.c_double),
                ("nucleus_cond1", C.c_double), ("trace", Trace)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        L.oracle_entry_f64.restype = C.c_double
        L.oracle_entry_f64.argtypes = [C.POINTER(Source), C.c_int64, C.c_int64]
        L.oracle_entry_f32.restype = C.c_float
        L.oracle_entry_f32.argtypes = [C.POINTER(Source), C.c_int64, C.c_int64]
        for sfx in ("f64", "f32"):
            f = getattr(L, "oracle_gepp_basis_" + sfx)
            f.restype = C.c_int
            f.argtypes = [P, C.c_int64, C.c_int, P, C.POINTER(Trace)]
            f = getattr(L, "oracle_maxvol_" + sfx)
            f.restype = C.c_int
            f.argtypes = [P, C.c_int64, C.c_int, P, C.c_int, C.c_double, C.c_int,
                          C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(Trace)]
        L.oracle_nucleus.restype = C.c_int
        L.oracle_nucleus.argtypes = [C.POINTER(Source), P, P, C.c_int, P, P, C.POINTER(C.c_double)]
        L.oracle_residual.restype = None
        L.oracle_residual.argtypes = [C.POINTER(Source), C.c_int64, C.c_int64, C.c_int, P, P,
                                      P, C.c_int, P, C.c_int, P]
        L.oracle_ca_cur.restype = C.c_int
        L.oracle_ca_cur.argtypes = [C.POINTER(Source), C.c_int64, C.c_int64, C.c_int, C.c_int,
                                    C.c_double, C.c_int, C.POINTER(Options), P, P, P, P,
                                    C.POINTER(Result)]
        L.oracle_cur_variant.restype = C.c_int
        L.oracle_cur_variant.argtypes = [C.POINTER(Source), C.c_int64, C.c_int64, C.c_int, C.c_int, C.c_int,
                                         C.c_int, C.c_int, C.c_int, C.POINTER(Options), P, P, P, P, P,
                                         C.POINTER(Result)]
        L.oracle_svd_jacobi.restype = C.c_int
        L.oracle_svd_jacobi.argtypes = [P, C.c_int, P, P, P]
        L.oracle_nucleus_trunc.restype = C.c_int
        L.oracle_nucleus_trunc.argtypes = [C.POINTER(Source), P, P, C.c_int, C.c_int, P, P,
                                           C.POINTER(C.c_double)]
        L.oracle_residual_explicit.restype = None
        L.oracle_residual_explicit.argtypes = [C.POINTER(Source), C.c_int64, C.c_int64, C.c_int, P, P, P,
                                               P, C.c_int, P, C.c_int, P]
        L.oracle_splitmix64.restype = C.c_uint64
        L.oracle_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.oracle_draw_distinct.restype = None
        L.oracle_draw_distinct.argtypes = [C.c_uint64, C.c_int64, C.c_int64, P]
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _new_trace() -> Trace:
    inf = float("inf")
    return Trace(inf, inf, inf, inf, inf)


# ---------------------------------------------------------------------------
# sources: keep the arrays alive alongside the C struct
# ---------------------------------------------------------------------------

@dataclass
class HostSource:
    kind: int
    dtype: int
    arrays: tuple
    struct: Source
    m: int
    n: int


def dense(a: np.ndarray, col_major: bool = False) -> HostSource:
    """Dense m x n matrix held in host memory (float32 or float64)."""
    if a.dtype not in (np.float32, np.float64):
        raise TypeError("dense source must be float32 or float64")
    dt = 0 if a.dtype == np.float32 else 1
    if col_major:
        arr = np.asfortranarray(a)
        lda = a.shape[0]
    else:
        arr = np.ascontiguousarray(a)
        lda = a.shape[1]
    s = Source(0, dt, _ptr(arr), lda, 1 if col_major else 0, 0, None, None)
    return HostSource(0, dt, (arr,), s, a.shape[0], a.shape[1])


def abridged(a: np.ndarray, depth: int, seed: int, col_major: bool = False) -> HostSource:
    """F A H: the dense matrix pre-processed by d-abridged Hadamard multipliers
    with random sign scaling on both sides (orthogonal F and H)."""
    src = dense(a, col_major)
    m, n = a.shape
    if depth < 1 or m % (1 << depth) or n % (1 << depth):
        raise ValueError("2^depth must divide both dimensions")
    src.struct.kind = 3
    src.struct.depth = depth
    src.struct.seed = seed & 0xFFFFFFFFFFFFFFFF
    src.struct.pm = m
    src.struct.pn = n
    src.kind = 3
    return src


def cauchy(x: np.ndarray, y: np.ndarray) -> HostSource:
    """a_ij = 1 / (x_i - y_j)."""
    x = np.ascontiguousarray(x)
    y = np.ascontiguousarray(y.astype(x.dtype))
    dt = 0 if x.dtype == np.float32 else 1
    s = Source(1, dt, None, 0, 0, 0, _ptr(x), _ptr(y))
    return HostSource(1, dt, (x, y), s, x.shape[0], y.shape[0])


def invdist(x: np.ndarray, y: np.ndarray) -> HostSource:
    """a_ij = 1 / |x_i - y_j| (0 where the points coincide)."""
    x = np.ascontiguousarray(x)
    y = np.ascontiguousarray(y.astype(x.dtype))
    dt = 0 if x.dtype == np.float32 else 1
    s = Source(2, dt, None, 0, 0, 0, _ptr(x), _ptr(y))
    return HostSource(2, dt, (x, y), s, x.shape[0], y.shape[0])


# ---------------------------------------------------------------------------
# individual steps
# ---------------------------------------------------------------------------

def entry(src: HostSource, i: int, j: int, precision: str = "f64") -> float:
    f = lib().oracle_entry_f64 if precision == "f64" else lib().oracle_entry_f32
    return float(f(C.byref(src.struct), int(i), int(j)))


def gepp_basis(strip: np.ndarray, precision: str = "f64"):
    """Partial-pivot LU start of maxvol on an m x k strip.

    Returns (k_eff, I, B, trace) with B = strip[:, :k_eff] strip[I, :k_eff]^{-1}."""
    dt = np.float64 if precision == "f64" else np.float32
    m, k = strip.shape
    B = np.asfortranarray(strip.astype(dt))
    I = np.zeros(k, dtype=np.int64)
    tr = _new_trace()
    f = lib().oracle_gepp_basis_f64 if precision == "f64" else lib().oracle_gepp_basis_f32
    keff = f(_ptr(B), m, k, _ptr(I), C.byref(tr))
    return keff, I[:max(keff, 0)].copy(), B[:, :max(keff, 0)].copy(), tr


def maxvol(strip: np.ndarray, tau: float = 0.01, init=None, max_swaps: int = 0,
           precision: str = "f64"):
    """maxvol on an m x k strip.  Returns dict(I, B, swaps, k_eff, capped, trace)."""
    dt = np.float64 if precision == "f64" else np.float32
    m, k = strip.shape
    B = np.asfortranarray(strip.astype(dt))
    I = np.zeros(k, dtype=np.int64)
    if init is not None:
        I[:] = np.asarray(init, dtype=np.int64)
    keff = C.c_int(0)
    capped = C.c_int(0)
    tr = _new_trace()
    f = lib().oracle_maxvol_f64 if precision == "f64" else lib().oracle_maxvol_f32
    sw = f(_ptr(B), m, k, _ptr(I), 1 if init is not None else 0, float(tau), int(max_swaps),
           C.byref(keff), C.byref(capped), C.byref(tr))
    ke = keff.value
    return dict(I=I[:ke].copy(), B=B[:, :ke].copy(), swaps=sw, k_eff=ke,
                capped=bool(capped.value), trace=tr)


def nucleus(src: HostSource, I, J):
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    k = len(I)
    G = np.zeros((k, k))
    U = np.zeros((k, k))
    cond = C.c_double(0.0)
    rc = lib().oracle_nucleus(C.byref(src.struct), _ptr(I), _ptr(J), k, _ptr(G), _ptr(U),
                              C.byref(cond))
    return rc, G, U, cond.value


def residual(src: HostSource, I, J, Q, S):
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    Q = np.ascontiguousarray(Q, dtype=np.int64)
    S = np.ascontiguousarray(S, dtype=np.int64)
    out = np.zeros(6)
    lib().oracle_residual(C.byref(src.struct), src.m, src.n, len(I), _ptr(I), _ptr(J),
                          _ptr(Q), len(Q), _ptr(S), len(S), _ptr(out))
    return dict(norm_e=out[0], norm_a=out[1], mean=out[2], var=out[3],
                est_abs=out[4], est_rel=out[5])


@dataclass
class OracleResult:
    status: int
    k: int
    I: np.ndarray
    J: np.ndarray
    G: np.ndarray
    U: np.ndarray
    sweeps_done: int
    swaps_total: int
    entries_read: int
    err_est_rel: float
    err_est_abs: float
    err_mean: float
    err_var: float
    nucleus_cond1: float
    trace: dict = field(default_factory=dict)

    def min_gap(self) -> float:
        t = self.trace
        return min(t["min_pivot_gap"], t["min_swap_gap"], t["min_stop_margin"],
                   t["min_rank_margin"], t["min_tol_margin"])


def ca_cur(src: HostSource, k: int, sweeps: int, tol: float, cand_cols, sample_rows,
           sample_cols, tau: float = 0.01, k_max: int = 0, k_step: int = 8,
           max_swaps: int = 0, warm_start: bool = True, precision: str = "f64") -> OracleResult:
    """Run the whole C-A / CUR on the host."""
    cand = np.ascontiguousarray(cand_cols, dtype=np.int64)
    Q = np.ascontiguousarray(sample_rows, dtype=np.int64)
    S = np.ascontiguousarray(sample_cols, dtype=np.int64)
    kcap = max(k, k_max)
    opt = Options(float(tau), int(k_max), int(k_step), int(max_swaps), 1 if warm_start else 0,
                  _ptr(cand), len(cand), _ptr(Q), len(Q), _ptr(S), len(S))
    I = np.zeros(kcap, dtype=np.int64)
    J = np.zeros(kcap, dtype=np.int64)
    G = np.zeros(kcap * kcap)
    U = np.zeros(kcap * kcap)
    res = Result()
    lib().oracle_ca_cur(C.byref(src.struct), src.m, src.n, int(k), int(sweeps), float(tol),
                        0 if precision == "f64" else 1, C.byref(opt), _ptr(I), _ptr(J),
                        _ptr(G), _ptr(U), C.byref(res))
    kk = res.k
    tr = {f: getattr(res.trace, f) for f, _ in Trace._fields_}
    return OracleResult(res.status, kk, I[:kk].copy(), J[:kk].copy(),
                        G[:kk * kk].reshape(kk, kk).copy(), U[:kk * kk].reshape(kk, kk).copy(),
                        res.sweeps_done, res.swaps_total, res.entries_read, res.err_est_rel,
                        res.err_est_abs, res.err_mean, res.err_var, res.nucleus_cond1, tr)


def cur_variant(src: HostSource, k: int, sweeps: int, cand_cols, sample_rows, sample_cols, init_rows=None,
                cur_rank: int = 0, inner_sweeps: int = 4, nucleus_rank: int = 0, tau: float = 0.01,
                max_swaps: int = 0, warm_start: bool = True, precision: str = "f64") -> OracleResult:
    """The fixed-rank CUR algorithms of the C-A tests (see oracle.h):
    sweeps = 0 takes I = init_rows, J = cand_cols[:k] at random; cur_rank
    reduces the k x k generator to an r x r one of locally maximal volume
    (Cynical); nucleus_rank truncates the nucleus (Primitive)."""
    cand = np.ascontiguousarray(cand_cols, dtype=np.int64)
    Q = np.ascontiguousarray(sample_rows, dtype=np.int64)
    S = np.ascontiguousarray(sample_cols, dtype=np.int64)
    rows = None if init_rows is None else np.ascontiguousarray(init_rows, dtype=np.int64)
    opt = Options(float(tau), 0, 8, int(max_swaps), 1 if warm_start else 0,
                  _ptr(cand), len(cand), _ptr(Q), len(Q), _ptr(S), len(S))
    I = np.zeros(k, dtype=np.int64)
    J = np.zeros(k, dtype=np.int64)
    G = np.zeros(k * k)
    U = np.zeros(k * k)
    res = Result()
    lib().oracle_cur_variant(C.byref(src.struct), src.m, src.n, int(k), int(sweeps), int(cur_rank),
                             int(inner_sweeps), int(nucleus_rank), 0 if precision == "f64" else 1, C.byref(opt),
                             None if rows is None else _ptr(rows), _ptr(I), _ptr(J), _ptr(G), _ptr(U),
                             C.byref(res))
    kk = max(res.k, 0)
    tr = {f: getattr(res.trace, f) for f, _ in Trace._fields_}
    return OracleResult(res.status, kk, I[:kk].copy(), J[:kk].copy(),
                        G[:kk * kk].reshape(kk, kk).copy(), U[:kk * kk].reshape(kk, kk).copy(),
                        res.sweeps_done, res.swaps_total, res.entries_read, res.err_est_rel,
                        res.err_est_abs, res.err_mean, res.err_var, res.nucleus_cond1, tr)


def svd_jacobi(G: np.ndarray):
    """One-sided Jacobi SVD of a square matrix: (W, V, sv, sweeps) with
    W = G V having orthogonal columns and sv their norms."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    k = G.shape[0]
    W = np.zeros((k, k))
    V = np.zeros((k, k))
    sv = np.zeros(k)
    sw = lib().oracle_svd_jacobi(_ptr(G), k, _ptr(W), _ptr(V), _ptr(sv))
    return W, V, sv, sw


def nucleus_trunc(src: HostSource, I, J, r: int):
    """G = A[I,J] and its rank-r truncated pseudo-inverse."""
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    k = len(I)
    G = np.zeros((k, k))
    U = np.zeros((k, k))
    cond = C.c_double(0.0)
    rc = lib().oracle_nucleus_trunc(C.byref(src.struct), _ptr(I), _ptr(J), k, int(r), _ptr(G), _ptr(U),
                                    C.byref(cond))
    return rc, G, U, cond.value


def residual_explicit(src: HostSource, I, J, U, Q, S):
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    U = np.ascontiguousarray(U, dtype=np.float64)
    Q = np.ascontiguousarray(Q, dtype=np.int64)
    S = np.ascontiguousarray(S, dtype=np.int64)
    out = np.zeros(6)
    lib().oracle_residual_explicit(C.byref(src.struct), src.m, src.n, len(I), _ptr(I), _ptr(J), _ptr(U),
                                   _ptr(Q), len(Q), _ptr(S), len(S), _ptr(out))
    return dict(norm_e=out[0], norm_a=out[1], mean=out[2], var=out[3], est_abs=out[4], est_rel=out[5])


def splitmix64(seed: int, ctr: int) -> int:
    return int(lib().oracle_splitmix64(seed, ctr))


def draw_distinct(seed: int, n: int, cnt: int) -> np.ndarray:
    out = np.zeros(cnt, dtype=np.int64)
    lib().oracle_draw_distinct(seed, n, cnt, _ptr(out))
    return out
