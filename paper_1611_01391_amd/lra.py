"""Thin ctypes binding of the gfx950 C-A / CUR library (include/lra.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Device memory and streams come from PyTorch tensors; the
library never sees a torch type.  If the built library is missing the
binding raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "liblra.so")

# status codes (lra_status)
OK, TOL_NOT_MET, MAXVOL_CAP, NUMERICAL_RANK, PENDING = 0, 1, 2, 3, 4
EINVAL, ERANK, ENOMEM, EBUDGET, EDEVICE, ENONFINITE, ESCRATCH = -1, -2, -3, -4, -5, -6, -7
# fixed device workspace of lra_ca_cur_noalloc (LRA_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20
SRC_DENSE, SRC_CAUCHY, SRC_INVDIST, SRC_PREPROCESSED = 0, 1, 2, 3
F32, F64 = 0, 1
PREC_FP64, PREC_MIXED, PREC_BF16SEL = 0, 1, 2

# every entry point declared in include/lra.h
EXPORTS = ["lra_default_options", "lra_create", "lra_destroy", "lra_ca_cur", "lra_maxvol",
           "lra_ca_cur_batched", "lra_submit", "lra_poll", "lra_wait", "lra_serve_config", "lra_set_timing",
           "lra_autotune_team", "lra_autotune_batched", "lra_tuning_save", "lra_tuning_load",
           "lra_get_stats", "lra_status_str", "lra_version", "lra_ca_cur_noalloc", "lra_cur_factors",
           "lra_top_svd"]


class LraError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_str(status)} ({status})")
        self.status = status


class Source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dtype", C.c_int32), ("a", C.c_void_p), ("lda", C.c_int64),
                ("col_major", C.c_int32), ("pre_depth", C.c_int32), ("x", C.c_void_p),
                ("y", C.c_void_p), ("pre_seed", C.c_uint64)]


class Options(C.Structure):
    _fields_ = [("tau", C.c_double), ("k_max", C.c_int32), ("k_step", C.c_int32),
                ("max_swaps", C.c_int32), ("warm_start", C.c_int32), ("precision", C.c_int32),
                ("sample_q", C.c_int32), ("sample_s", C.c_int32), ("team_wgs", C.c_int32),
                ("reserved", C.c_int32), ("seed", C.c_uint64), ("init_cols", C.c_void_p),
                ("n_init_cols", C.c_int64), ("sample_rows", C.c_void_p),
                ("sample_cols", C.c_void_p), ("cur_rank", C.c_int32), ("inner_sweeps", C.c_int32),
                ("nucleus_rank", C.c_int32), ("reserved2", C.c_int32), ("init_rows", C.c_void_p)]


class ResultC(C.Structure):
    _fields_ = [("I", C.c_void_p), ("J", C.c_void_p), ("G", C.c_void_p), ("U", C.c_void_p),
                ("C_out", C.c_void_p), ("R_out", C.c_void_p), ("k", C.c_int32),
                ("status", C.c_int32), ("sweeps_done", C.c_int32), ("swaps_total", C.c_int32),
                ("entries_read", C.c_int64), ("err_est_rel", C.c_double),
                ("err_est_abs", C.c_double), ("err_mean", C.c_double), ("err_var", C.c_double),
                ("nucleus_cond1", C.c_double), ("t_submit_us", C.c_double),
                ("t_start_us", C.c_double), ("t_end_us", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("launches", C.c_int64), ("engine_ms_total", C.c_double),
                ("last_engine_ms", C.c_double), ("last_grid", C.c_int32),
                ("last_teams", C.c_int32), ("ticks", C.c_int64), ("device_allocs", C.c_int64),
                ("device_bytes", C.c_int64)]


class Block(C.Structure):
    _fields_ = [("src", Source), ("m", C.c_int64), ("n", C.c_int64), ("k", C.c_int32),
                ("sweeps", C.c_int32), ("tol", C.c_double)]


_BLOCK_DT = np.dtype(Block)
_RESULT_DT = np.dtype(ResultC)
_SOURCE_DT = np.dtype(Source)


def _block_array(blocks):
    """The C array of lra_block for a sequence of (DeviceSource, k, sweeps,
    tol), filled a field at a time over all blocks (thousands of far-field
    blocks per call: per-element ctypes assignments cost milliseconds)."""
    nb = len(blocks)
    arr = (Block * max(1, nb))()
    if nb:
        a = np.frombuffer(arr, dtype=_BLOCK_DT)
        a["src"] = np.frombuffer(b"".join([bytes(b[0].struct) for b in blocks]), dtype=_SOURCE_DT)
        a["m"] = [b[0].m for b in blocks]
        a["n"] = [b[0].n for b in blocks]
        a["k"] = [int(b[1]) for b in blocks]
        a["sweeps"] = [int(b[2]) for b in blocks]
        a["tol"] = [float(b[3]) for b in blocks]
    return arr


class RequestC(C.Structure):
    _fields_ = [("src", Source), ("m", C.c_int64), ("n", C.c_int64), ("k", C.c_int32),
                ("sweeps", C.c_int32), ("tol", C.c_double), ("opts", Options),
                ("result", C.POINTER(ResultC))]


_lib = None


def lib():
    """Load liblra.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1611_01391_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.lra_default_options.argtypes = [C.POINTER(Options)]
        L.lra_default_options.restype = None
        L.lra_create.argtypes = [C.POINTER(P), P, C.c_size_t]
        L.lra_create.restype = C.c_int
        L.lra_destroy.argtypes = [P]
        L.lra_destroy.restype = None
        L.lra_ca_cur.argtypes = [P, C.POINTER(Source), C.c_int64, C.c_int64, C.c_int, C.c_int,
                                 C.c_double, C.POINTER(Options), C.POINTER(ResultC)]
        L.lra_ca_cur.restype = C.c_int
        L.lra_ca_cur_noalloc.argtypes = L.lra_ca_cur.argtypes
        L.lra_ca_cur_noalloc.restype = C.c_int
        L.lra_cur_factors.argtypes = [P, C.POINTER(Source), C.c_int64, C.c_int64, C.c_int, P, P, C.c_int32, P, P]
        L.lra_cur_factors.restype = C.c_int
        L.lra_top_svd.argtypes = [P, C.c_int64, C.c_int64, C.c_int, C.c_int, C.c_int32, P, C.c_int64, P, P,
                                  C.c_int64, P, C.c_int64, P, P, C.c_int64, P, P]
        L.lra_top_svd.restype = C.c_int
        L.lra_maxvol.argtypes = [P, P, C.c_int32, C.c_int64, C.c_int64, C.c_int, C.c_double,
                                 C.c_int, P, P, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.lra_maxvol.restype = C.c_int
        L.lra_ca_cur_batched.argtypes = [P, C.POINTER(Block), C.c_int, C.POINTER(Options),
                                         C.POINTER(ResultC)]
        L.lra_ca_cur_batched.restype = C.c_int
        L.lra_submit.argtypes = [P, C.POINTER(RequestC), C.POINTER(C.c_uint64)]
        L.lra_submit.restype = C.c_int
        L.lra_poll.argtypes = [P, C.c_uint64]
        L.lra_poll.restype = C.c_int
        L.lra_wait.argtypes = [P, C.c_uint64]
        L.lra_wait.restype = C.c_int
        L.lra_serve_config.argtypes = [P, C.c_size_t, C.c_int, C.c_int]
        L.lra_serve_config.restype = C.c_int
        L.lra_autotune_team.argtypes = [P, C.POINTER(Source), C.c_int64, C.c_int64, C.c_int, C.c_int,
                                        C.c_double, C.POINTER(Options), C.POINTER(C.c_int),
                                        C.POINTER(C.c_double)]
        L.lra_autotune_team.restype = C.c_int
        L.lra_autotune_batched.argtypes = [P, C.POINTER(Block), C.c_int, C.POINTER(Options),
                                           C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.lra_autotune_batched.restype = C.c_int
        L.lra_tuning_save.argtypes = [P, C.c_char_p]
        L.lra_tuning_save.restype = C.c_int
        L.lra_tuning_load.argtypes = [P, C.c_char_p]
        L.lra_tuning_load.restype = C.c_int
        L.lra_set_timing.argtypes = [P, C.c_int, C.c_int]
        L.lra_set_timing.restype = C.c_int
        L.lra_get_stats.argtypes = [P, C.POINTER(Stats)]
        L.lra_get_stats.restype = C.c_int
        L.lra_status_str.argtypes = [C.c_int]
        L.lra_status_str.restype = C.c_char_p
        L.lra_version.argtypes = []
        L.lra_version.restype = C.c_char_p
        _lib = L
    return _lib


def status_str(s: int) -> str:
    return lib().lra_status_str(int(s)).decode()


def default_options(**kw) -> Options:
    o = Options()
    lib().lra_default_options(C.byref(o))
    for key, val in kw.items():
        if not hasattr(o, key):
            raise TypeError(f"unknown option {key}")
        setattr(o, key, val)
    return o


# ---------------------------------------------------------------------------
# sources over torch device tensors
# ---------------------------------------------------------------------------

def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError("sources must be float32 or float64 tensors")


def _require_cuda(t):
    if not t.is_cuda:
        raise TypeError("sources must live in device memory (a cuda tensor)")


@dataclass
class DeviceSource:
    struct: Source
    m: int
    n: int
    keep: tuple = ()


def dense(A, col_major: bool = False) -> DeviceSource:
    """A dense m x n device matrix (row-major tensor, or a column-major view)."""
    _require_cuda(A)
    m, n = A.shape
    if col_major:
        if A.stride(0) != 1:
            raise ValueError("col_major source needs stride(0) == 1")
        lda = A.stride(1)
    else:
        if A.stride(1) != 1:
            raise ValueError("row-major source needs stride(1) == 1")
        lda = A.stride(0)
    s = Source(SRC_DENSE, _dtype_code(A), A.data_ptr(), lda, 1 if col_major else 0, 0, None, None)
    return DeviceSource(s, m, n, (A,))


def preprocessed(A, depth: int, seed: int = 0, col_major: bool = False) -> DeviceSource:
    """F A H: the dense device matrix A through d-abridged Hadamard
    multipliers with random sign scaling on both sides (orthogonal F, H);
    2^depth must divide both dimensions."""
    src = dense(A, col_major)
    src.struct.kind = SRC_PREPROCESSED
    src.struct.pre_depth = int(depth)
    src.struct.pre_seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return src


def cauchy(x, y) -> DeviceSource:
    """a_ij = 1 / (x_i - y_j) for device vectors x (m) and y (n)."""
    _require_cuda(x)
    _require_cuda(y)
    if x.dtype != y.dtype or not x.is_contiguous() or not y.is_contiguous():
        raise ValueError("x and y must be contiguous and of one dtype")
    s = Source(SRC_CAUCHY, _dtype_code(x), None, 0, 0, 0, x.data_ptr(), y.data_ptr())
    return DeviceSource(s, x.numel(), y.numel(), (x, y))


def invdist(x, y) -> DeviceSource:
    """a_ij = 1 / |x_i - y_j| (0 where equal) for device point sets x, y."""
    src = cauchy(x, y)
    src.struct.kind = SRC_INVDIST
    return src


# ---------------------------------------------------------------------------
# results
# ---------------------------------------------------------------------------

@dataclass
class Result:
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
    t_submit_us: float = 0.0
    t_start_us: float = 0.0
    t_end_us: float = 0.0
    C: object = None
    R: object = None


class _ResultBuf:
    def __init__(self, kcap: int):
        self.kcap = kcap
        self.I = np.zeros(kcap, dtype=np.int64)
        self.J = np.zeros(kcap, dtype=np.int64)
        self.G = np.zeros(kcap * kcap)
        self.U = np.zeros(kcap * kcap)
        self.c = ResultC()
        self.c.I = self.I.ctypes.data
        self.c.J = self.J.ctypes.data
        self.c.G = self.G.ctypes.data
        self.c.U = self.U.ctypes.data

    def to_result(self, C_t=None, R_t=None) -> Result:
        r = self.c
        k = max(0, r.k)
        return Result(r.status, k, self.I[:k].copy(), self.J[:k].copy(),
                      self.G[:k * k].reshape(k, k).copy(), self.U[:k * k].reshape(k, k).copy(),
                      r.sweeps_done, r.swaps_total, r.entries_read, r.err_est_rel, r.err_est_abs,
                      r.err_mean, r.err_var, r.nucleus_cond1, r.t_submit_us, r.t_start_us,
                      r.t_end_us, C_t, R_t)


def _i64(a) -> Optional[np.ndarray]:
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _options(opts: dict, init_cols=None, sample_rows=None, sample_cols=None):
    """lra_options from keyword options; host index arrays (init_cols,
    sample_rows, sample_cols, init_rows) are converted and returned with the
    struct so that they outlive the call."""
    opts = dict(opts)
    rows = _i64(opts.pop("init_rows", None))
    o = default_options(**opts)
    cand, Q, S = _i64(init_cols), _i64(sample_rows), _i64(sample_cols)
    if cand is not None:
        o.init_cols = cand.ctypes.data
        o.n_init_cols = len(cand)
    if Q is not None:
        o.sample_rows = Q.ctypes.data
        o.sample_q = len(Q)
    if S is not None:
        o.sample_cols = S.ctypes.data
        o.sample_s = len(S)
    if rows is not None:
        o.init_rows = rows.ctypes.data
    return o, (cand, Q, S, rows)


# ---------------------------------------------------------------------------
# context
# ---------------------------------------------------------------------------

class Context:
    """An lra_ctx bound to the current device and torch's current stream."""

    def __init__(self, stream=None, hbm_budget_bytes: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the library runs on gfx950 only")
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self._h = C.c_void_p()
        st = lib().lra_create(C.byref(self._h), C.c_void_p(stream.cuda_stream), hbm_budget_bytes)
        if st != OK:
            raise LraError(st, "lra_create")
        self._keep = {}

    def close(self):
        if self._h:
            lib().lra_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- kernel timing ----------------------------------------------------
    def set_timing(self, enable: bool = True, reset: bool = True):
        st = lib().lra_set_timing(self._h, 1 if enable else 0, 1 if reset else 0)
        if st != OK:
            raise LraError(st, "lra_set_timing")

    def stats(self) -> dict:
        s = Stats()
        lib().lra_get_stats(self._h, C.byref(s))
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    # -- one problem ------------------------------------------------------
    def ca_cur(self, src: DeviceSource, k: int, sweeps: int, tol: float = 0.0, *,
               init_cols=None, sample_rows=None, sample_cols=None, factors: bool = False,
               raise_on_error: bool = True, **opts) -> Result:
        return self._ca_cur("lra_ca_cur", src, k, sweeps, tol, init_cols, sample_rows, sample_cols,
                            factors, raise_on_error, opts)

    def ca_cur_noalloc(self, src: DeviceSource, k: int, sweeps: int, tol: float = 0.0, *,
                       init_cols=None, sample_rows=None, sample_cols=None, factors: bool = False,
                       raise_on_error: bool = True, **opts) -> Result:
        """lra_ca_cur_noalloc: as ca_cur, with the library's fixed per-device
        workspace instead of allocated memory (the C_out / R_out tensors of
        factors=True are the caller's, allocated here before the call)."""
        return self._ca_cur("lra_ca_cur_noalloc", src, k, sweeps, tol, init_cols, sample_rows, sample_cols,
                            factors, raise_on_error, opts)

    def _ca_cur(self, fn, src, k, sweeps, tol, init_cols, sample_rows, sample_cols, factors, raise_on_error,
                opts) -> Result:
        import torch
        o, keep = _options(opts, init_cols, sample_rows, sample_cols)
        kcap = max(k, o.k_max)
        buf = _ResultBuf(kcap)
        C_t = R_t = None
        if factors:
            dt = torch.float64 if o.precision == PREC_FP64 else torch.float32
            dev = src.keep[0].device
            C_t = torch.empty(kcap * src.m, dtype=dt, device=dev)
            R_t = torch.empty(kcap * src.n, dtype=dt, device=dev)
            buf.c.C_out = C_t.data_ptr()
            buf.c.R_out = R_t.data_ptr()
        st = getattr(lib(), fn)(self._h, C.byref(src.struct), src.m, src.n, int(k), int(sweeps),
                                float(tol), C.byref(o), C.byref(buf.c))
        if st < 0 and raise_on_error:
            raise LraError(st, fn)
        if st < 0:
            buf.c.status = st
        res = buf.to_result()
        if factors and st >= 0:
            kk = res.k
            res.C = C_t[:kk * src.m].view(kk, src.m).t()       # m x k (column-major)
            res.R = R_t[:kk * src.n].view(kk, src.n)           # k x n (row-major)
        return res

    # -- CUR factors of given index sets ---------------------------------
    def cur_factors(self, src: DeviceSource, I, J, dtype=None, C_out=None, R_out=None):
        """lra_cur_factors: C = A[:, J] (returned as an m x k view of a
        column-major buffer) and R = A[I, :] (k x n), on the device."""
        import torch
        I, J = _i64(I), _i64(J)
        k = len(I)
        if len(J) != k:
            raise ValueError("I and J must have the same length")
        dt = dtype or (torch.float64 if src.struct.dtype == F64 else torch.float32)
        dev = src.keep[0].device
        if C_out is None:
            C_out = torch.empty(k * src.m, dtype=dt, device=dev)
        if R_out is None:
            R_out = torch.empty(k * src.n, dtype=dt, device=dev)
        st = lib().lra_cur_factors(self._h, C.byref(src.struct), src.m, src.n, k, I.ctypes.data, J.ctypes.data,
                                   F64 if dt == torch.float64 else F32, C_out.data_ptr(), R_out.data_ptr())
        if st != OK:
            raise LraError(st, "lra_cur_factors")
        return C_out.view(k, src.m).t(), R_out.view(k, src.n)

    # -- LRA -> top SVD ---------------------------------------------------
    def top_svd(self, Cf, W, Rf, r: int, S_out=None, Tt_out=None):
        """lra_top_svd: the rank-r top SVD S diag(sigma) T^T of the LRA
        C W R.  Cf: m x k device tensor with stride(0) == 1 (a column-major
        view, as cur_factors returns), Rf: k x n device tensor with
        stride(1) == 1, both float32 or float64; W: k x k host array.
        Returns (S: m x r column-major view, sigma: numpy array, Tt: r x n,
        piv_c, piv_r)."""
        import torch
        _require_cuda(Cf)
        _require_cuda(Rf)
        m, k = Cf.shape
        k2, n = Rf.shape
        if k2 != k or Cf.dtype != Rf.dtype or Cf.dtype not in (torch.float32, torch.float64):
            raise ValueError("C (m x k) and R (k x n) of one floating dtype")
        if Cf.stride(0) != 1 and k > 1:
            raise ValueError("C needs stride(0) == 1 (a column-major view)")
        if Rf.stride(1) != 1 and n > 1:
            raise ValueError("R needs stride(1) == 1 (row-major)")
        ldc = Cf.stride(1) if k > 1 else m
        ldr = Rf.stride(0) if k > 1 else n
        Wh = np.ascontiguousarray(np.asarray(W, dtype=np.float64))
        if Wh.shape != (k, k):
            raise ValueError("W must be k x k")
        if S_out is None:
            S_out = torch.empty(r * m, dtype=torch.float64, device=Cf.device)
        if Tt_out is None:
            Tt_out = torch.empty(r * n, dtype=torch.float64, device=Cf.device)
        sigma = np.zeros(r)
        pc = np.zeros(k, dtype=np.int64)
        pr = np.zeros(k, dtype=np.int64)
        st = lib().lra_top_svd(self._h, m, n, k, int(r), F64 if Cf.dtype == torch.float64 else F32, Cf.data_ptr(),
                               ldc, Wh.ctypes.data, Rf.data_ptr(), ldr, S_out.data_ptr(), m, sigma.ctypes.data,
                               Tt_out.data_ptr(), n, pc.ctypes.data, pr.ctypes.data)
        if st != OK:
            raise LraError(st, "lra_top_svd")
        return S_out.view(r, m).t(), sigma, Tt_out.view(r, n), pc, pr

    # -- maxvol alone -----------------------------------------------------
    def maxvol(self, strip, tau: float = 0.01, init=None, max_swaps: int = 0):
        """maxvol on an m x k device strip (any layout with unit row stride of
        a column-major view, i.e. strip.stride(0) == 1)."""
        _require_cuda(strip)
        m, k = strip.shape
        if strip.stride(0) != 1:
            strip = strip.t().contiguous().t()
        ld = strip.stride(1) if k > 1 else m
        I = np.zeros(k, dtype=np.int64)
        init_a = _i64(init)
        sw = C.c_int(0)
        ke = C.c_int(0)
        st = lib().lra_maxvol(self._h, strip.data_ptr(), _dtype_code(strip), m, ld, int(k),
                              float(tau), int(max_swaps),
                              None if init_a is None else init_a.ctypes.data, I.ctypes.data,
                              C.byref(sw), C.byref(ke))
        if st < 0:
            raise LraError(st, "lra_maxvol")
        return dict(I=I[:ke.value].copy(), swaps=sw.value, k_eff=ke.value, status=st)

    # -- autotuning -------------------------------------------------------
    def autotune_team(self, src: DeviceSource, k: int, sweeps: int, tol: float = 0.0, *,
                      init_cols=None, sample_rows=None, sample_cols=None, **opts):
        """Time team sizes for problems of this size class; returns (team, ms)."""
        o, keep = _options(opts, init_cols, sample_rows, sample_cols)
        team = C.c_int(0)
        ms = C.c_double(0.0)
        st = lib().lra_autotune_team(self._h, C.byref(src.struct), src.m, src.n, int(k), int(sweeps),
                                     float(tol), C.byref(o), C.byref(team), C.byref(ms))
        if st != OK:
            raise LraError(st, "lra_autotune_team")
        return team.value, ms.value

    def autotune_batched(self, blocks: Sequence[tuple], **opts):
        """Time planning floors for shared launches; returns (floor_rows, ms)."""
        o = default_options(**opts)
        nb = len(blocks)
        arr = _block_array(blocks)
        fl = C.c_int64(0)
        ms = C.c_double(0.0)
        st = lib().lra_autotune_batched(self._h, arr, nb, C.byref(o), C.byref(fl), C.byref(ms))
        if st != OK:
            raise LraError(st, "lra_autotune_batched")
        return fl.value, ms.value

    def tuning_save(self, path: str):
        st = lib().lra_tuning_save(self._h, path.encode())
        if st != OK:
            raise LraError(st, "lra_tuning_save")

    def tuning_load(self, path: str):
        st = lib().lra_tuning_load(self._h, path.encode())
        if st != OK:
            raise LraError(st, "lra_tuning_load")

    # -- batched ----------------------------------------------------------
    def ca_cur_batched(self, blocks: Sequence[tuple], raise_on_error: bool = True, **opts):
        """blocks: sequence of (DeviceSource, k, sweeps, tol).  Returns
        (worst status, list of Result); the index and nucleus arrays of all
        blocks are views into shared buffers."""
        o = default_options(**opts)
        nb = len(blocks)
        arr = _block_array(blocks)
        kcaps = np.maximum(np.frombuffer(arr, dtype=_BLOCK_DT)["k"][:nb].astype(np.int64), o.k_max)
        off = np.zeros(max(1, nb) + 1, dtype=np.int64)
        off2 = np.zeros(max(1, nb) + 1, dtype=np.int64)
        np.cumsum(kcaps, out=off[1:nb + 1])
        np.cumsum(kcaps * kcaps, out=off2[1:nb + 1])
        I = np.zeros(max(1, off[nb]), dtype=np.int64)
        J = np.zeros(max(1, off[nb]), dtype=np.int64)
        G = np.zeros(max(1, off2[nb]))
        U = np.zeros(max(1, off2[nb]))
        # the result records, filled field by field over all blocks at once
        res_arr = (ResultC * max(1, nb))()
        rv = np.frombuffer(res_arr, dtype=_RESULT_DT)[:nb]
        rv["I"] = I.ctypes.data + 8 * off[:nb]
        rv["J"] = J.ctypes.data + 8 * off[:nb]
        rv["G"] = G.ctypes.data + 8 * off2[:nb]
        rv["U"] = U.ctypes.data + 8 * off2[:nb]
        st = lib().lra_ca_cur_batched(self._h, arr, nb, C.byref(o), res_arr)
        if st < 0 and raise_on_error and st not in (ERANK, ENONFINITE):
            raise LraError(st, "lra_ca_cur_batched")
        ks = np.maximum(rv["k"], 0).tolist()
        i0s, g0s = off[:nb].tolist(), off2[:nb].tolist()
        f = [rv[name].tolist() for name in ("status", "sweeps_done", "swaps_total", "entries_read", "err_est_rel",
                                            "err_est_abs", "err_mean", "err_var", "nucleus_cond1")]
        out = []
        for b in range(nb):
            k, i0, g0 = ks[b], i0s[b], g0s[b]
            out.append(Result(f[0][b], k, I[i0:i0 + k], J[i0:i0 + k],
                              G[g0:g0 + k * k].reshape(k, k), U[g0:g0 + k * k].reshape(k, k),
                              f[1][b], f[2][b], f[3][b], f[4][b], f[5][b], f[6][b], f[7][b], f[8][b]))
        return st, out

    # -- serving ----------------------------------------------------------
    def serve_config(self, arena_bytes: int = 0, phases_per_tick: int = 0, max_active: int = 0):
        st = lib().lra_serve_config(self._h, int(arena_bytes), int(phases_per_tick), int(max_active))
        if st != OK:
            raise LraError(st, "lra_serve_config")

    def submit(self, src: DeviceSource, k: int, sweeps: int, tol: float = 0.0, *,
               init_cols=None, sample_rows=None, sample_cols=None, **opts) -> int:
        """Queue one request; returns its ticket (see poll / wait)."""
        o, keep = _options(opts, init_cols, sample_rows, sample_cols)
        buf = _ResultBuf(max(int(k), o.k_max))
        req = RequestC()
        req.src = src.struct
        req.m = src.m
        req.n = src.n
        req.k = int(k)
        req.sweeps = int(sweeps)
        req.tol = float(tol)
        req.opts = o
        req.result = C.pointer(buf.c)
        t = C.c_uint64(0)
        st = lib().lra_submit(self._h, C.byref(req), C.byref(t))
        if st < 0:
            raise LraError(st, "lra_submit")
        self._keep[t.value] = (buf, src)
        return t.value

    def poll(self, ticket: int) -> Optional[Result]:
        """None while pending, else the Result (status < 0 for a failed request)."""
        st = lib().lra_poll(self._h, ticket)
        if st == PENDING:
            return None
        if ticket not in self._keep:
            raise LraError(st, "lra_poll")
        buf, _ = self._keep.pop(ticket)
        buf.c.status = st
        return buf.to_result()

    def wait(self, ticket: int) -> Result:
        st = lib().lra_wait(self._h, ticket)
        if ticket not in self._keep:
            raise LraError(st, "lra_wait")
        buf, _ = self._keep.pop(ticket)
        buf.c.status = st
        return buf.to_result()
