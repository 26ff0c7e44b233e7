"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every symbol that include/lra.h declares, and its argument checks reject
invalid calls before touching a device."""
import ctypes as C
import os
import re

import pytest

from paper_1611_01391_amd import lra

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lra.h")).read()
    return sorted(set(re.findall(r"\b(lra_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared() == sorted(lra.EXPORTS)


def test_library_exports_every_symbol():
    L = lra.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_status_strings_and_version():
    assert lra.status_str(lra.OK) == "ok"
    assert "invalid" in lra.status_str(lra.EINVAL)
    assert lra.lib().lra_version().decode().startswith("lra-gfx950")


def test_default_options():
    o = lra.default_options()
    assert o.tau == 0.01 and o.k_step == 8 and o.warm_start == 1 and o.sample_q == 64


def test_create_rejects_null():
    assert lra.lib().lra_create(None, None, 0) == lra.EINVAL


def test_calls_reject_null_context():
    L = lra.lib()
    res = lra.ResultC()
    src = lra.Source()
    assert L.lra_ca_cur(None, C.byref(src), 10, 10, 2, 1, 0.0, None, C.byref(res)) == lra.EINVAL
    assert L.lra_ca_cur_batched(None, None, 1, None, None) == lra.EINVAL
    assert L.lra_ca_cur_noalloc(None, C.byref(src), 10, 10, 2, 1, 0.0, None, C.byref(res)) == lra.EINVAL


def test_noalloc_scratch_size_matches_header():
    text = open(os.path.join(ROOT, "include", "lra.h")).read()
    m = re.search(r"#define LRA_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == lra.NOALLOC_SCRATCH_BYTES
    assert "fixed scratch" in lra.status_str(lra.ESCRATCH)


def test_block_records_filled_field_by_field():
    """The batched call's block records are written through a numpy view of
    the C array: each record must read back, through ctypes, exactly the
    fields a per-element assignment would have written."""
    class Src:
        def __init__(self, i):
            self.struct = lra.Source()
            self.struct.kind = i % 4
            self.struct.dtype = i % 2
            self.struct.a = 4096 + 8 * i
            self.struct.lda = 1000 + i
            self.struct.col_major = i % 2
            self.struct.pre_depth = i % 3
            self.struct.x = 77 + i
            self.struct.y = 99 + i
            self.struct.pre_seed = (1 << 63) + i
            self.m, self.n = 500 + i, 700 + 2 * i
    blocks = [(Src(i), 8 + i % 5, 1 + i % 4, 1e-8 * (i + 1)) for i in range(37)]
    arr = lra._block_array(blocks)
    for i, (src, k, sweeps, tol) in enumerate(blocks):
        r = arr[i]
        for f, _ in lra.Source._fields_:
            assert getattr(r.src, f) == getattr(src.struct, f), (i, f)
        assert (r.m, r.n, r.k, r.sweeps, r.tol) == (src.m, src.n, k, sweeps, tol), i
    assert len(lra._block_array([])) == 1
