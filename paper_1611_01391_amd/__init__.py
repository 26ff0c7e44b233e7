"""MI355X (gfx950) Cross-Approximation / CUR low-rank approximation.

The library itself is ``lib/liblra.so`` (C ABI in ``include/lra.h``, built by
``build.py``); ``lra`` is its thin ctypes binding.
"""
from . import lra  # noqa: F401
from .lra import Context, cauchy, dense, invdist  # noqa: F401

__all__ = ["lra", "Context", "dense", "cauchy", "invdist"]
