"""apsort: radix sort of 32-bit integer keys on MI355X (gfx950).

The sort runs in hand-written HIP kernels inside ``libapsort.so``; ``binding`` is a thin ctypes
layer over its C ABI (``include/apsort.h``).  Importing this package loads nothing: the library is
opened on first use, and every entry point raises if it is missing.
"""
from __future__ import annotations

__all__ = ["binding", "inputs"]
