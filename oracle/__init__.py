"""CPU oracle for the radix sort of 32-bit keys (Weaver & Lynes, "Sorting Integers on the AP1000").

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline leg are
the only callers.  The HIP library never imports, links or calls anything here, and nothing here
imports the HIP package.  The arithmetic lives in ``apsort_oracle.c`` (plain C, single-threaded
except for the timing variant, compiled with gcc); this module only marshals numpy arrays into it.

Functions and the passages they follow:
  digit_hist      -- Sec. 3.2, first loop of bucket(): per-digit bucket counts.
  bucket_pass     -- Sec. 3.2 bucketing of one 8-bit digit (counts, cumulative totals, partial sort).
  sort_u32        -- Sec. 3.3.1 LSD radix sort, each pass being the Sec. 3.2 bucketing step.
  sort_u32_mt     -- the same passes, each split over host threads (for the CPU timing baseline).
  slice_starts    -- Sec. 1.1 even distribution over P cells, lower cell takes the extra element
                     (footnote to Sec. 3.4.2).
  splitters       -- first key of each cell p = 1..P-1, all-ones sentinel for an empty cell
                     ("infinity padding", Sec. 2.1.1).
  sort_segmented  -- one independent local sort per segment (Sec. 3.3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "apsort_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so (plain -O2, no vectorisation tricks)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _bind(path: str):
    """Open a compiled oracle library and declare its C signatures."""
    lib = ctypes.CDLL(path)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_digit_hist.argtypes = [u32p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, u64p]
    lib.oracle_sort_u32.argtypes = [u32p, u32p, ctypes.c_size_t]
    lib.oracle_sort_u32_mt.argtypes = [u32p, u32p, ctypes.c_size_t, ctypes.c_int]
    lib.oracle_sort_u32_mt.restype = ctypes.c_int
    lib.oracle_bucket_pass.argtypes = [u32p, u32p, ctypes.c_size_t, ctypes.c_int]
    lib.oracle_bucket_pass.restype = None
    lib.oracle_slice_starts.argtypes = [ctypes.c_size_t, ctypes.c_int, u64p]
    lib.oracle_splitters.argtypes = [u32p, ctypes.c_size_t, ctypes.c_int, u32p]
    lib.oracle_sort_segmented.argtypes = [u32p, u64p, ctypes.c_int]
    lib.oracle_bucket_pass_pairs.argtypes = [u32p, u32p, u32p, u32p, ctypes.c_size_t, ctypes.c_int]
    lib.oracle_bucket_pass_pairs.restype = None
    lib.oracle_sort_pairs_u32.argtypes = [u32p, u32p, u32p, u32p, ctypes.c_size_t]
    lib.oracle_merge_u32.argtypes = [u32p, ctypes.c_size_t, u32p, ctypes.c_size_t, u32p]
    for f in (lib.oracle_digit_hist, lib.oracle_sort_u32, lib.oracle_slice_starts,
              lib.oracle_splitters, lib.oracle_sort_segmented):
        f.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _bind(_LIB)
    return _lib


def _u32(a) -> np.ndarray:
    """uint32 view of ``a``: int32 is reinterpreted bit for bit, wider integers must fit in 32 bits."""
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        return a
    if a.dtype == np.int32:
        return a.view(np.uint32)
    if a.dtype.kind in "iu":
        if a.size and (a.min() < 0 or a.max() > 0xFFFFFFFF):
            raise ValueError("keys must be 32-bit unsigned values")
        return a.astype(np.uint32)
    raise TypeError(f"integer keys expected, got {a.dtype}")


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _p64(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def digit_hist(keys, shift: int, bits: int) -> np.ndarray:
    """Bucket counts of the ``bits``-bit digit at ``shift`` (Sec. 3.2)."""
    k = _u32(keys)
    h = np.zeros(1 << bits, dtype=np.uint64)
    if _load().oracle_digit_hist(_p32(k), k.size, shift, bits, _p64(h)) != 0:
        raise ValueError("oracle_digit_hist: invalid argument")
    return h


def bucket_pass(keys, shift: int) -> np.ndarray:
    """One stable bucketing pass on the 8-bit digit at ``shift`` (Sec. 3.2 partial sort)."""
    k = _u32(keys)
    out = np.empty_like(k)
    if not 0 <= shift <= 24:
        raise ValueError("shift must be in [0, 24]")
    if k.size:
        _load().oracle_bucket_pass(_p32(k), _p32(out), k.size, shift)
    return out


def sort_u32(keys) -> np.ndarray:
    """Sorted copy of ``keys`` by four stable 8-bit bucketing passes (Sec. 3.3.1)."""
    k = _u32(keys)
    out = np.empty_like(k)
    if k.size and _load().oracle_sort_u32(_p32(k), _p32(out), k.size) != 0:
        raise MemoryError("oracle_sort_u32 failed")
    return out


def sort_u32_mt(keys, threads: int) -> np.ndarray:
    """The same sort with every pass split over ``threads`` host threads (timing variant)."""
    k = _u32(keys)
    out = np.empty_like(k)
    if k.size and _load().oracle_sort_u32_mt(_p32(k), _p32(out), k.size, int(threads)) != 0:
        raise ValueError("oracle_sort_u32_mt: invalid argument or out of memory")
    return out


def slice_starts(n: int, P: int) -> np.ndarray:
    """First sorted position of each of the P cells, plus n at index P (Sec. 1.1)."""
    s = np.zeros(P + 1, dtype=np.uint64)
    if _load().oracle_slice_starts(n, P, _p64(s)) != 0:
        raise ValueError("oracle_slice_starts: invalid argument")
    return s


def splitters(sorted_keys, P: int) -> np.ndarray:
    """Lowest key of cells 1..P-1, all-ones for an empty cell."""
    k = _u32(sorted_keys)
    sp = np.zeros(max(P - 1, 0), dtype=np.uint32)
    if _load().oracle_splitters(_p32(k), k.size, P, _p32(sp) if P > 1 else None) != 0:
        raise ValueError("oracle_splitters: invalid argument")
    return sp


def sort_segmented(keys, offsets) -> np.ndarray:
    """Copy of ``keys`` with every segment [offsets[s], offsets[s+1]) sorted independently."""
    k = _u32(keys).copy()
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    nseg = off.size - 1
    if nseg < 0:
        raise ValueError("offsets needs at least one entry")
    if nseg and off[-1] > k.size:
        raise ValueError("offsets exceed the key array")
    if _load().oracle_sort_segmented(_p32(k), _p64(off), nseg) != 0:
        raise ValueError("oracle_sort_segmented: invalid offsets or out of memory")
    return k


def bucket_pass_pairs(keys, values, shift: int) -> tuple[np.ndarray, np.ndarray]:
    """One stable bucketing pass on the keys' 8-bit digit at ``shift``, values moving with keys."""
    k, v = _u32(keys), _u32(values)
    if k.size != v.size:
        raise ValueError("keys and values differ in length")
    if not 0 <= shift <= 24:
        raise ValueError("shift must be in [0, 24]")
    ok, ov = np.empty_like(k), np.empty_like(v)
    if k.size:
        _load().oracle_bucket_pass_pairs(_p32(k), _p32(v), _p32(ok), _p32(ov), k.size, shift)
    return ok, ov


def sort_pairs_u32(keys, values) -> tuple[np.ndarray, np.ndarray]:
    """(keys, values) sorted by key with four stable bucketing passes; equal keys keep input order."""
    k, v = _u32(keys), _u32(values)
    if k.size != v.size:
        raise ValueError("keys and values differ in length")
    ok, ov = np.empty_like(k), np.empty_like(v)
    if k.size and _load().oracle_sort_pairs_u32(_p32(k), _p32(v), _p32(ok), _p32(ov), k.size) != 0:
        raise MemoryError("oracle_sort_pairs_u32 failed")
    return ok, ov


def merge_u32(a, b) -> np.ndarray:
    """Merge of two nondecreasing key arrays (Sec. 3.4 / 4.6 merge step); ties take ``a`` first."""
    x, y = _u32(a), _u32(b)
    out = np.empty(x.size + y.size, dtype=np.uint32)
    if out.size and _load().oracle_merge_u32(_p32(x) if x.size else None, x.size,
                                             _p32(y) if y.size else None, y.size, _p32(out)) != 0:
        raise ValueError("oracle_merge_u32: invalid argument")
    return out
