"""Checks of a sort's result that use neither sort implementation.

Each helper states a property the output of the method must have whatever the input:
the sorted sequence is nondecreasing; it is a permutation of the input (identical 2^16-bin histogram
of the top 16 bits and identical order-independent multiset hashes); the P cells of the output
contract (Sec. 1.1, footnote to Sec. 3.4.2) differ in size by at most one with the lower ids larger
and sum to n; every splitter equals the first key of its cell and the splitters never decrease.
"""
from __future__ import annotations

import numpy as np

_M64 = (1 << 64) - 1


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea & Flood 2014) applied elementwise to uint64 values."""
    z = x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def multiset_hash(keys: np.ndarray) -> tuple[int, int]:
    """(sum, xor) of SplitMix64(key) over the keys, both mod 2^64; independent of order."""
    h = splitmix64(np.asarray(keys, dtype=np.uint32))
    with np.errstate(over="ignore"):
        s = int(np.sum(h, dtype=np.uint64))
    x = int(np.bitwise_xor.reduce(h)) if h.size else 0
    return s, x


def hist_top16(keys: np.ndarray) -> np.ndarray:
    return np.bincount(np.asarray(keys, dtype=np.uint32) >> np.uint32(16), minlength=1 << 16)


def is_nondecreasing(a: np.ndarray) -> bool:
    a = np.asarray(a, dtype=np.uint32)
    return bool(a.size < 2 or np.all(a[1:] >= a[:-1]))


def same_multiset(a: np.ndarray, b: np.ndarray) -> bool:
    return (np.asarray(a).size == np.asarray(b).size
            and np.array_equal(hist_top16(a), hist_top16(b))
            and multiset_hash(a) == multiset_hash(b))


def check_cell_sizes(n: int, P: int, starts: np.ndarray) -> None:
    starts = np.asarray(starts, dtype=np.int64)
    assert starts.size == P + 1
    assert starts[0] == 0 and starts[-1] == n
    sizes = np.diff(starts)
    assert sizes.min() >= 0
    assert sizes.max() - sizes.min() <= 1
    # lower ids take the extra element: sizes never increase with the cell id
    assert np.all(sizes[1:] <= sizes[:-1])


def check_splitters(sorted_keys: np.ndarray, P: int, spl: np.ndarray) -> None:
    """Each splitter p-1 is >= every key of cells < p and <= every key of cells >= p, and equals
    the first key of cell p when that cell is non-empty (all-ones when it is empty)."""
    s = np.asarray(sorted_keys, dtype=np.uint32)
    spl = np.asarray(spl, dtype=np.uint32)
    n = s.size
    assert spl.size == max(P - 1, 0)
    q, r = divmod(n, P)
    for p in range(1, P):
        start = p * q + min(p, r)
        size = q + (1 if p < r else 0)
        if size == 0:
            assert spl[p - 1] == 0xFFFFFFFF
        else:
            assert spl[p - 1] == s[start]
            if start > 0:
                assert s[start - 1] <= spl[p - 1]
    if spl.size > 1:
        assert np.all(spl[1:] >= spl[:-1])
