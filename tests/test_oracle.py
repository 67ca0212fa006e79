"""Pins of the CPU oracle against things other than itself (CPU only).

- hand-worked fixtures under tests/golden/ (LSD trace, cell sizes), each citing its passage;
- library special cases: numpy.sort for the sorted sequence, numpy's stable argsort for a single
  bucketing pass, numpy.bincount for digit histograms;
- brute force: every sequence of length <= 5 over eight boundary values against Python's sorted();
- closed forms: a permutation of [0, n) sorts to the identity with splitters at the cell starts,
  constant, sorted and reversed inputs;
- invariants checked by code that shares nothing with the oracle (tests/invariants.py).
"""
from __future__ import annotations

import itertools
import os

import numpy as np
import pytest

import oracle
from paper_cs_0004013_amd import inputs
from tests import invariants as inv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
BOUNDARY = [0, 1, 255, 256, 65535, (1 << 31) - 1, 1 << 31, (1 << 32) - 1]


def _read_trace():
    rows = {}
    with open(os.path.join(GOLDEN, "lsd_trace.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, *vals = line.split()
            rows[name] = vals
    return rows


def _hex(vals):
    return np.array([int(v, 16) for v in vals], dtype=np.uint32)


def test_golden_lsd_trace():
    t = _read_trace()
    x = _hex(t["input"])
    p0 = oracle.bucket_pass(x, 0)
    assert p0.tolist() == _hex(t["pass0"]).tolist()
    p8 = oracle.bucket_pass(p0, 8)
    assert p8.tolist() == _hex(t["pass8"]).tolist()
    assert oracle.sort_u32(x).tolist() == _hex(t["sorted"]).tolist()
    h = oracle.digit_hist(x, 8, 8)
    want = {int(k, 16): int(c) for k, c in (kv.split(":") for kv in t["hist8"])}
    assert {i: int(c) for i, c in enumerate(h) if c} == want
    s = oracle.sort_u32(x)
    assert oracle.splitters(s, 4).tolist() == _hex(t["split4"]).tolist()
    assert oracle.splitters(s, 8).tolist() == _hex(t["split8"]).tolist()


def _read_slices():
    cases = []
    with open(os.path.join(GOLDEN, "slices.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            lhs, rhs = line.split(":")
            n, P = (int(v) for v in lhs.split())
            sizes = []
            for tok in rhs.split():
                if "*" in tok:
                    k, x = tok.split("*")
                    sizes += [int(x)] * int(k)
                else:
                    sizes.append(int(tok))
            cases.append((n, P, sizes))
    return cases


@pytest.mark.parametrize("n,P,sizes", _read_slices())
def test_golden_cell_sizes(n, P, sizes):
    st = oracle.slice_starts(n, P)
    assert np.diff(st.astype(np.int64)).tolist() == sizes
    inv.check_cell_sizes(n, P, st)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 7, 63, 64, 65, 255, 256, 257, 1000, 4097])
@pytest.mark.parametrize("P", [1, 2, 3, 63, 64, 65])
def test_cell_sizes_property(n, P):
    inv.check_cell_sizes(n, P, oracle.slice_starts(n, P))
    for PP in (n, n + 1):
        if PP >= 1:
            inv.check_cell_sizes(n, PP, oracle.slice_starts(n, PP))


def test_exhaustive_tiny_domain():
    """All sequences of length 0..5 over eight boundary values, against sorted()."""
    seqs = [s for L in range(6) for s in itertools.product(BOUNDARY, repeat=L)]
    lengths = np.array([len(s) for s in seqs], dtype=np.int64)
    off = np.zeros(len(seqs) + 1, dtype=np.uint64)
    np.cumsum(lengths, out=off[1:])
    flat = np.array([v for s in seqs for v in s], dtype=np.uint32)
    got = oracle.sort_segmented(flat, off)
    for i, s in enumerate(seqs):
        assert got[off[i]:off[i + 1]].tolist() == sorted(s), s


@pytest.mark.parametrize("n", list(range(0, 300, 7)) + [1 << 12, (1 << 16) + 3, 1 << 20])
def test_vs_numpy_sort(n):
    rng = np.random.default_rng(n)
    x = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    assert np.array_equal(oracle.sort_u32(x), np.sort(x))


@pytest.mark.parametrize("threads", [1, 2, 3, 8, 16])
@pytest.mark.parametrize("n", [0, 1, 5, 15, 300, 70_001, (1 << 20) + 3])
def test_mt_variant_vs_numpy_and_single_thread(n, threads):
    """The timing variant (passes split over threads) gives numpy's sort, and bit for bit the
    single-thread oracle's output, for thread counts above and below n."""
    rng = np.random.default_rng(n + 17 * threads)
    x = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    got = oracle.sort_u32_mt(x, threads)
    assert np.array_equal(got, np.sort(x))
    assert np.array_equal(got, oracle.sort_u32(x))


@pytest.mark.parametrize("dist", ["c", "e"])
def test_mt_variant_clustered(dist):
    ks = inputs.keyset(dist, 200_001, seed=5)
    assert np.array_equal(oracle.sort_u32_mt(ks.keys, 7), np.sort(ks.keys))


@pytest.mark.parametrize("dist", inputs.DISTS)
def test_distributions_vs_numpy_and_invariants(dist):
    ks = inputs.keyset(dist, 100_003, seed=7)
    s = oracle.sort_u32(ks.keys)
    assert np.array_equal(s, np.sort(ks.keys))
    assert inv.is_nondecreasing(s)
    assert inv.same_multiset(s, ks.keys)
    inv.check_splitters(s, 64, oracle.splitters(s, 64))


def test_adversarial_vs_numpy():
    ks = inputs.adversarial(1 << 18, seed=0)
    s = oracle.sort_u32(ks.keys)
    assert np.array_equal(s, np.sort(ks.keys))


@pytest.mark.parametrize("shift", [0, 8, 16, 24])
def test_bucket_pass_is_stable_digit_sort(shift):
    """One bucketing pass equals numpy's stable argsort on the digit (library special case)."""
    rng = np.random.default_rng(shift)
    x = rng.integers(0, 1 << 32, size=50_000, dtype=np.uint64).astype(np.uint32)
    x[::3] = x[0]  # many ties
    digit = (x >> np.uint32(shift)) & np.uint32(255)
    want = x[np.argsort(digit, kind="stable")]
    assert np.array_equal(oracle.bucket_pass(x, shift), want)


@pytest.mark.parametrize("shift,bits", [(0, 8), (8, 8), (16, 8), (24, 8), (0, 4), (28, 4), (0, 11),
                                        (11, 11), (22, 10), (0, 16)])
def test_digit_hist_vs_bincount(shift, bits):
    rng = np.random.default_rng(bits)
    x = rng.integers(0, 1 << 32, size=70_001, dtype=np.uint64).astype(np.uint32)
    h = oracle.digit_hist(x, shift, bits)
    want = np.bincount((x >> np.uint32(shift)) & np.uint32((1 << bits) - 1), minlength=1 << bits)
    assert np.array_equal(h, want.astype(np.uint64))
    assert int(h.sum()) == x.size


@pytest.mark.parametrize("n", [1, 5, 64, 1000, 65537])
def test_closed_forms(n):
    rng = np.random.default_rng(n)
    perm = rng.permutation(n).astype(np.uint32)
    s = oracle.sort_u32(perm)
    assert np.array_equal(s, np.arange(n, dtype=np.uint32))
    st = oracle.slice_starts(n, 64)
    assert oracle.splitters(s, 64).tolist() == [
        int(st[p]) if st[p] < st[p + 1] else 0xFFFFFFFF for p in range(1, 64)]
    v = np.full(n, 0x5A5A5A5A, dtype=np.uint32)
    assert np.array_equal(oracle.sort_u32(v), v)
    assert set(oracle.splitters(v, 4).tolist()) <= {0x5A5A5A5A, 0xFFFFFFFF}
    asc = np.sort(rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32))
    assert np.array_equal(oracle.sort_u32(asc), asc)
    assert np.array_equal(oracle.sort_u32(asc[::-1].copy()), asc)


def test_segmented_vs_per_segment_numpy():
    L = inputs.segment_lengths(64, seed=3, lo=0 + 1, hi=5000)
    L[::9] = 0
    keys, off, _ = inputs.segment_keys(L)
    got = oracle.sort_segmented(keys, off)
    for s in range(L.size):
        a, b = int(off[s]), int(off[s + 1])
        assert np.array_equal(got[a:b], np.sort(keys[a:b]))


def test_invalid_arguments():
    with pytest.raises(ValueError):
        oracle.slice_starts(10, 0)
    with pytest.raises(ValueError):
        oracle.sort_segmented(np.zeros(4, np.uint32), np.array([0, 3, 2], np.uint64))


# ---- (key, value) pairs: stability is observable ----------------------------------------------

def test_pairs_exhaustive_tiny_domain():
    """All key sequences of length 0..4 over six boundary values, values = input positions, against
    Python's sorted() on (key, position) pairs ordered by key (a stable sort)."""
    vals6 = BOUNDARY[:6]
    for L in range(5):
        for s in itertools.product(vals6, repeat=L):
            k = np.array(s, dtype=np.uint32)
            pos = np.arange(L, dtype=np.uint32)
            ok, ov = oracle.sort_pairs_u32(k, pos)
            want = sorted(zip(s, range(L)), key=lambda p: p[0])
            assert ok.tolist() == [p[0] for p in want] and ov.tolist() == [p[1] for p in want], s


@pytest.mark.parametrize("dist", inputs.DISTS)
def test_pairs_values_are_stable_argsort(dist):
    """With values = positions the output values are numpy's stable argsort (many equal keys in
    (c) and (e)); arbitrary values follow their keys."""
    ks = inputs.keyset(dist, 70_001, seed=13)
    pos = np.arange(ks.keys.size, dtype=np.uint32)
    ok, ov = oracle.sort_pairs_u32(ks.keys, pos)
    perm = np.argsort(ks.keys, kind="stable")
    assert np.array_equal(ov, perm.astype(np.uint32))
    assert np.array_equal(ok, ks.keys[perm])
    payload = (pos * np.uint32(2654435761)) ^ np.uint32(0x5BD1E995)
    ok2, ov2 = oracle.sort_pairs_u32(ks.keys, payload)
    assert np.array_equal(ok2, ok) and np.array_equal(ov2, payload[perm])


@pytest.mark.parametrize("shift", [0, 8, 16, 24])
def test_pairs_bucket_pass_is_stable_digit_sort(shift):
    rng = np.random.default_rng(shift + 5)
    k = rng.integers(0, 1 << 32, size=9_999, dtype=np.uint64).astype(np.uint32)
    v = rng.integers(0, 1 << 32, size=9_999, dtype=np.uint64).astype(np.uint32)
    ok, ov = oracle.bucket_pass_pairs(k, v, shift)
    perm = np.argsort((k >> np.uint32(shift)) & np.uint32(255), kind="stable")
    assert np.array_equal(ok, k[perm]) and np.array_equal(ov, v[perm])


def test_pairs_keys_match_key_sort():
    rng = np.random.default_rng(99)
    k = rng.integers(0, 1 << 32, size=123_457, dtype=np.uint64).astype(np.uint32)
    v = rng.integers(0, 1 << 32, size=k.size, dtype=np.uint64).astype(np.uint32)
    ok, _ = oracle.sort_pairs_u32(k, v)
    assert np.array_equal(ok, oracle.sort_u32(k))


# ---- merge of two sorted runs (merge-exchange, Sec. 3.4 / 4.6) ---------------------------------

def test_merge_exhaustive_tiny_domain():
    """Every pair of nondecreasing sequences of length 0..3 over six boundary values, against
    sorted() of the concatenation."""
    vals6 = sorted(BOUNDARY[:6])
    seqs = [list(s) for L in range(4) for s in itertools.combinations_with_replacement(vals6, L)]
    for a in seqs:
        for b in seqs:
            got = oracle.merge_u32(np.array(a, np.uint32), np.array(b, np.uint32))
            assert got.tolist() == sorted(a + b), (a, b)


@pytest.mark.parametrize("na,nb", [(0, 0), (0, 7), (9, 0), (1, 1), (1000, 3), (3, 1000), (70_001, 65_536),
                                   (1 << 18, (1 << 18) + 11)])
def test_merge_vs_numpy(na, nb):
    rng = np.random.default_rng(na * 31 + nb)
    a = np.sort(rng.integers(0, 1 << 32, size=na, dtype=np.uint64).astype(np.uint32))
    b = np.sort(rng.integers(0, 1 << 20, size=nb, dtype=np.uint64).astype(np.uint32) * np.uint32(4096))
    assert np.array_equal(oracle.merge_u32(a, b), np.sort(np.concatenate([a, b])))


def test_merge_closed_forms():
    a = np.arange(0, 200, 2, dtype=np.uint32)
    b = np.arange(1, 200, 2, dtype=np.uint32)
    assert np.array_equal(oracle.merge_u32(a, b), np.arange(200, dtype=np.uint32))   # interleave
    lo = np.arange(50, dtype=np.uint32)
    hi = np.arange(50, 90, dtype=np.uint32)
    assert np.array_equal(oracle.merge_u32(hi, lo), np.arange(90, dtype=np.uint32))  # b entirely first
    eq = np.full(33, 7, np.uint32)
    assert np.array_equal(oracle.merge_u32(eq, eq[:5]), np.full(38, 7, np.uint32))
