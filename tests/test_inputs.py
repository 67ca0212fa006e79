"""Seeded generators: determinism, sizes and the shape each distribution is meant to have (CPU)."""
from __future__ import annotations

import numpy as np
import pytest

from paper_cs_0004013_amd import inputs


@pytest.mark.parametrize("dist", inputs.DISTS)
def test_deterministic_and_in_range(dist):
    a = inputs.keyset(dist, 10_000, seed=3)
    b = inputs.keyset(dist, 10_000, seed=3)
    c = inputs.keyset(dist, 10_000, seed=4)
    assert a.keys.dtype == np.uint32 and a.keys.size == 10_000
    assert np.array_equal(a.keys, b.keys)
    assert not np.array_equal(a.keys, c.keys)
    assert int(a.keys.max()) <= inputs.KEY_MAX
    assert int(a.cell_sizes.sum()) == 10_000 and a.cell_sizes.size == 64


def test_distribution_shapes():
    n = 200_000
    assert np.unique(inputs.keyset("c", n, 1).keys).size == 1
    e = inputs.keyset("e", n, 2).keys
    assert np.unique(e).size <= 16 * 256
    b = inputs.keyset("b", n, 3)
    ratio = b.cell_sizes.max() / b.cell_sizes.min()
    assert 300 < ratio < 500          # 1.1^63 ~ 405
    d = inputs.keyset("d", n, 4).keys
    # 70% of the keys sit within a few sigma of 32 centres: far fewer distinct top-12-bit values
    # are populated densely than for uniform keys
    top = np.bincount(d >> np.uint32(19), minlength=4096)
    dense = int((top > 4 * n / 4096).sum())
    assert 32 <= dense < 500          # uniform keys would give none


def test_adversarial_shape():
    ks = inputs.adversarial(1 << 20, seed=0)
    tops = np.unique(ks.keys >> np.uint32(16))
    assert tops.size <= 4 and int(tops.max()) < (1 << 15)
    vals, counts = np.unique(ks.keys, return_counts=True)
    assert counts.max() >= 900        # hot keys written ~1000 times
    assert int(ks.cell_sizes.sum()) == ks.keys.size


def test_segments():
    L = inputs.segment_lengths(4096, seed=0)
    assert L.min() >= 64 and L.max() <= 1 << 18
    assert 1.1e8 < L.sum() < 1.5e8    # ~1.29e8 keys in total
    keys, off, dists = inputs.segment_keys(L[:50])
    assert off[0] == 0 and off[-1] == keys.size and np.all(np.diff(off.astype(np.int64)) == L[:50])
    assert set(dists) <= set(inputs.DISTS)


def test_request_trace():
    tr = inputs.request_trace(1000, rate_per_s=1000.0)
    assert len(tr) == 1000
    ts = np.array([r.arrival_s for r in tr])
    assert np.all(np.diff(ts) >= 0)
    assert all((1 << 10) <= r.n <= (1 << 24) for r in tr)
    assert all(0 <= r.pool_offset <= (1 << 26) - r.n for r in tr)
    assert abs(ts[-1] - 1.0) < 0.2
