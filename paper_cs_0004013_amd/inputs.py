"""Seeded synthetic key generators shared by the tests, the smoke check and the benchmark.

This module only draws random numbers; it holds none of the sort's arithmetic (no digit, bucket,
rank or slice computation), so that both the HIP path and the CPU oracle can be fed from it.

The paper's contest data came from an object file of the contest organisers that is not available;
its five "keys" are described only qualitatively (Sec. 1.1 table: random / random with bad balance /
uniform / some clustering / clustered).  The generators below are synthetic stand-ins with that
intent.  Every draw uses numpy's PCG64 with an explicit seed; "uniform" means i.i.d. integers in
[0, 2^31 - 1] (positive 32-bit integers).

  dist 'a'  random values, good balance                      (key 1)
  dist 'b'  random values, input cells sized 1.1^i           (key 2)
  dist 'c'  every key equal to one random value              (key 3)
  dist 'd'  70% from 32 Gaussians (sigma 2^20), 30% uniform  (key 4)
  dist 'e'  16 bands of width 2^8 at random centres          (key 5)
  adversarial(): top 16 bits take 4 values, low 16 uniform, 5% of the keys are 1000-fold copies.
  segment_lengths() / segment_keys(): 4096 log-uniform segments in [64, 2^18], one dist each.
  request_trace(): Poisson arrivals of log-uniform request sizes in [2^10, 2^24].
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

KEY_MAX = (1 << 31) - 1          # largest positive 32-bit integer
DISTS = ("a", "b", "c", "d", "e")
CELLS = 64


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _largest_remainder(weights: np.ndarray, total: int) -> np.ndarray:
    """Integer sizes proportional to ``weights`` that sum exactly to ``total``."""
    w = np.asarray(weights, dtype=np.float64)
    exact = w / w.sum() * total
    base = np.floor(exact).astype(np.int64)
    short = int(total - base.sum())
    if short > 0:
        order = np.argsort(-(exact - base), kind="stable")
        base[order[:short]] += 1
    return base


def _uniform(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.integers(0, KEY_MAX, size=n, dtype=np.uint32, endpoint=True)


def dist_keys(dist: str, n: int, rng: np.random.Generator) -> np.ndarray:
    """n keys of distribution ``dist`` (values only; cell sizes are separate metadata)."""
    if dist in ("a", "b"):
        return _uniform(rng, n)
    if dist == "c":
        v = rng.integers(0, KEY_MAX, dtype=np.uint32, endpoint=True)
        return np.full(n, v, dtype=np.uint32)
    if dist == "d":
        centres = rng.integers(0, KEY_MAX, size=32, dtype=np.int64, endpoint=True)
        from_mix = rng.random(n) < 0.7
        comp = rng.integers(0, 32, size=n)
        g = np.rint(centres[comp] + rng.standard_normal(n) * float(1 << 20))
        g = np.clip(g, 0, KEY_MAX).astype(np.uint32)
        u = _uniform(rng, n)
        return np.where(from_mix, g, u).astype(np.uint32)
    if dist == "e":
        centres = rng.integers(128, KEY_MAX - 128, size=16, dtype=np.int64, endpoint=True)
        j = rng.integers(0, 16, size=n)
        off = rng.integers(-128, 128, size=n, dtype=np.int64)
        return (centres[j] + off).astype(np.uint32)
    raise ValueError(f"unknown distribution {dist!r}")


@dataclass
class KeySet:
    keys: np.ndarray          # uint32[n], the input array in HBM order
    cell_sizes: np.ndarray    # int64[64], how the input is split into initial cells (sums to n)
    name: str


def keyset(dist: str, n: int, seed: int) -> KeySet:
    """One of the five contest-like key sets, n keys, as 64 input cells."""
    rng = rng_for(seed)
    keys = dist_keys(dist, n, rng)
    if dist == "b":
        sizes = _largest_remainder(1.1 ** np.arange(CELLS), n)
    else:
        sizes = _largest_remainder(np.ones(CELLS), n)
    return KeySet(keys, sizes, f"{dist}:n={n}:seed={seed}")


def adversarial(n: int, seed: int) -> KeySet:
    """Top 16 bits from 4 values in [0, 2^15), low 16 bits uniform; m = round(0.05 n / 1000) hot
    keys (same law) each written 1000 times at uniformly drawn positions (with replacement);
    64 input cells with Dirichlet(0.3) sizes."""
    rng = rng_for(seed)
    tops = rng.choice(1 << 15, size=4, replace=False).astype(np.uint32)
    keys = (tops[rng.integers(0, 4, size=n)] << np.uint32(16)) | \
        rng.integers(0, 1 << 16, size=n, dtype=np.uint32)
    m = int(round(0.05 * n / 1000))
    if m:
        hot = (tops[rng.integers(0, 4, size=m)] << np.uint32(16)) | \
            rng.integers(0, 1 << 16, size=m, dtype=np.uint32)
        pos = rng.integers(0, n, size=m * 1000)
        keys[pos] = np.repeat(hot, 1000)
    sizes = _largest_remainder(rng.dirichlet(np.full(CELLS, 0.3)), n)
    return KeySet(keys.astype(np.uint32), sizes, f"adversarial:n={n}:seed={seed}")


def segment_lengths(nseg: int = 4096, seed: int = 0, lo: int = 64, hi: int = 1 << 18) -> np.ndarray:
    """Log-uniform segment lengths floor(exp(U[ln lo, ln hi])) clipped to [lo, hi]."""
    rng = rng_for(seed)
    L = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=nseg))).astype(np.int64)
    return np.clip(L, lo, hi)


def segment_keys(lengths: np.ndarray) -> tuple[np.ndarray, np.ndarray, list[str]]:
    """Concatenated keys of all segments and CSR offsets (uint32).  Segment s draws its
    distribution and keys from seed s."""
    lengths = np.asarray(lengths, dtype=np.int64)
    offsets = np.zeros(lengths.size + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    keys = np.empty(int(offsets[-1]), dtype=np.uint32)
    dists = []
    for s, L in enumerate(lengths):
        rng = rng_for(s)
        d = DISTS[int(rng.integers(0, 5))]
        keys[offsets[s]:offsets[s + 1]] = dist_keys(d, int(L), rng)
        dists.append(d)
    return keys, offsets.astype(np.uint32), dists


@dataclass
class Request:
    rid: int
    n: int
    dist: str
    pool_offset: int
    arrival_s: float


def request_trace(nreq: int, rate_per_s: float, pool_keys: int = 1 << 26, seed: int = 0,
                  lo: int = 1 << 10, hi: int = 1 << 24) -> list[Request]:
    """Poisson arrivals at ``rate_per_s``; request r draws its size (log-uniform [lo, hi]), its
    distribution and its window into the distribution's key pool from seed r."""
    arr = rng_for(seed + 1_000_003)
    gaps = arr.exponential(1.0 / rate_per_s, size=nreq)
    t = np.cumsum(gaps)
    out = []
    for r in range(nreq):
        g = rng_for(r)
        n = int(np.clip(np.floor(np.exp(g.uniform(math.log(lo), math.log(hi)))), lo, hi))
        d = DISTS[int(g.integers(0, 5))]
        off = int(g.integers(0, pool_keys - n + 1))
        out.append(Request(r, n, d, off, float(t[r])))
    return out
