"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds only random-number generation: no hashing, counting,
placement or probing.  The GPU tests, the benchmark and the oracle tests all
draw their inputs from here, so both sides of every parity check see the same
arrays.  All generators use numpy's PCG64 with an explicit seed.

Shapes (see Sec. 4 "Input sizes & Key Distribution" and Sec. 5):
  * uniform keys over the full key width (the default random input),
  * the sequence 1..N the paper uses for its framework comparisons,
  * uniform keys over a reduced range N/R, giving R appearances per key on
    average (the duplicate-key experiments of Sec. 5.1),
  * bounded Zipf keys (heavy skew, many keys per bucket),
  * probe sets with a given fraction drawn from the build keys,
  * size mixes for batched tables and a Poisson request stream for serving,
  * collections of sets with power-law sizes (rows of a sparse matrix) and
    random set pairs, for build-once / intersect-many (Sec. 3.4).
"""
from __future__ import annotations

import numpy as np

U32_MAX = 0xFFFFFFFF


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def _dtype(key_bits: int):
    if key_bits == 32:
        return np.uint32
    if key_bits == 64:
        return np.uint64
    raise ValueError("key_bits must be 32 or 64")


def uniform_keys(n: int, key_bits: int = 32, seed: int = 0) -> np.ndarray:
    """n keys uniform over [0, 2^key_bits)."""
    rng = _rng(seed)
    dt = _dtype(key_bits)
    return rng.integers(0, np.iinfo(dt).max, size=int(n), dtype=dt, endpoint=True)


def sequence_keys(n: int, key_bits: int = 32) -> np.ndarray:
    """The sequence 1, 2, ..., n."""
    return np.arange(1, int(n) + 1, dtype=_dtype(key_bits))


def duplicate_keys(n: int, appearances: float, key_bits: int = 32, seed: int = 0) -> np.ndarray:
    """n keys uniform over [1, n / appearances]: each value appears
    `appearances` times on average (values below 1 widen the range)."""
    rng = _rng(seed)
    hi = max(1, int(round(n / float(appearances))))
    return rng.integers(1, hi, size=int(n), dtype=_dtype(key_bits), endpoint=True)


def _inverse_cdf(cdf: np.ndarray, u: np.ndarray) -> np.ndarray:
    """For each u in [0, 1), the first index r with cdf[r] > u (what
    np.searchsorted(cdf, u, side="right") returns; cdf ends at 1).  A guide
    table over equal-width cells of [0, 1) (indexed search) brackets each
    answer, and a vectorised bisection inside the bracket finishes it, so that
    2^28 draws take seconds instead of a full binary search each."""
    cells = min(1 << 24, max(1, cdf.size))
    edges = np.arange(cells + 1, dtype=np.float64) / cells
    guide = np.searchsorted(cdf, edges, side="right")
    np.minimum(guide, cdf.size - 1, out=guide)
    j = np.minimum((u * cells).astype(np.int64), cells - 1)
    lo = guide[j]              # cdf[lo - 1] <= j / cells <= u
    hi = guide[j + 1]          # cdf[hi] > u, or hi is the last index
    idx = np.nonzero(lo < hi)[0]
    while idx.size:
        a, b = lo[idx], hi[idx]
        mid = (a + b) >> 1
        right = cdf[mid] <= u[idx]
        lo[idx] = np.where(right, mid + 1, a)
        hi[idx] = np.where(right, b, mid)
        idx = idx[lo[idx] < hi[idx]]
    return lo


def zipf_keys(n: int, s: float, distinct: int = 1 << 24, seed: int = 0,
              map_seed: int | None = None) -> np.ndarray:
    """n uint32 keys with a bounded Zipf law over `distinct` ranks,
    p(r) proportional to r^-s, sampled by inverse CDF.  Rank r maps to a key by
    a seeded odd-multiplier bijection on uint32 so that frequent keys are not
    small integers.  The bijection comes from `map_seed` when given (so that a
    build side and a probe side drawn with different seeds share one law over
    the same keys), else from `seed`."""
    rng = _rng(seed)
    r = np.arange(1, int(distinct) + 1, dtype=np.float64)
    cdf = np.cumsum(r ** (-float(s)))
    cdf /= cdf[-1]
    u = rng.random(int(n))
    rank = _inverse_cdf(cdf, u).astype(np.uint64)
    rank = np.minimum(rank, distinct - 1)
    mrng = rng if map_seed is None else _rng(map_seed)
    mult = (int(mrng.integers(1, 1 << 31)) << 1) | 1
    add = int(mrng.integers(0, 1 << 32))
    return ((rank * np.uint64(mult) + np.uint64(add)) & np.uint64(U32_MAX)).astype(np.uint32)


def probe_queries(keys: np.ndarray, m: int, hit_fraction: float = 0.5, seed: int = 1,
                  key_bits: int | None = None) -> np.ndarray:
    """m queries: each position independently takes, with probability
    `hit_fraction`, a key drawn uniformly (with replacement) from `keys`, and
    otherwise a uniform random value over the key width.  The random half may
    also hit by chance."""
    keys = np.asarray(keys)
    if key_bits is None:
        key_bits = 64 if keys.dtype.itemsize == 8 else 32
    dt = _dtype(key_bits)
    rng = _rng(seed)
    m = int(m)
    rand = rng.integers(0, np.iinfo(dt).max, size=m, dtype=dt, endpoint=True)
    if keys.size == 0 or m == 0:
        return rand
    pick = rng.integers(0, keys.size, size=m, dtype=np.int64)
    hit = rng.random(m) < float(hit_fraction)
    return np.where(hit, keys[pick].astype(dt), rand)


def batched_sizes(tables: int = 4096, lo_log2: float = 8.0, hi_log2: float = 20.0,
                  seed: int = 7) -> np.ndarray:
    """Table sizes floor(2^U), U uniform in [lo_log2, hi_log2]."""
    rng = _rng(seed)
    u = rng.uniform(lo_log2, hi_log2, size=int(tables))
    return np.floor(np.exp2(u)).astype(np.int64)


def log_uniform_sizes(count: int, lo_log2: float, hi_log2: float, rng) -> np.ndarray:
    u = rng.uniform(lo_log2, hi_log2, size=int(count))
    return np.floor(np.exp2(u)).astype(np.int64)


def serving_stream(requests: int, rate_per_s: float, build_fraction: float = 0.3,
                   build_log2=(10.0, 24.0), probe_log2=(10.0, 22.0), seed: int = 11):
    """A Poisson request stream: exponential inter-arrival times at
    `rate_per_s`; each request is a build (probability `build_fraction`) with a
    log-uniform key count, or a probe with a log-uniform query count.
    Returns (arrival_seconds[float64], is_build[bool], size[int64],
    data_seed[int64])."""
    rng = _rng(seed)
    r = int(requests)
    gaps = rng.exponential(1.0 / float(rate_per_s), size=r)
    arrival = np.cumsum(gaps)
    is_build = rng.random(r) < float(build_fraction)
    bsz = log_uniform_sizes(r, build_log2[0], build_log2[1], rng)
    psz = log_uniform_sizes(r, probe_log2[0], probe_log2[1], rng)
    size = np.where(is_build, bsz, psz)
    data_seed = rng.integers(0, 1 << 40, size=r, dtype=np.int64)
    return arrival, is_build, size, data_seed


def collection_sets(sets: int, mean_size: float, key_range: int, key_bits: int = 32,
                    seed: int = 0, tail: float = 1.5, max_size: int = 1 << 16):
    """`sets` key sets shaped like the rows of a sparse matrix: sizes from a
    Pareto (Lomax) law with tail exponent `tail`, mean about `mean_size`,
    clipped to [1, max_size]; keys (column indices) uniform in [0, key_range),
    drawn independently, so a set may repeat a key (rarely, for sets much
    smaller than key_range).  Returns (keys, offsets int64[sets + 1])."""
    r = _rng(seed)
    scale = max(mean_size - 1.0, 0.0) * (tail - 1.0)
    sizes = np.minimum(1 + np.floor(r.pareto(tail, sets) * scale), max_size).astype(np.int64)
    off = np.zeros(sets + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    keys = r.integers(0, key_range, int(off[-1]), dtype=np.uint64)
    return keys.astype(_dtype(key_bits)), off


def set_pairs(count: int, sets_a: int, sets_b: int, seed: int = 0) -> np.ndarray:
    """`count` uniformly random (i, j) pairs, i < sets_a, j < sets_b, as
    uint32[count, 2]."""
    r = _rng(seed)
    p = np.empty((count, 2), dtype=np.uint32)
    p[:, 0] = r.integers(0, max(sets_a, 1), count)
    p[:, 1] = r.integers(0, max(sets_b, 1), count)
    return p
