"""CPU oracle for the HashGraph hot path (arXiv:1907.02900).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import
this package.  The GPU library never does, and this package never imports the
GPU library: the two share no code.

The arithmetic lives in ``hg_oracle.c`` (plain sequential C, compiled with
gcc) and, for the multi-core CPU baseline, ``hg_oracle_omp.c`` (the same
definitions on all host cores, pinned against the sequential functions); this
module only marshals numpy arrays.  See the headers of those files for which
section, equation or algorithm of the paper each function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hg_oracle.c")
_SRC_OMP = os.path.join(_HERE, "hg_oracle_omp.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, ENOMEM, ECAPACITY = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile hg_oracle.c and hg_oracle_omp.c into liboracle.so (gcc -O2,
    OpenMP for the multi-core variant, no GPU code)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", "-o",
                               tmp, _SRC, _SRC_OMP])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    u64, u32, i32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p
    lib.orc_fmix32.argtypes, lib.orc_fmix32.restype = [u32], u32
    lib.orc_fmix64.argtypes, lib.orc_fmix64.restype = [u64], u64
    lib.orc_bucket_one.argtypes, lib.orc_bucket_one.restype = [u64, i32, u64, u64], u32
    lib.orc_hash.argtypes, lib.orc_hash.restype = [vp, u64, i32, u64, u64, vp], i32
    lib.orc_count.argtypes, lib.orc_count.restype = [vp, u64, u64, vp], i32
    lib.orc_exclusive_scan.argtypes, lib.orc_exclusive_scan.restype = [vp, u64, vp], i32
    lib.orc_place.argtypes, lib.orc_place.restype = [vp, vp, u64, i32, u64, vp, vp, vp], i32
    lib.orc_build.argtypes, lib.orc_build.restype = [vp, u64, i32, u64, u64, vp, vp, vp], i32
    lib.orc_probe_counts.argtypes = [vp, u64, vp, u64, i32, vp, ctypes.POINTER(u64)]
    lib.orc_probe_counts.restype = i32
    lib.orc_probe_pairs.argtypes = [vp, u64, vp, u64, i32, vp, vp, u64, ctypes.POINTER(u64)]
    lib.orc_probe_pairs.restype = i32
    lib.orc_count_one.argtypes, lib.orc_count_one.restype = [vp, u64, i32, u64], u64
    lib.orc_omp_threads.argtypes, lib.orc_omp_threads.restype = [], i32
    lib.orc_build_omp.argtypes, lib.orc_build_omp.restype = [vp, u64, i32, u64, u64, vp, vp,
                                                             vp], i32
    lib.orc_probe_counts_omp.argtypes = [vp, u64, vp, u64, i32, vp, ctypes.POINTER(u64)]
    lib.orc_probe_counts_omp.restype = i32
    _lib = lib
    return lib


def _keys(a, key_bits=None):
    a = np.ascontiguousarray(a)
    if key_bits is None:
        key_bits = 64 if a.dtype.itemsize == 8 else 32
    dt = np.uint64 if key_bits == 64 else np.uint32
    if a.dtype != dt:
        a = a.astype(dt)
    return np.ascontiguousarray(a), key_bits


def _p(a):
    return a.ctypes.data if a.size else None


def fmix32(x: int) -> int:
    return int(_load().orc_fmix32(int(x) & 0xFFFFFFFF))


def fmix64(x: int) -> int:
    return int(_load().orc_fmix64(int(x) & 0xFFFFFFFFFFFFFFFF))


def bucket_one(key: int, V: int, seed: int = 0, key_bits: int = 32) -> int:
    return int(_load().orc_bucket_one(int(key), key_bits, int(V), int(seed) & 0xFFFFFFFFFFFFFFFF))


def hash_buckets(keys, V: int, seed: int = 0, key_bits=None) -> np.ndarray:
    """Eq. 1 for every key: fmix(key ^ seed) mod V."""
    k, kb = _keys(keys, key_bits)
    h = np.empty(k.size, dtype=np.uint32)
    rc = _load().orc_hash(_p(k), k.size, kb, int(V), int(seed) & 0xFFFFFFFFFFFFFFFF, _p(h))
    if rc:
        raise ValueError("orc_hash rc=%d" % rc)
    return h


def count(h, V: int) -> np.ndarray:
    h = np.ascontiguousarray(h, dtype=np.uint32)
    c = np.empty(int(V), dtype=np.uint32)
    rc = _load().orc_count(_p(h), h.size, int(V), _p(c))
    if rc:
        raise ValueError("orc_count rc=%d" % rc)
    return c


def exclusive_scan(counts) -> np.ndarray:
    c = np.ascontiguousarray(counts, dtype=np.uint32)
    o = np.empty(c.size + 1, dtype=np.uint32)
    rc = _load().orc_exclusive_scan(_p(c), c.size, _p(o))
    if rc:
        raise ValueError("orc_exclusive_scan rc=%d" % rc)
    return o


def build_table(keys, V: int, seed: int = 0, key_bits=None):
    """The stable HashGraph table: (offsets[V+1], ids[n], bucketed keys[n])."""
    k, kb = _keys(keys, key_bits)
    off = np.empty(int(V) + 1, dtype=np.uint32)
    ids = np.empty(k.size, dtype=np.uint32)
    ek = np.empty(k.size, dtype=k.dtype)
    rc = _load().orc_build(_p(k), k.size, kb, int(V), int(seed) & 0xFFFFFFFFFFFFFFFF,
                           _p(off), _p(ids), _p(ek))
    if rc:
        raise ValueError("orc_build rc=%d" % rc)
    return off, ids, ek


def probe_counts(keys, queries, key_bits=None):
    """count[j] = #{i : keys[i] == queries[j]} (no hash), and the uint64 total."""
    k, kb = _keys(keys, key_bits)
    q, _ = _keys(queries, kb)
    c = np.empty(q.size, dtype=np.uint32)
    tot = ctypes.c_uint64(0)
    rc = _load().orc_probe_counts(_p(k), k.size, _p(q), q.size, kb, _p(c), ctypes.byref(tot))
    if rc:
        raise ValueError("orc_probe_counts rc=%d" % rc)
    return c, int(tot.value)


def probe_pairs(keys, queries, key_bits=None, capacity=None):
    """Matching (build_id, probe_id) pairs, probe id ascending then build id."""
    k, kb = _keys(keys, key_bits)
    q, _ = _keys(queries, kb)
    lib = _load()
    if capacity is None:
        _, total = probe_counts(k, q, kb)
        capacity = total
    b = np.empty(int(capacity), dtype=np.uint32)
    p = np.empty(int(capacity), dtype=np.uint32)
    tot = ctypes.c_uint64(0)
    rc = lib.orc_probe_pairs(_p(k), k.size, _p(q), q.size, kb, _p(b), _p(p), int(capacity),
                             ctypes.byref(tot))
    if rc == ECAPACITY:
        return None, None, int(tot.value)
    if rc:
        raise ValueError("orc_probe_pairs rc=%d" % rc)
    return b, p, int(tot.value)


def omp_threads() -> int:
    """Threads the multi-core variant uses (OpenMP's current maximum)."""
    return int(_load().orc_omp_threads())


def build_table_omp(keys, V: int, seed: int = 0, key_bits=None):
    """build_table on all host cores (same output, bit for bit)."""
    k, kb = _keys(keys, key_bits)
    off = np.empty(int(V) + 1, dtype=np.uint32)
    ids = np.empty(k.size, dtype=np.uint32)
    ek = np.empty(k.size, dtype=k.dtype)
    rc = _load().orc_build_omp(_p(k), k.size, kb, int(V), int(seed) & 0xFFFFFFFFFFFFFFFF,
                               _p(off), _p(ids), _p(ek))
    if rc:
        raise ValueError("orc_build_omp rc=%d" % rc)
    return off, ids, ek


def probe_counts_omp(keys, queries, key_bits=None):
    """probe_counts on all host cores (same output, bit for bit)."""
    k, kb = _keys(keys, key_bits)
    q, _ = _keys(queries, kb)
    c = np.empty(q.size, dtype=np.uint32)
    tot = ctypes.c_uint64(0)
    rc = _load().orc_probe_counts_omp(_p(k), k.size, _p(q), q.size, kb, _p(c),
                                      ctypes.byref(tot))
    if rc:
        raise ValueError("orc_probe_counts_omp rc=%d" % rc)
    return c, int(tot.value)


def count_one(keys, q: int, key_bits=None) -> int:
    """Brute-force count of one query over all keys."""
    k, kb = _keys(keys, key_bits)
    return int(_load().orc_count_one(_p(k), k.size, kb, int(q) & 0xFFFFFFFFFFFFFFFF))


# ---- collections of sets (build once, intersect many; Sec. 3.4) -------------


def set_hash_range(n: int, shift: int = 0) -> int:
    """Hash range of one set of a collection: the smallest power of two that
    is >= max(n, 1), times 2**shift, clamped to [1, 2**31].  (A layout rule of
    the collections, which the paper leaves open: powers of two let every
    set's bucket be the low bits of the same hash.)"""
    p = 1
    while p < max(int(n), 1):
        p *= 2
    e = p.bit_length() - 1 + int(shift)
    return 1 << min(max(e, 0), 31)


def collection_table(keys, set_off, seed: int = 0, shift: int = 0, key_bits=None):
    """Every set's stable table (build_table of its keys with range
    set_hash_range(n_s, shift)), concatenated: returns (bucket_base[S+1],
    offsets[sum V + 1], ids[n], keys[n]) where set s owns buckets
    [bucket_base[s], bucket_base[s+1]), offsets are absolute positions and
    ids are positions in the concatenated input."""
    k, kb = _keys(keys, key_bits)
    so = np.asarray(set_off, dtype=np.int64)
    S = so.size - 1
    ranges = [set_hash_range(so[s + 1] - so[s], shift) for s in range(S)]
    bb = np.zeros(S + 1, dtype=np.uint64)
    bb[1:] = np.cumsum(np.asarray(ranges, dtype=np.uint64))
    off = np.empty(int(bb[-1]) + 1, dtype=np.uint32)
    ids = np.empty(k.size, dtype=np.uint32)
    ek = np.empty(k.size, dtype=k.dtype)
    for s in range(S):
        lo, hi = int(so[s]), int(so[s + 1])
        o, i, e = build_table(k[lo:hi], ranges[s], seed, kb)
        off[int(bb[s]):int(bb[s + 1])] = o[:-1] + lo
        ids[lo:hi] = i + lo
        ek[lo:hi] = e
    off[-1] = k.size
    return bb, off, ids, ek


def pair_match_counts(keys_a, off_a, keys_b, off_b, pairs, key_bits=None):
    """For each pair (i, j): the number of (x, y) with x an entry of set i of
    a, y an entry of set j of b and equal keys (the join size of the two
    sets), as the total of Probe-Standard counts of set j's keys against set
    i's keys."""
    ka, kb = _keys(keys_a, key_bits)
    kbk, _ = _keys(keys_b, kb)
    oa = np.asarray(off_a, dtype=np.int64)
    ob = np.asarray(off_b, dtype=np.int64)
    pr = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    out = np.zeros(pr.shape[0], dtype=np.uint64)
    for q, (i, j) in enumerate(pr):
        a = ka[oa[i]:oa[i + 1]]
        b = kbk[ob[j]:ob[j + 1]]
        if a.size and b.size:
            out[q] = probe_counts(a, b, kb)[1]
    return out
