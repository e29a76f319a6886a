"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Everything on this path is integer work, so every comparison is bit-exact:
buckets, counts, offsets, pair totals and pairs.  V2 places stably, so its
table equals the oracle's stable table entry by entry; V1 places by atomics,
so its buckets are compared as sorted id lists (multisets) and its offsets
exactly.  Sizes span many partition tiles (4096 entries) plus ragged tails,
both one- and two-pass partition plans, heavy bins (more keys than a bin holds
in LDS) and the degenerate ranges V = 1 and V > n.
"""
import numpy as np
import pytest

import oracle
from paper_1907_02900_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1907_02900_amd import hg as _hg
    _hg.lib()
    return _hg


def say(*a):
    print("[case]", *a, flush=True)


def dt(kb):
    return np.uint64 if kb == 64 else np.uint32


def keys_for(kind, n, kb, seed):
    if kind == "uniform":
        return workloads.uniform_keys(n, kb, seed)
    if kind == "dup8":
        return workloads.duplicate_keys(n, 8.0, kb, seed)
    if kind == "zipf":
        return workloads.zipf_keys(n, 1.2, distinct=1 << 14, seed=seed).astype(dt(kb))
    if kind == "equal":
        return np.full(n, 12345, dtype=dt(kb))
    raise ValueError(kind)


def table_np(hg, t, kb):
    off, ids, ek = t.export()
    torch.cuda.synchronize()
    return hg.to_numpy(off, np.uint32), hg.to_numpy(ids, np.uint32), hg.to_numpy(ek, dt(kb))


# ------------------------------------------------------------- single steps


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("n,V,seed", [(0, 5, 0), (1, 1, 3), (4097, 7, 1), (100003, 1000003, 9),
                                      (65536, (1 << 32) - 1, 2**40 + 77), (50000, 1 << 20, 5)])
def test_hash_matches_oracle(hg, kb, n, V, seed):
    say("hash", kb, n, V, seed)
    k = workloads.uniform_keys(n, kb, seed=n + 1)
    d = hg.hg_hash(hg.to_device(k), V, seed)
    got = hg.to_numpy(d, np.uint32)
    assert np.array_equal(got, oracle.hash_buckets(k, V, seed, kb))


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("n,V", [(0, 9), (10000, 1), (300001, 4099), (1 << 20, 1 << 20),
                                 (65, 3), (200003, (1 << 25) + 1)])
def test_histogram_matches_oracle(hg, kb, n, V):
    say("histogram", kb, n, V)
    k = workloads.duplicate_keys(n, 3.0, kb, seed=7) if n else np.zeros(0, dt(kb))
    got = hg.to_numpy(hg.hg_histogram(hg.to_device(k), V, 11), np.uint32)
    assert np.array_equal(got, oracle.count(oracle.hash_buckets(k, V, 11, kb), V))


@pytest.mark.parametrize("V", [0, 1, 15, 4095, 4096, 4097, 65536 * 3 + 5, (1 << 22) + 3])
def test_exclusive_scan_matches_oracle(hg, V):
    say("scan", V)
    rng = np.random.default_rng(V)
    c = rng.integers(0, 7, size=V, dtype=np.uint32)
    got = hg.to_numpy(hg.hg_exclusive_scan(hg.to_device(c)), np.uint32)
    assert np.array_equal(got, oracle.exclusive_scan(c))


def test_exclusive_scan_wraps_modulo_2_32(hg):
    c = np.full(10000, 1 << 20, dtype=np.uint32)  # sum 10000 * 2^20 > 2^32
    got = hg.to_numpy(hg.hg_exclusive_scan(hg.to_device(c)), np.uint32)
    exp = (np.arange(10001, dtype=np.uint64) * (1 << 20)) & 0xFFFFFFFF
    assert np.array_equal(got, exp.astype(np.uint32))


# ------------------------------------------------------------------ builds

BUILD_CASES = [
    # kind, n, V  -- one-pass, two-pass, heavy bins, V = 1, V >> n, ragged tails
    ("uniform", 0, 17),
    ("uniform", 1, 1),
    ("uniform", 5, 10),
    ("uniform", 4096, 4096),
    ("uniform", 4097, 1000),
    ("uniform", 100003, 100003),
    ("uniform", (1 << 20), 1 << 20),
    ("uniform", (1 << 21) + 17, (1 << 21) + 17),
    ("uniform", (1 << 21) + 5, 1 << 19),
    ("uniform", 300000, 1 << 30),
    ("uniform", 200000, 1),
    ("uniform", 200000, 3),
    # bins above 2^17 keys are split over several workgroups
    ("equal", 600000, 1000),
    ("uniform", (1 << 19) + 3, 2),
    ("zipf", 1 << 20, 1 << 20),
    ("dup8", 500000, 250000),
    ("zipf", 400000, 400000),
    ("equal", 70000, 4096),
]


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("kind,n,V", BUILD_CASES)
def test_build_v2_equals_stable_oracle(hg, kb, kind, n, V):
    say("build-v2", kb, kind, n, V)
    k = keys_for(kind, n, kb, seed=n % 97)
    t = hg.hg_build(hg.to_device(k), V, seed=12345, variant=hg.VARIANT_V2)
    off, ids, ek = table_np(hg, t, kb)
    o_off, o_ids, o_ek = oracle.build_table(k, V, 12345, kb)
    assert np.array_equal(off, o_off)
    assert np.array_equal(ids, o_ids)
    assert np.array_equal(ek, o_ek)
    t.free()


@pytest.mark.parametrize("bins", [1, 2, 64, 1000, 4096])
def test_build_v2_bin_counts(hg, bins):
    """Alg. 2 with an explicit bin count, including the degenerate Bins = 1."""
    n, V = 150001, 60000
    say("build-v2-bins", bins)
    k = workloads.uniform_keys(n, 32, seed=4)
    t = hg.hg_build(hg.to_device(k), V, seed=3, variant=hg.VARIANT_V2, bins=bins)
    off, ids, ek = table_np(hg, t, 32)
    o_off, o_ids, o_ek = oracle.build_table(k, V, 3)
    assert np.array_equal(off, o_off) and np.array_equal(ids, o_ids) and np.array_equal(ek, o_ek)


def check_v1(off, ids, ek, k, V, seed, kb):
    o_off, o_ids, _ = oracle.build_table(k, V, seed, kb)
    assert np.array_equal(off, o_off)
    # bucket contents as multisets: sort ids inside each bucket
    seg = np.searchsorted(off.astype(np.int64), np.arange(ids.size), side="right") - 1
    order = np.lexsort((ids, seg))
    assert np.array_equal(ids[order], o_ids)
    assert np.array_equal(ek, k[ids])


@pytest.mark.parametrize("plain", [False, True])
@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("kind,n,V", [("uniform", 0, 3), ("uniform", 1000, 1),
                                      ("uniform", 100003, 100003), ("dup8", 400000, 1 << 16),
                                      ("zipf", 300000, 300000), ("uniform", (1 << 20) + 3, 1 << 20),
                                      ("equal", 200001, 97), ("zipf", 250007, (1 << 26) + 3),
                                      ("dup8", 123457, (1 << 25) - 1)])
def test_build_v1_matches_oracle_as_multisets(hg, kb, kind, n, V, plain):
    # plain: one atomic per key; otherwise same-bucket lanes of a wave share one
    say("build-v1", kb, kind, n, V, plain)
    k = keys_for(kind, n, kb, seed=5)
    t = hg.hg_build(hg.to_device(k), V, seed=99, variant=hg.VARIANT_V1, v1_plain=plain)
    off, ids, ek = table_np(hg, t, kb)
    check_v1(off, ids, ek, k, V, 99, kb)


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("kind,n,V", BUILD_CASES)
def test_build_v2_any_order_matches_oracle_as_multisets(hg, kb, kind, n, V):
    # any_order: offsets exact, buckets as multisets, probes exact
    say("build-v2-any", kb, kind, n, V)
    k = keys_for(kind, n, kb, seed=n % 89)
    t = hg.hg_build(hg.to_device(k), V, seed=777, any_order=True)
    off, ids, ek = table_np(hg, t, kb)
    check_v1(off, ids, ek, k, V, 777, kb)
    q = workloads.probe_queries(k if n else workloads.uniform_keys(8, kb, 0), 50000, 0.5,
                                seed=3, key_bits=kb)
    c, tot = hg.hg_probe(t, hg.to_device(q), counts=True, total=True)
    exp, etot = oracle.probe_counts(k, q, kb)
    assert np.array_equal(hg.to_numpy(c, np.uint32), exp) and tot == etot
    t.free()


def test_any_order_rejects_stable(hg):
    k = hg.to_device(workloads.uniform_keys(100, 32, 1))
    with pytest.raises(hg.HGError) as e:
        hg.hg_build(k, 10, any_order=True, stable=1)
    assert e.value.status == hg.HG_ERR_INVALID_ARG


def test_table_rebuild_reuses_capacity(hg):
    t = hg.Table.create(1 << 18, 1 << 18, 32)
    for i, (n, V) in enumerate([(1 << 18, 1 << 18), (1000, 77), (70000, 1 << 17)]):
        say("rebuild", n, V)
        k = workloads.uniform_keys(n, 32, seed=i)
        t.rebuild(hg.to_device(k), V, seed=i)
        off, ids, ek = table_np(hg, t, 32)
        o = oracle.build_table(k, V, i)
        assert np.array_equal(off, o[0]) and np.array_equal(ids, o[1]) and np.array_equal(ek, o[2])
    with pytest.raises(hg.HGError) as e:
        t.rebuild(hg.to_device(workloads.uniform_keys(10, 32, 1)), (1 << 18) + 1)
    assert e.value.status == hg.HG_ERR_CAPACITY


# ------------------------------------------------------------------ probes


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("kind,n,m,V", [("uniform", 0, 100, 7), ("uniform", 1000, 0, 1000),
                                        ("uniform", 100003, 200001, 100003),
                                        ("dup8", 300000, 300000, 1 << 16),
                                        ("zipf", 200000, 300000, 200000),
                                        ("uniform", 50000, 50000, 1),
                                        # load 8: most buckets hold 4..32 keys
                                        ("uniform", 400000, 300000, 50000)])
def test_probe_counts_match_oracle(hg, kb, variant, kind, n, m, V):
    say("probe", kb, variant, kind, n, m, V)
    k = keys_for(kind, n, kb, seed=1)
    q = workloads.probe_queries(k if n else workloads.uniform_keys(8, kb, 0), m, 0.5, seed=2,
                                key_bits=kb)
    t = hg.hg_build(hg.to_device(k), V, seed=7, variant=variant)
    c, tot = hg.hg_probe(t, hg.to_device(q), counts=True, total=True)
    got = hg.to_numpy(c, np.uint32)
    exp, etot = oracle.probe_counts(k, q, kb)
    assert np.array_equal(got, exp)
    assert tot == etot


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("kind,n,m,V,index", [
    ("uniform", 0, 5000, 7, True),                    # empty table
    ("uniform", 1000, 1, 1000, True),                 # one query
    ("uniform", 100003, 3 * 4096 + 123, 100003, True),  # a few tiles and a ragged tail
    ("uniform", 300007, 300007, 300007, True),        # 1024 ranges, V not a power of two
    ("uniform", 200000, 250001, 600, True),           # fewer buckets than ranges
    ("uniform", 50000, 70000, 1, True),               # one bucket, one range
    ("dup8", 300000, 300000, 1 << 16, False),         # no index: offsets and edge scans
    ("zipf", 200000, 300000, 200000, True),           # long buckets answered by key runs
    ("uniform", 400000, 300000, 50000, True)])        # buckets of 4..32 keys
def test_grouped_probe_matches_oracle(hg, kb, kind, n, m, V, index):
    # queries partitioned by bucket range, probed range by range and their
    # counts put back in input order: the same counts and total as the oracle,
    # over stable and any-order tables, in both probing orders
    say("grouped probe", kb, kind, n, m, V, index)
    k = keys_for(kind, n, kb, seed=31)
    q = workloads.probe_queries(k if n else workloads.uniform_keys(8, kb, 0), m, 0.5, seed=32,
                                key_bits=kb)
    exp, etot = oracle.probe_counts(k, q, kb)
    dq = hg.to_device(q)
    for any_order in (False, True):
        t = hg.hg_build(hg.to_device(k), V, seed=33, index=index, any_order=any_order)
        for order in (hg.PROBE_GROUPED, hg.PROBE_INPUT_ORDER, hg.PROBE_AUTO,
                      hg.PROBE_GROUPED_UNLESS_SKEWED):
            c, tot = hg.hg_probe_ordered(t, dq, order, counts=True, total=True)
            assert np.array_equal(hg.to_numpy(c, np.uint32), exp), (any_order, order)
            assert tot == etot
        for order in (hg.PROBE_GROUPED, hg.PROBE_GROUPED_UNLESS_SKEWED):
            _, tot = hg.hg_probe_ordered(t, dq, order, counts=False, total=True)
            assert tot == etot
        c, tot = hg.hg_probe_ordered(t, dq[:0], hg.PROBE_GROUPED, total=True)
        assert c.numel() == 0 and tot == 0


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("qkind", ["uniform", "zipf"])
def test_grouped_unless_skewed_takes_either_path(hg, kb, qkind):
    # uniform queries spread over the ranges and are grouped; Zipf queries
    # crowd into a few ranges and keep input order (the device decides after
    # the histogram): counts and total equal the oracle's either way, on two
    # calls in a row
    say("grouped unless skewed", kb, qkind)
    n, m, V = 300007, 400009, 300007
    k = keys_for("uniform", n, kb, seed=41)
    if qkind == "zipf":
        q = workloads.zipf_keys(m, 1.2, distinct=1 << 14, seed=42).astype(dt(kb))
        k = np.concatenate([k, q[:n // 4]])
    else:
        q = workloads.probe_queries(k, m, 0.5, seed=42, key_bits=kb)
    exp, etot = oracle.probe_counts(k, q, kb)
    t = hg.hg_build(hg.to_device(k), V, seed=43)
    for _ in range(2):
        c, tot = hg.hg_probe_ordered(t, hg.to_device(q), hg.PROBE_GROUPED_UNLESS_SKEWED,
                                     counts=True, total=True)
        assert np.array_equal(hg.to_numpy(c, np.uint32), exp)
        assert tot == etot


def test_grouped_probe_rejects_unknown_order(hg):
    k = workloads.uniform_keys(1000, 32, 3)
    t = hg.hg_build(hg.to_device(k), 1000, seed=1)
    with pytest.raises(hg.HGError):
        hg.hg_probe_ordered(t, hg.to_device(k), 4)


@pytest.mark.parametrize("kb", [32, 64])
def test_probe_pairs_match_oracle_in_canonical_order(hg, kb):
    n, m, V = 200003, 150001, 100000
    say("pairs", kb)
    k = workloads.duplicate_keys(n, 4.0, kb, seed=3)
    q = workloads.probe_queries(k, m, 0.6, seed=4, key_bits=kb)
    t = hg.hg_build(hg.to_device(k), V, seed=5)
    b, p, tot = hg.hg_probe_pairs(t, hg.to_device(q))
    eb, ep, etot = oracle.probe_pairs(k, q, kb)
    assert tot == etot
    # V2 tables are stable, so pairs come out as (probe id asc, build id asc)
    assert np.array_equal(hg.to_numpy(p, np.uint32), ep)
    assert np.array_equal(hg.to_numpy(b, np.uint32), eb)


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("kind,n,V", [("uniform", 300007, 300007), ("uniform", 120000, 1 << 20),
                                      ("dup8", 200000, 50000), ("equal", 20000, 97),
                                      ("equal", 400000, 97), ("uniform", 300000, 1),
                                      ("zipf", 150000, 150000)])
def test_probe_index_on_and_off_agree_with_oracle(hg, kb, kind, n, V):
    # the per-bucket index holds each bucket's bounds and first keys; buckets
    # of 0, 1, 2 and many keys (light and heavy bins) all occur here
    say("index", kb, kind, n, V)
    k = keys_for(kind, n, kb, seed=11)
    q = workloads.probe_queries(k, n + 4321, 0.5, seed=12, key_bits=kb)
    exp, etot = oracle.probe_counts(k, q, kb)
    eb, ep, _ = oracle.probe_pairs(k, q, kb) if etot <= 5_000_000 else (None, None, None)
    dq = hg.to_device(q)
    for index in (True, False):
        t = hg.hg_build(hg.to_device(k), V, seed=21, index=index)
        c, tot = hg.hg_probe(t, dq, counts=True, total=True)
        assert np.array_equal(hg.to_numpy(c, np.uint32), exp), index
        assert tot == etot
        if eb is not None:
            b, p, tot2 = hg.hg_probe_pairs(t, dq)
            assert tot2 == etot
            assert np.array_equal(hg.to_numpy(p, np.uint32), ep)
            assert np.array_equal(hg.to_numpy(b, np.uint32), eb)


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("R", [8.0, 16.0, 32.0])
def test_probe_index_of_medium_buckets(hg, kb, R):
    # keys repeated about R times, V = n (the appearances sweep's shape):
    # buckets of 9-16 and 17-32 entries get their index entries from groups
    # of 16 and 32 lanes; stable and any-order builds
    say("medium buckets", kb, R)
    n = 400003
    k = workloads.duplicate_keys(n, R, kb, seed=71)
    q = workloads.probe_queries(k, 300001, 0.5, seed=72, key_bits=kb)
    exp, etot = oracle.probe_counts(k, q, kb)
    dk, dq = hg.to_device(k), hg.to_device(q)
    for any_order in (False, True):
        t = hg.hg_build(dk, n, seed=73, any_order=any_order)
        c, tot = hg.hg_probe(t, dq, counts=True, total=True)
        assert np.array_equal(hg.to_numpy(c, np.uint32), exp), any_order
        assert tot == etot


def test_probe_index_follows_rebuilds(hg):
    # one table object rebuilt with the index, without it, and with it again
    # under other keys and ranges: a probe never sees a stale index
    t = hg.Table.create(1 << 18, 1 << 18)
    for step, (n, V, index) in enumerate([(200000, 150000, True), (100000, 90000, False),
                                          (250000, 1 << 18, True), (0, 1000, True),
                                          (5000, 3, True)]):
        say("rebuild", step, n, V, index)
        k = workloads.duplicate_keys(n, 2.0, 32, seed=30 + step) if n else \
            np.zeros(0, np.uint32)
        q = workloads.probe_queries(k if n else workloads.uniform_keys(8, 32, 0), 70000, 0.5,
                                    seed=40 + step)
        t.rebuild(hg.to_device(k), V, seed=step, index=index)
        c, tot = hg.hg_probe(t, hg.to_device(q), counts=True, total=True)
        exp, etot = oracle.probe_counts(k, q)
        assert np.array_equal(hg.to_numpy(c, np.uint32), exp)
        assert tot == etot
    t.free()


def test_probe_pairs_v1_as_sets_and_capacity(hg):
    n, m, V = 50000, 40000, 30000
    k = workloads.duplicate_keys(n, 2.0, 32, seed=8)
    q = workloads.probe_queries(k, m, 0.5, seed=9)
    t = hg.hg_build(hg.to_device(k), V, seed=1, variant=hg.VARIANT_V1)
    eb, ep, etot = oracle.probe_pairs(k, q)
    b, p, tot = hg.hg_probe_pairs(t, hg.to_device(q), capacity=etot - 1)
    assert b is None and tot == etot
    b, p, tot = hg.hg_probe_pairs(t, hg.to_device(q), capacity=etot)
    got = np.stack([hg.to_numpy(p, np.uint32), hg.to_numpy(b, np.uint32)], 1)
    exp = np.stack([ep, eb], 1)
    got = got[np.lexsort((got[:, 1], got[:, 0]))]
    assert np.array_equal(got, exp)


# --------------------------------------------------------------- intersect


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("na,nb,V,kind", [(100000, 150000, 80000, "dup8"),
                                          (0, 1000, 10, "uniform"), (1000, 0, 10, "uniform"),
                                          (200000, 300000, 200000, "zipf")])
def test_intersect_matches_oracle(hg, kb, na, nb, V, kind):
    say("intersect", kb, na, nb, V, kind)
    ka = keys_for(kind, na, kb, seed=21) if na else np.zeros(0, dt(kb))
    kbk = keys_for(kind, nb, kb, seed=22) if nb else np.zeros(0, dt(kb))
    a = hg.hg_build(hg.to_device(ka), V, seed=31)
    b = hg.hg_build(hg.to_device(kbk), V, seed=31)
    c, _, _, tot = hg.hg_intersect(a, b, counts=True, total=True)
    exp, etot = oracle.probe_counts(ka, kbk, kb)
    assert np.array_equal(hg.to_numpy(c, np.uint32), exp)
    assert tot == etot
    if 0 < etot < 5_000_000:
        c2, ai, bi, tot2 = hg.hg_intersect(a, b, counts=False, capacity=etot)
        assert tot2 == etot
        got = np.stack([hg.to_numpy(bi, np.uint32), hg.to_numpy(ai, np.uint32)], 1)
        got = got[np.lexsort((got[:, 1], got[:, 0]))]
        eb, ep, _ = oracle.probe_pairs(ka, kbk, kb)
        assert np.array_equal(got, np.stack([ep, eb], 1))


@pytest.mark.parametrize("kb,nb,any_order", [(32, (3 << 20) + 17, False), (32, 1 << 22, True),
                                             (64, (1 << 21) + 4097, False),
                                             (32, (1 << 20) + 1, True)])
def test_intersect_counts_by_input_windowed_scatter(hg, kb, nb, any_order):
    """Counts by B's input index above 2^20 entries go through the windowed
    scatter (B's ids partitioned by their top bits into L2-sized windows, the
    last window partial, a window count that is not a multiple of eight):
    they equal the oracle's counts of B's keys against A."""
    say("intersect windowed", kb, nb, any_order)
    ka = workloads.duplicate_keys(nb // 2 + 3, 3.0, kb, seed=61)
    kbk = workloads.probe_queries(ka, nb, 0.5, seed=62, key_bits=kb)
    V = nb // 2 + 11
    a = hg.hg_build(hg.to_device(ka), V, seed=8)
    b = hg.hg_build(hg.to_device(kbk), V, seed=8, any_order=any_order)
    c, _, _, tot = hg.hg_intersect(a, b, counts=True, total=True)
    exp, etot = oracle.probe_counts(ka, kbk, kb)
    assert tot == etot
    assert np.array_equal(hg.to_numpy(c, np.uint32), exp)


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("kind", ["uniform", "dup100"])
def test_intersect_edge_order_counts(hg, kb, kind):
    """hg_intersect_edges: per B edge, the count of A entries with that edge's
    key; the same counts as hg_intersect, in B's edge order."""
    ka = keys_for(kind, 150000, kb, seed=51) if kind == "uniform" else \
        workloads.duplicate_keys(150000, 100.0, kb, seed=51)
    kbk = workloads.probe_queries(ka, 120000, 0.6, seed=52, key_bits=kb)
    V = 100000
    a = hg.hg_build(hg.to_device(ka), V, seed=7)
    b = hg.hg_build(hg.to_device(kbk), V, seed=7)
    c, tot = hg.hg_intersect_edges(a, b)
    _, _, bek = b.export()
    exp, etot = oracle.probe_counts(ka, hg.to_numpy(bek, dt(kb)), kb)
    assert np.array_equal(hg.to_numpy(c, np.uint32), exp) and tot == etot
    _, tot2 = hg.hg_intersect_edges(a, b, counts=False)
    assert tot2 == etot


def skew_keys(kind, n, kb, seed):
    if kind == "zipf15":
        return workloads.zipf_keys(n, 1.5, distinct=1 << 12, seed=seed,
                                   map_seed=5).astype(dt(kb))
    if kind == "dup100":
        return workloads.duplicate_keys(n, 100.0, kb, seed)
    if kind == "few":  # a handful of keys, each in a long bucket
        return (workloads.uniform_keys(n, 32, seed) % 7 + 1000).astype(dt(kb))
    if kind == "dup30":  # about two keys of 30 copies per bucket (V = n / 60)
        return workloads.duplicate_keys(n, 30.0, kb, seed)
    if kind == "dup10":  # about twenty keys of 10 copies per bucket (V = n / 200)
        return workloads.duplicate_keys(n, 10.0, kb, seed)
    raise ValueError(kind)


# Which construction path of the key runs each case takes:
#   dup100 (V = 2^14): buckets of one repeated key inside LDS bins (one run,
#     ids read from the edge array);
#   dup30 (V = n/60): LDS bins whose long buckets hold a few keys (the other
#     keys sorted across one wave);
#   dup10 (V = n/200): LDS bins whose long buckets hold more than 64 entries
#     of other keys (the general pass, sorted in LDS);
#   few (V = 5000): buckets of one key in bins too large for LDS (chunked path,
#     one run);
#   zipf15 (V = n): bins too large for LDS holding a dominant key and a few
#     others (chunked path, others sorted in LDS);
#   zipf15 (V = 1): one bucket of every key (chunked path, others radix-sorted
#     through global memory).
@pytest.mark.parametrize("any_order", [False, True])
@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("kind,n,m,V", [("zipf15", 200000, 300000, 200000),
                                        ("dup100", 150000, 150000, 1 << 14),
                                        ("dup30", 200000, 150000, 200000 // 60),
                                        ("dup10", 200000, 150000, 200000 // 200),
                                        ("few", 60000, 50000, 5000),
                                        ("zipf15", 30000, 40000, 1)])
def test_long_buckets_use_key_runs_with_exact_results(hg, kb, kind, n, m, V, any_order):
    # buckets longer than 32 entries are probed through their key runs:
    # counts, pairs and intersections must equal the oracle's, and equal the
    # same table probed by scanning (index off)
    say("key runs", kb, kind, n, m, V, any_order)
    k = skew_keys(kind, n, kb, seed=41)
    q = skew_keys(kind, m, kb, seed=42)
    q[::3] = workloads.uniform_keys(q[::3].size, kb, 43)  # some misses into long buckets
    exp, etot = oracle.probe_counts(k, q, kb)
    dq = hg.to_device(q)
    t = hg.hg_build(hg.to_device(k), V, seed=17, any_order=any_order)
    ts = hg.hg_build(hg.to_device(k), V, seed=17, index=False)
    c, tot = hg.hg_probe(t, dq, counts=True, total=True)
    assert np.array_equal(hg.to_numpy(c, np.uint32), exp) and tot == etot
    c2, _ = hg.hg_probe(ts, dq, counts=True)
    assert torch.equal(c, c2)
    # pairs for the queries whose matches stay small
    light = np.nonzero(exp <= 200)[0][:20000]
    qs = q[light]
    b, p, ptot = hg.hg_probe_pairs(t, hg.to_device(qs))
    eb, ep, et = oracle.probe_pairs(k, qs, kb)
    assert ptot == et
    b, p = hg.to_numpy(b, np.uint32)[:et], hg.to_numpy(p, np.uint32)[:et]
    assert np.array_equal(p, ep)
    if any_order:  # build ids inside one query follow the bucket's order
        o = np.lexsort((b, p))
        b = b[o]
    assert np.array_equal(b, eb)
    # intersection: A = the table with runs, B = a table of the light queries
    tb = hg.hg_build(hg.to_device(qs), V, seed=17)
    ci, _, _, itot = hg.hg_intersect(t, tb, counts=True, total=True)
    assert itot == et
    assert np.array_equal(hg.to_numpy(ci, np.uint32), oracle.probe_counts(k, qs, kb)[0])
    if 0 < et < 5_000_000:
        _, ai, bi, tot2 = hg.hg_intersect(t, tb, counts=False, capacity=et)
        got = np.stack([hg.to_numpy(bi, np.uint32), hg.to_numpy(ai, np.uint32)], 1)
        got = got[np.lexsort((got[:, 1], got[:, 0]))]
        assert tot2 == et and np.array_equal(got, np.stack([ep, eb], 1))


def test_intersect_rejects_mismatched_tables(hg):
    k = hg.to_device(workloads.uniform_keys(1000, 32, 1))
    a = hg.hg_build(k, 100, seed=1)
    for b in (hg.hg_build(k, 101, seed=1), hg.hg_build(k, 100, seed=2)):
        with pytest.raises(hg.HGError) as e:
            hg.hg_intersect(a, b)
        assert e.value.status == hg.HG_ERR_MISMATCH


def test_probe_counts_do_not_depend_on_range_seed_or_variant(hg):
    """Metamorphic: the count definition has no hash in it."""
    k = workloads.duplicate_keys(100000, 5.0, 32, seed=40)
    q = workloads.probe_queries(k, 80000, 0.5, seed=41)
    dq = hg.to_device(q)
    ref = None
    for V, seed, var in [(1, 0, 2), (7, 1, 1), (100000, 2, 2), (1 << 25, 3, 2), (3, 4, 1)]:
        t = hg.hg_build(hg.to_device(k), V, seed=seed, variant=var)
        c, _ = hg.hg_probe(t, dq)
        got = hg.to_numpy(c, np.uint32)
        if ref is None:
            ref = got
        assert np.array_equal(got, ref)
    assert np.array_equal(ref, oracle.probe_counts(k, q)[0])


def test_random_access_micro_roofline(hg):
    """The micro-roofline kernels run and order as the memory hierarchy does:
    an L2-sized footprint serves random reads faster than an HBM-sized one."""
    l2 = hg.random_access_rate(hg.MICRO_READ16, 1 << 22, 1 << 24)
    hbm = hg.random_access_rate(hg.MICRO_READ16, 1 << 30, 1 << 24)
    at = hg.random_access_rate(hg.MICRO_ATOMIC4, 1 << 22, 1 << 22)
    r4 = hg.random_access_rate(hg.MICRO_READ4, 1 << 12, 1 << 20)
    assert l2 > hbm > 0 and at > 0 and r4 > 0
