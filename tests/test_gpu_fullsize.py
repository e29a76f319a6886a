"""Parity at the workloads' full sizes, in the benchmark's launch configuration.

Sizes: 2^28 uniform uint32 keys with hash ranges 2^26, 2^28 and 2^30 (V1 and
V2), 2^28 queries with 50% hits; 2^27 uint64 keys; skewed joins with 2^27
Zipf build keys over 2^24 distinct values, hash range 2^27 and 2^28 Zipf
queries.  Tables are built as the benchmark builds them (a table created at
capacity, rebuilt in place, probed for counts into a preallocated buffer).

A full oracle table at these sizes would take long on the host, so a built
table is checked by properties that together admit exactly one table, the
oracle's stable one, with the bucket of every key taken from the oracle's hash
(Eq. 1 in C):
  1. offsets equal the exclusive prefix sum of the per-bucket key counts;
  2. ids hold every input index exactly once;
  3. ekeys[p] == keys[ids[p]];
  4. the key at edge p hashes to the bucket whose segment holds p;
  5. (V2) ids ascend inside every bucket.
V1 satisfies 1-4; after sorting ids inside each bucket it must equal the V2
table.  Probe counts are compared with the oracle's counts for every query
(the oracle matches keys by a sort-merge, without hashing).  The checks run as
torch tensor operations, independent of the library's kernels.
"""
import numpy as np
import pytest

import oracle
from paper_1907_02900_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 1 << 28
MASK = 0xFFFFFFFF


@pytest.fixture(scope="module")
def hg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1907_02900_amd import hg as _hg
    _hg.lib()
    return _hg


def say(*a):
    print("[case]", *a, flush=True)


def u64(t):
    """device int32/int64 view of unsigned data -> int64 holding the value"""
    return t.to(torch.int64) & MASK if t.dtype == torch.int32 else t


def check_table(hg, table, keys_dev, h_dev, V, stable):
    """Properties 1-5 (5 if stable).  h_dev: oracle bucket of every input key
    (int64, device).  Returns (offsets, ids) as int64 device tensors."""
    info = table.info()
    n = keys_dev.numel()
    assert info.n == n and info.hash_range == V
    off, ids, ek = table.export()
    off, ids, ek = u64(off), u64(ids), u64(ek)
    cnt = torch.bincount(h_dev, minlength=V)
    exp_off = torch.zeros(V + 1, dtype=torch.int64, device=off.device)
    torch.cumsum(cnt, 0, out=exp_off[1:])
    assert torch.equal(off, exp_off), "offsets"
    del exp_off
    assert int(ids.min()) >= 0 and int(ids.max()) < n
    assert bool((torch.bincount(ids, minlength=n) == 1).all()), "ids not a permutation"
    assert torch.equal(ek, keys_dev[ids]), "ekeys != keys[ids]"
    seg = torch.repeat_interleave(torch.arange(V, device=off.device), cnt, output_size=n)
    del cnt
    assert torch.equal(h_dev[ids], seg), "edge in the wrong bucket"
    if stable and n > 1:
        ok = (seg[1:] != seg[:-1]) | (ids[1:] > ids[:-1])
        assert bool(ok.all()), "ids not ascending inside a bucket"
    del seg, ek
    return off, ids


def sort_within_buckets(off, ids, V):
    n = ids.numel()
    seg = torch.repeat_interleave(torch.arange(V, device=ids.device), off[1:] - off[:-1],
                                  output_size=n)
    order = torch.argsort(seg * (1 << 32) + ids)
    return ids[order]


@pytest.fixture(scope="module")
def uniform(hg):
    say("uniform inputs 2^28")
    keys = workloads.uniform_keys(N, 32, seed=0)
    q = workloads.probe_queries(keys, N, 0.5, seed=1)
    say("oracle counts 2^28 x 2^28")
    exp, etot = oracle.probe_counts(keys, q)
    return keys, q, exp, etot


@pytest.mark.parametrize("layout", ["any_order", "stable"])
def test_full_uniform_bench_step(hg, uniform, layout):
    """The benchmark's timed step exactly as bench.py runs it: a table created
    at capacity (2^28 keys, V = 2^28), rebuilt in place with the probe index
    (any order, as timed by default; stable with --stable), then
    Probe-Standard counts of all 2^28 queries into a preallocated buffer
    (grouped by bucket range, as hg_probe chooses here, and in input order).
    Offsets are exact; the buckets, as multisets, equal the oracle's (ids
    sorted inside each bucket equal torch's stable argsort of the oracle's
    buckets); the stable layout equals it entry for entry; every count and the
    total equal the oracle's."""
    keys, q, exp, etot = uniform
    V = N
    any_order = layout == "any_order"
    say("V2 build (%s, index) + probe, n = V = m = 2^28" % layout)
    dk, dq = hg.to_device(keys), hg.to_device(q)
    table = hg.Table.create(N, V, 32)
    counts = torch.empty(N, dtype=torch.int32, device="cuda")
    for _ in range(2):  # a rebuild over a previous build, as in the timed loop
        table.rebuild(dk, V, seed=0, variant=hg.VARIANT_V2, any_order=any_order)
        hg.hg_probe(table, dq, counts=True, total=False, out=counts)
    _, tot = hg.hg_probe(table, dq, counts=False, total=True)
    torch.cuda.synchronize()
    assert np.array_equal(hg.to_numpy(counts, np.uint32), exp)
    assert tot == etot
    # hg_probe groups the queries by bucket range at this size; the same
    # counts probed in input order
    counts.fill_(-1)
    hg.hg_probe_ordered(table, dq, hg.PROBE_INPUT_ORDER, out=counts)
    torch.cuda.synchronize()
    assert np.array_equal(hg.to_numpy(counts, np.uint32), exp)
    del counts
    h = torch.from_numpy(oracle.hash_buckets(keys, V, 0).astype(np.int64)).cuda()
    off, ids = check_table(hg, table, u64(dk), h, V, stable=not any_order)
    stable_ids = torch.sort(h, stable=True).indices
    del h
    if any_order:
        ids = sort_within_buckets(off, ids, V)
    assert torch.equal(ids, stable_ids), "buckets differ from the oracle's as multisets"
    table.free()


@pytest.mark.parametrize("layout", ["stable", "any_order"])
def test_full_uniform_pairs_materialised(hg, uniform, layout):
    """All ~1.5e8 matching pairs of the 2^28 x 2^28 uniform workload: the
    total equals the oracle's, every pair joins equal keys, each probe id
    appears exactly its oracle count times, probe ids ascend and no pair
    repeats, which with the counts leaves exactly the oracle's pair set.  In
    the stable table build ids also ascend inside each probe id (the oracle's
    canonical order); in the any-order table (the benchmark's layout) they
    follow the table's bucket order."""
    keys, q, exp, etot = uniform
    V = N
    any_order = layout == "any_order"
    say("pairs, n = V = m = 2^28, %s" % layout)
    dk, dq = hg.to_device(keys), hg.to_device(q)
    table = hg.Table.create(N, V, 32)
    table.rebuild(dk, V, seed=0, variant=hg.VARIANT_V2, any_order=any_order)
    b, p, tot = hg.hg_probe_pairs(table, dq)
    torch.cuda.synchronize()
    assert tot == etot
    bi, pi = u64(b), u64(p)
    del b, p
    assert bool((pi[1:] >= pi[:-1]).all())
    cnt = torch.bincount(pi, minlength=N)
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), exp)
    del cnt
    assert bool((u64(dk)[bi] == u64(dq)[pi]).all())
    if any_order:
        order = torch.argsort(pi * (1 << 32) + bi)
        bi, pi = bi[order], pi[order]
        del order
    same = pi[1:] == pi[:-1]
    assert bool((bi[1:][same] > bi[:-1][same]).all())
    table.free()


@pytest.mark.parametrize("log2V", [26, 28, 30])
def test_full_range_sweep_v1_and_v2(hg, uniform, log2V):
    keys, q, exp, etot = uniform
    V = 1 << log2V
    say("range sweep V = 2^%d" % log2V)
    dk, dq = hg.to_device(keys), hg.to_device(q)
    kd = u64(dk)
    h = torch.from_numpy(oracle.hash_buckets(keys, V, 5).astype(np.int64)).cuda()
    table = hg.Table.create(N, V, 32)
    counts = torch.empty(N, dtype=torch.int32, device="cuda")
    table.rebuild(dk, V, seed=5, variant=hg.VARIANT_V2)
    _, ids2 = check_table(hg, table, kd, h, V, stable=True)
    hg.hg_probe(table, dq, counts=True, out=counts)
    assert np.array_equal(hg.to_numpy(counts, np.uint32), exp)
    table.rebuild(dk, V, seed=5, variant=hg.VARIANT_V1)
    off1, ids1 = check_table(hg, table, kd, h, V, stable=False)
    assert torch.equal(sort_within_buckets(off1, ids1, V), ids2)
    del off1, ids1, ids2
    hg.hg_probe(table, dq, counts=True, out=counts)
    assert np.array_equal(hg.to_numpy(counts, np.uint32), exp)
    table.free()


def test_full_uint64_keys(hg):
    n = N // 2
    say("uint64 keys 2^27")
    keys = workloads.uniform_keys(n, 64, seed=3)
    q = workloads.probe_queries(keys, n, 0.5, seed=4)
    dk, dq = hg.to_device(keys), hg.to_device(q)
    table = hg.Table.create(n, n, 64)
    table.rebuild(dk, n, seed=0)
    h = torch.from_numpy(oracle.hash_buckets(keys, n, 0).astype(np.int64)).cuda()
    check_table(hg, table, dk, h, n, stable=True)
    del h
    c, tot = hg.hg_probe(table, dq, counts=True, total=True)
    exp, etot = oracle.probe_counts(keys, q)
    assert np.array_equal(hg.to_numpy(c, np.uint32), exp)
    assert tot == etot
    table.free()


def test_full_2p30_keys_two_tier_build(hg):
    # 2^30 keys, V = 2^30: 2^18 final bins reached by two partition passes of
    # 9 bits each; the table is checked by the same properties, and the
    # counts of 2^20 sampled queries against the oracle
    n = 1 << 30
    say("2^30 keys, V = 2^30")
    keys = workloads.uniform_keys(n, 32, seed=8)
    dk = hg.to_device(keys)
    table = hg.Table.create(n, n, 32)
    table.rebuild(dk, n, seed=3)
    h = torch.from_numpy(oracle.hash_buckets(keys, n, 3).astype(np.int64)).cuda()
    check_table(hg, table, u64(dk), h, n, stable=True)
    del h
    q = workloads.probe_queries(keys, 1 << 20, 0.5, seed=9)
    c, tot = hg.hg_probe(table, hg.to_device(q), counts=True, total=True)
    say("oracle counts 2^30 x 2^20")
    exp, etot = oracle.probe_counts(keys, q)
    assert np.array_equal(hg.to_numpy(c, np.uint32), exp) and tot == etot
    table.free()


@pytest.mark.parametrize("s", [0.8, 1.2, 1.5])
def test_full_zipf_join(hg, s):
    nb, V = N // 2, N // 2
    say("zipf join s=%.1f: build 2^27, probe 2^28" % s)
    # both sides draw from one law over the same keys (shared rank -> key map)
    keys = workloads.zipf_keys(nb, s, distinct=1 << 24, seed=21, map_seed=99)
    q = workloads.zipf_keys(N, s, distinct=1 << 24, seed=22, map_seed=99)
    dk, dq = hg.to_device(keys), hg.to_device(q)
    table = hg.Table.create(nb, V, 32)
    table.rebuild(dk, V, seed=9)
    h = torch.from_numpy(oracle.hash_buckets(keys, V, 9).astype(np.int64)).cuda()
    check_table(hg, table, u64(dk), h, V, stable=True)
    del h
    say("zipf oracle counts")
    exp, etot = oracle.probe_counts(keys, q)
    c, tot = hg.hg_probe(table, dq, counts=True, total=True)
    assert np.array_equal(hg.to_numpy(c, np.uint32), exp)
    assert tot == etot
    # pairs: the total for all 2^28 queries (too many to materialise), then
    # the materialised pairs of 4096 queries whose matches fit in memory
    b, p, ptot = hg.hg_probe_pairs(table, dq, capacity=0)
    assert b is None and ptot == etot
    rng = np.random.default_rng(2)
    light = np.nonzero(exp <= 64)[0]
    pick = np.sort(rng.choice(light, size=min(4096, light.size), replace=False))
    qs = q[pick]
    b, p, ptot = hg.hg_probe_pairs(table, hg.to_device(qs))
    eb, ep, et = oracle.probe_pairs(keys, qs)
    assert ptot == et
    assert np.array_equal(hg.to_numpy(p, np.uint32), ep)
    assert np.array_equal(hg.to_numpy(b, np.uint32), eb)
    # bucket-wise intersection with a table of the queries (same hash)
    say("zipf intersect")
    tq = hg.hg_build(dq, V, seed=9)
    cb, _, _, itot = hg.hg_intersect(table, tq, counts=True, total=True)
    assert itot == etot
    assert np.array_equal(hg.to_numpy(cb, np.uint32), exp)
    tq.free()
    table.free()


def test_full_collection_build_once_intersect_many(hg):
    """The benchmark's collection: 2^20 sets (mean 32 keys, Pareto tail 1.5,
    at most 2^16), columns uniform over 2^20, 2^24 random pairs.  Sampled sets
    (every heavy one and 3000 others) equal the oracle's per-set tables; the
    counts of 20000 sampled pairs equal the oracle's join sizes, the total
    equals the sum of all counts, and the total is the same when it is asked
    for alone."""
    S = 1 << 20
    kc, oc = workloads.collection_sets(S, 32, 1 << 20, seed=31)
    pc = workloads.set_pairs(1 << 24, S, S, seed=32)
    say("collection", S, kc.size)
    c = hg.Collection(hg.to_device(kc), torch.from_numpy(oc.astype(np.int32)).cuda(), seed=5)
    bb, off, ids, ek = c.arrays()
    torch.cuda.synchronize()
    bb = hg.to_numpy(bb, np.uint64)
    off = hg.to_numpy(off, np.uint32)
    ids = hg.to_numpy(ids, np.uint32)
    ek = hg.to_numpy(ek, np.uint32)
    sizes = np.diff(oc)
    rng = np.random.default_rng(8)
    sample = np.union1d(np.flatnonzero(sizes > 1536), rng.choice(S, 3000, replace=False))
    for s in sample:
        lo, hi = int(oc[s]), int(oc[s + 1])
        V = oracle.set_hash_range(hi - lo)
        assert int(bb[s + 1] - bb[s]) == V
        o, i, e = oracle.build_table(kc[lo:hi], V, 5, 32)
        b0 = int(bb[s])
        assert np.array_equal(off[b0:b0 + V + 1].astype(np.int64) - lo, o.astype(np.int64)), s
        assert np.array_equal(ids[lo:hi].astype(np.int64) - lo, i.astype(np.int64)), s
        assert np.array_equal(ek[lo:hi], e), s
    cnt, tot = c.intersect(c, torch.from_numpy(pc.view(np.int32)).cuda())
    got = hg.to_numpy(cnt, np.uint64)
    assert tot == int(got.sum())
    q = rng.choice(pc.shape[0], 20000, replace=False)
    assert np.array_equal(got[q], oracle.pair_match_counts(kc, oc, kc, oc, pc[q]))
    _, tot2 = c.intersect(c, torch.from_numpy(pc.view(np.int32)).cuda(), counts=False)
    assert tot2 == tot
    c.free()
