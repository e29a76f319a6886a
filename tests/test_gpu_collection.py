"""Collections: many sets built once, intersected pair by pair (Sec. 3.4).

The concatenated tables must equal the oracle's stable per-set tables bit for
bit (bucket bases, offsets, ids, keys), for sets built in LDS windows and for
heavy sets built by the radix-sort path, at the window boundaries, with
repeated keys (long buckets), both key widths and several range shifts.  Pair
counts must equal the oracle's join sizes for every pair, including empty
sets, self pairs, pairs whose walked side spans many workgroups, and pairs
across two collections.
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


def dt(kb):
    return np.uint64 if kb == 64 else np.uint32


def mixed_sets(kb, seed, dup_range=None):
    """Tiny, window-boundary and heavy sets in one collection."""
    rng = np.random.default_rng(seed)
    sizes = list(rng.integers(0, 40, 2500))
    sizes += [1535, 1536, 1537, 1538, 0, 2047, 2048, 2049, 1, 3000, 0, 0]
    sizes += list(rng.integers(0, 6, 300))
    sizes += [20000, 70001, 5]
    rng.shuffle(sizes)
    off = np.zeros(len(sizes) + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    n = int(off[-1])
    if dup_range:
        keys = rng.integers(0, dup_range, n).astype(dt(kb))
    else:
        keys = workloads.uniform_keys(n, kb, seed + 1)
    return keys, off


def dev_off(off):
    return torch.from_numpy(off.astype(np.int32)).cuda()


def check_collection(hg, c, keys, off, seed, shift, kb):
    bb, o, ids, ek = c.arrays()
    torch.cuda.synchronize()
    e_bb, e_off, e_ids, e_ek = oracle.collection_table(keys, off, seed, shift, kb)
    S = off.size - 1
    got_bb = hg.to_numpy(bb, np.uint64)
    assert np.array_equal(got_bb[:S + 1], e_bb) and got_bb[S + 1] == e_bb[-1]
    assert np.array_equal(hg.to_numpy(o, np.uint32), e_off)
    assert np.array_equal(hg.to_numpy(ids, np.uint32), e_ids)
    assert np.array_equal(hg.to_numpy(ek, dt(kb)), e_ek)
    info = c.info()
    assert info.sets == S and info.n == keys.size and info.buckets == int(e_bb[-1])


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("shift", [0, -1, 2])
def test_collection_tables_match_oracle(hg, kb, shift):
    print("[case] collection build", kb, shift, flush=True)
    keys, off = mixed_sets(kb, 10 + shift)
    c = hg.Collection(hg.to_device(keys), dev_off(off), seed=77, range_shift=shift)
    check_collection(hg, c, keys, off, 77, shift, kb)
    assert c.info().heavy_keys > 0
    c.free()


def test_collection_long_buckets_take_the_stable_path(hg):
    # keys from 6 values: buckets far longer than the insertion-sort limit
    keys, off = mixed_sets(32, 3, dup_range=6)
    c = hg.Collection(hg.to_device(keys), dev_off(off), seed=5)
    check_collection(hg, c, keys, off, 5, 0, 32)
    c.free()


@pytest.mark.parametrize("sizes", [[], [0], [0, 0, 0], [1], [5000], [1536] * 40, [1537] * 7])
def test_collection_edge_shapes(hg, sizes):
    off = np.zeros(len(sizes) + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    keys = workloads.duplicate_keys(int(off[-1]), 2.0, 32, seed=len(sizes))
    c = hg.Collection(hg.to_device(keys) if keys.size else torch.empty(0, dtype=torch.int32,
                                                                        device="cuda"),
                      dev_off(off), seed=1)
    check_collection(hg, c, keys, off, 1, 0, 32)
    if len(sizes):
        pairs = workloads.set_pairs(50, len(sizes), len(sizes), seed=2)
        cnt, tot = c.intersect(c, torch.from_numpy(pairs.view(np.int32)).cuda())
        exp = oracle.pair_match_counts(keys, off, keys, off, pairs)
        assert np.array_equal(hg.to_numpy(cnt, np.uint64), exp) and tot == int(exp.sum())
    c.free()


def test_collection_rejects_bad_offsets(hg):
    keys = hg.to_device(workloads.uniform_keys(100, 32, 1))
    for bad in ([0, 50, 40, 100], [3, 50, 100]):
        with pytest.raises(hg.HGError) as e:
            hg.Collection(keys, dev_off(np.array(bad, np.int64)))
        assert e.value.status == hg.HG_ERR_INVALID_ARG


@pytest.mark.parametrize("kb", [32, 64])
def test_pair_counts_match_oracle(hg, kb):
    print("[case] collection pairs", kb, flush=True)
    keys, off = mixed_sets(kb, 21, dup_range=5000)
    S = off.size - 1
    c = hg.Collection(hg.to_device(keys), dev_off(off), seed=9)
    pairs = workloads.set_pairs(30000, S, S, seed=4)
    sizes = np.diff(off)
    big = np.flatnonzero(sizes > 1536).astype(np.uint32)
    empty = np.flatnonzero(sizes == 0).astype(np.uint32)
    extra = np.array([(i, i) for i in big] + [(i, j) for i in big for j in big] +
                     [(empty[0], big[0]), (big[0], empty[0]), (empty[0], empty[0])], np.uint32)
    pairs = np.concatenate([pairs, extra])
    cnt, tot = c.intersect(c, torch.from_numpy(pairs.view(np.int32)).cuda())
    exp = oracle.pair_match_counts(keys, off, keys, off, pairs, kb)
    got = hg.to_numpy(cnt, np.uint64)
    assert np.array_equal(got, exp)
    assert tot == int(exp.sum())
    # the total alone, and the counts alone
    _, tot2 = c.intersect(c, torch.from_numpy(pairs.view(np.int32)).cuda(), counts=False)
    cnt3, none = c.intersect(c, torch.from_numpy(pairs.view(np.int32)).cuda(), total=False)
    assert tot2 == tot and none is None and np.array_equal(hg.to_numpy(cnt3, np.uint64), exp)
    c.free()


def test_pairs_across_two_collections(hg):
    ka, oa = workloads.collection_sets(3000, 30, 4000, seed=1, max_size=5000)
    kb_, ob = workloads.collection_sets(2000, 50, 4000, seed=2, max_size=9000)
    a = hg.Collection(hg.to_device(ka), dev_off(oa), seed=3)
    b = hg.Collection(hg.to_device(kb_), dev_off(ob), seed=3, range_shift=1)
    pairs = workloads.set_pairs(40000, 3000, 2000, seed=5)
    cnt, tot = a.intersect(b, torch.from_numpy(pairs.view(np.int32)).cuda())
    exp = oracle.pair_match_counts(ka, oa, kb_, ob, pairs)
    assert np.array_equal(hg.to_numpy(cnt, np.uint64), exp) and tot == int(exp.sum())
    # swapping the collections swaps the pair order and nothing else
    cnt2, _ = b.intersect(a, torch.from_numpy(pairs[:, ::-1].copy().view(np.int32)).cuda())
    assert np.array_equal(hg.to_numpy(cnt2, np.uint64), exp)
    # errors: different seeds, an index out of range, no pairs
    other = hg.Collection(hg.to_device(kb_), dev_off(ob), seed=4)
    with pytest.raises(hg.HGError) as e:
        a.intersect(other, torch.from_numpy(pairs.view(np.int32)).cuda())
    assert e.value.status == hg.HG_ERR_MISMATCH
    bad = pairs[:10].copy()
    bad[3, 1] = 2000
    with pytest.raises(hg.HGError) as e:
        a.intersect(b, torch.from_numpy(bad.view(np.int32)).cuda())
    assert e.value.status == hg.HG_ERR_INVALID_ARG
    c0, t0 = a.intersect(b, torch.empty((0, 2), dtype=torch.int32, device="cuda"))
    assert c0.numel() == 0 and t0 == 0
    for x in (a, b, other):
        x.free()


@pytest.mark.parametrize("size_hi", [2, 200])
def test_pair_counts_both_staging_paths(hg, size_hi):
    """Sets of one or two keys give workgroups of 2048 work items with more
    pairs than the LDS metadata holds (the direct path); sets of up to 200
    keys give few pairs per workgroup (the staged path)."""
    rng = np.random.default_rng(size_hi)
    sizes = rng.integers(1, size_hi + 1, 20000)
    off = np.zeros(sizes.size + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    keys = rng.integers(0, 300, int(off[-1])).astype(np.uint32)
    c = hg.Collection(hg.to_device(keys), dev_off(off), seed=2)
    pairs = workloads.set_pairs(60000, sizes.size, sizes.size, seed=3)
    cnt, tot = c.intersect(c, torch.from_numpy(pairs.view(np.int32)).cuda())
    exp = oracle.pair_match_counts(keys, off, keys, off, pairs)
    assert np.array_equal(hg.to_numpy(cnt, np.uint64), exp) and tot == int(exp.sum())
    c.free()
