"""Decremental HashGraph: erasing keys from a built table.

After an erase every reader must see exactly the remaining multiset: the
exported (compacted) CSR equals the oracle's stable table with the erased
entries taken out (original ids kept, order inside a bucket kept), probe
counts and pairs equal the oracle's on the remaining entries, and
intersections use only live entries on either side.  Erases are applied in
rounds, on tables with short buckets, long buckets (key runs) and 64-bit
keys.
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


def keys_for(kind, n, kb, seed):
    if kind == "uniform":
        return workloads.uniform_keys(n, kb, seed)
    if kind == "dup8":
        return workloads.duplicate_keys(n, 8.0, kb, seed)
    if kind == "zipf":
        return workloads.zipf_keys(n, 1.3, distinct=1 << 12, seed=seed).astype(dt(kb))
    raise ValueError(kind)


def remaining_table(full, V, gone):
    """The oracle's stable table without the entries whose key is in `gone`."""
    off, ids, ek = full
    keep = ~np.isin(ek, gone)
    seg = np.searchsorted(off.astype(np.int64), np.arange(ids.size), side="right") - 1
    off2 = np.zeros(V + 1, np.uint32)
    np.cumsum(np.bincount(seg[keep], minlength=V), out=off2[1:])
    return off2, ids[keep], ek[keep]


def export_np(hg, t, kb):
    off, ids, ek = t.export()
    torch.cuda.synchronize()
    return hg.to_numpy(off, np.uint32), hg.to_numpy(ids, np.uint32), hg.to_numpy(ek, dt(kb))


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("kind,n,V", [("uniform", 300000, 300000), ("dup8", 400000, 1 << 16),
                                      ("zipf", 200000, 200000)])
def test_erase_rounds_match_oracle(hg, kb, kind, n, V):
    print("[case] erase", kb, kind, n, V, flush=True)
    k = keys_for(kind, n, kb, seed=5)
    q = workloads.probe_queries(k, 150000, 0.6, seed=6, key_bits=kb)
    full = oracle.build_table(k, V, 23, kb)
    t = hg.hg_build(hg.to_device(k), V, seed=23)
    rng = np.random.default_rng(7)
    distinct = np.unique(k)
    gone = np.zeros(0, dt(kb))
    for rnd, frac in enumerate((0.3, 0.2, 1.0)):
        pick = rng.choice(distinct, size=int(frac * distinct.size), replace=False)
        absent = workloads.uniform_keys(500, kb, 100 + rnd)
        batch = np.concatenate([pick, pick[: pick.size // 4], absent]).astype(dt(kb))
        rng.shuffle(batch)
        removed = t.erase(hg.to_device(batch))
        before = int(np.isin(k, gone).sum())
        gone = np.union1d(gone, pick).astype(dt(kb))
        live = ~np.isin(k, gone)
        assert removed == int((~live).sum()) - before, rnd
        assert t.live() == int(live.sum()) and t.info().n == n
        assert t.lengths() is not None
        # the exported CSR is the stable table of what remains
        off, ids, ek = export_np(hg, t, kb)
        e_off, e_ids, e_ek = remaining_table(full, V, gone)
        assert np.array_equal(off, e_off), rnd
        assert np.array_equal(ids, e_ids), rnd
        assert np.array_equal(ek, e_ek), rnd
        # probes see only live entries
        c, tot = hg.hg_probe(t, hg.to_device(q), counts=True, total=True)
        exp = oracle.probe_counts(k[live], q, kb)[0]
        assert np.array_equal(hg.to_numpy(c, np.uint32), exp), rnd
        assert tot == int(exp.sum())
        if oracle.probe_counts(k, q, kb)[1] < 5_000_000:
            eb, ep, et = oracle.probe_pairs(k, q, kb)
            keep = live[eb]
            b, p, ptot = hg.hg_probe_pairs(t, hg.to_device(q))
            assert ptot == int(keep.sum())
            if ptot:
                assert np.array_equal(hg.to_numpy(p, np.uint32), ep[keep]), rnd
                assert np.array_equal(hg.to_numpy(b, np.uint32), eb[keep]), rnd
        # intersection with the erased table as A
        tq = hg.hg_build(hg.to_device(q), V, seed=23)
        ci, _, _, itot = hg.hg_intersect(t, tq, counts=True, total=True)
        assert itot == int(exp.sum())
        assert np.array_equal(hg.to_numpy(ci, np.uint32), exp)
        tq.free()
    t.free()


def test_erased_table_as_intersect_b_side(hg):
    n, V = 200000, 150000
    k = workloads.duplicate_keys(n, 4.0, 32, seed=11)
    q = workloads.probe_queries(k, 120000, 0.7, seed=12)
    a = hg.hg_build(hg.to_device(k), V, seed=4)
    b = hg.hg_build(hg.to_device(q), V, seed=4)
    gone = np.unique(q)[::3]
    b.erase(hg.to_device(gone))
    live_q = ~np.isin(q, gone)
    c, _, _, tot = hg.hg_intersect(a, b, counts=True, total=True)
    exp = oracle.probe_counts(k, q)[0]
    got = hg.to_numpy(c, np.uint32)
    assert np.array_equal(got[live_q], exp[live_q])
    assert tot == int(exp[live_q].sum())
    # pairs: only B's live entries
    _, ai, bi, tot2 = hg.hg_intersect(a, b, counts=False, capacity=tot)
    eb, ep, _ = oracle.probe_pairs(k, q)
    keep = live_q[ep]
    gotp = np.stack([hg.to_numpy(bi, np.uint32), hg.to_numpy(ai, np.uint32)], 1)
    gotp = gotp[np.lexsort((gotp[:, 1], gotp[:, 0]))]
    assert tot2 == int(keep.sum())
    assert np.array_equal(gotp, np.stack([ep[keep], eb[keep]], 1))


def test_erase_any_order_table_and_rebuild(hg):
    n, V = 250000, 200000
    k = workloads.duplicate_keys(n, 3.0, 32, seed=21)
    t = hg.Table.create(n, V, 32)
    t.rebuild(hg.to_device(k), V, seed=2, any_order=True)
    gone = np.unique(k)[::2]
    t.erase(hg.to_device(gone))
    live = ~np.isin(k, gone)
    off, ids, ek = export_np(hg, t, 32)
    e_off, e_ids, _ = remaining_table(oracle.build_table(k, V, 2), V, gone)
    assert np.array_equal(off, e_off)
    seg = np.searchsorted(off.astype(np.int64), np.arange(ids.size), side="right") - 1
    assert np.array_equal(ids[np.lexsort((ids, seg))], e_ids)  # buckets as multisets
    assert np.array_equal(ek, k[ids])
    q = workloads.probe_queries(k, 80000, 0.5, seed=22)
    c, _ = hg.hg_probe(t, hg.to_device(q))
    assert np.array_equal(hg.to_numpy(c, np.uint32), oracle.probe_counts(k[live], q)[0])
    # queries grouped by bucket range see the same live lengths
    c, _ = hg.hg_probe_ordered(t, hg.to_device(q), hg.PROBE_GROUPED)
    assert np.array_equal(hg.to_numpy(c, np.uint32), oracle.probe_counts(k[live], q)[0])
    # a rebuild starts from a full table again
    t.rebuild(hg.to_device(k), V, seed=2)
    assert t.lengths() is None and t.live() == n
    off, ids, ek = export_np(hg, t, 32)
    o = oracle.build_table(k, V, 2)
    assert np.array_equal(off, o[0]) and np.array_equal(ids, o[1]) and np.array_equal(ek, o[2])
    t.free()


def test_erase_needs_the_probe_index(hg):
    k = hg.to_device(workloads.uniform_keys(1000, 32, 1))
    for t in (hg.hg_build(k, 500, variant=hg.VARIANT_V1), hg.hg_build(k, 500, index=False)):
        with pytest.raises(hg.HGError) as e:
            t.erase(k[:10])
        assert e.value.status == hg.HG_ERR_INVALID_ARG


def test_erase_from_split_bins_and_key_runs(hg):
    """Three keys share 600000 entries: buckets of 200000 entries (key runs,
    bins split over workgroups).  Erasing one key leaves two long buckets
    that lost their key runs (scanned); probes, pairs and the export still
    match the oracle on what remains."""
    rng = np.random.default_rng(41)
    vals = np.array([7, 123456789, 4000000000], np.uint32)
    k = vals[rng.integers(0, 3, 600000)]
    V = 1000
    t = hg.hg_build(hg.to_device(k), V, seed=3)
    removed = t.erase(hg.to_device(vals[1:2]))
    live = k != vals[1]
    assert removed == int((~live).sum())
    off, ids, ek = export_np(hg, t, 32)
    e_off, e_ids, e_ek = remaining_table(oracle.build_table(k, V, 3), V, vals[1:2])
    assert np.array_equal(off, e_off) and np.array_equal(ids, e_ids) and np.array_equal(ek, e_ek)
    q = np.concatenate([vals, workloads.uniform_keys(50, 32, 5)]).astype(np.uint32)
    c, tot = hg.hg_probe(t, hg.to_device(q), counts=True, total=True)
    exp = oracle.probe_counts(k[live], q)[0]
    assert np.array_equal(hg.to_numpy(c, np.uint32), exp) and tot == int(exp.sum())
    q1 = np.array([vals[0], vals[2], vals[1]], np.uint32)
    b, p, ptot = hg.hg_probe_pairs(t, hg.to_device(q1))
    eb, ep, etot = oracle.probe_pairs(k[live], q1)
    assert ptot == etot
    # the oracle numbers build entries among the live keys: map back to ids
    live_ids = np.flatnonzero(live).astype(np.uint32)
    assert np.array_equal(hg.to_numpy(p, np.uint32), ep)
    assert np.array_equal(hg.to_numpy(b, np.uint32), live_ids[eb])
    t.free()


def test_erase_everything(hg):
    k = workloads.duplicate_keys(100000, 2.0, 32, seed=8)
    V = 50000
    t = hg.hg_build(hg.to_device(k), V, seed=1)
    assert t.erase(hg.to_device(np.unique(k))) == k.size
    assert t.live() == 0
    off, ids, ek = export_np(hg, t, 32)
    assert np.array_equal(off, np.zeros(V + 1, np.uint32)) and ids.size == 0 and ek.size == 0
    c, tot = hg.hg_probe(t, hg.to_device(k[:1000]), counts=True, total=True)
    assert tot == 0 and not hg.to_numpy(c, np.uint32).any()
    # erasing again (nothing left) removes nothing
    assert t.erase(hg.to_device(k[:10])) == 0
    t.free()
