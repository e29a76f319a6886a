"""Indexed builds are asynchronous: a table made by hg_table_create is rebuilt
(with the probe index and the key runs of long buckets) and probed inside a
captured HIP graph, with no allocation and no host wait in either call.

The graph is replayed several times; before each replay the key buffer gets
new contents and unrelated eager library work runs, and after each replay the
table (offsets exact, buckets as the oracle's stable table, or as multisets
for any order) and the probe counts are compared with the oracle's for the
keys the replay saw."""
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


def make_keys(kind, n, kb, seed):
    if kind == "uniform":
        return workloads.uniform_keys(n, kb, seed)
    if kind == "dup30":  # long buckets of a few keys each
        return workloads.duplicate_keys(n, 30.0, kb, seed)
    if kind == "zipf":  # bins too large for LDS, long buckets of many keys
        return workloads.zipf_keys(n, 1.3, distinct=1 << 12, seed=seed).astype(dt(kb))
    raise ValueError(kind)


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("kind,n,V,any_order", [("uniform", 300007, 300007, True),
                                                ("dup30", 250000, 250000 // 60, False),
                                                ("zipf", 200000, 200000, True),
                                                ("zipf", 150000, 3000, False)])
def test_indexed_build_and_probe_replay_from_a_graph(hg, kb, kind, n, V, any_order):
    print("[case] graph build+probe", kb, kind, n, V, any_order, flush=True)
    keys = make_keys(kind, n, kb, seed=3)
    q = workloads.probe_queries(keys, n, 0.5, seed=4, key_bits=kb)
    dk, dq = hg.to_device(keys), hg.to_device(q)
    t = hg.Table.create(n, V, kb)
    counts = torch.empty(n, dtype=torch.int32, device="cuda")
    # eager first (sets the kernels' LDS limits once per device)
    t.rebuild(dk, V, seed=11, any_order=any_order)
    hg.hg_probe(t, dq, counts=True, out=counts)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        t.rebuild(dk, V, seed=11, any_order=any_order)
        hg.hg_probe(t, dq, counts=True, out=counts)
    flip = dt(kb)(0x9E3779B1)
    for rep in range(3):
        if rep:
            keys = (keys ^ flip).astype(dt(kb))  # same duplicate structure, new keys
            q = (q ^ flip).astype(dt(kb))
            dk.copy_(hg.to_device(keys))
            dq.copy_(hg.to_device(q))
            other = hg.hg_build(hg.to_device(workloads.uniform_keys(7000, kb, rep)), 999)
            hg.hg_probe(other, hg.to_device(workloads.uniform_keys(500, kb, rep)))
            torch.cuda.synchronize()
            other.free()
        counts.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        exp, _ = oracle.probe_counts(keys, q, kb)
        assert np.array_equal(hg.to_numpy(counts, np.uint32), exp), rep
        off, ids, ek = t.export()
        torch.cuda.synchronize()
        o_off, o_ids, _ = oracle.build_table(keys, V, 11, kb)
        off, ids, ek = hg.to_numpy(off, np.uint32), hg.to_numpy(ids, np.uint32), hg.to_numpy(ek, dt(kb))
        assert np.array_equal(off, o_off), rep
        assert np.array_equal(ek, keys[ids]), rep
        if any_order:
            seg = np.repeat(np.arange(V), np.diff(off.astype(np.int64)))
            ids = ids[np.lexsort((ids, seg))]
        assert np.array_equal(ids, o_ids), rep
    # the index the graph wrote serves the pairs too
    light = np.nonzero(exp <= 50)[0][:5000]
    b, p, tot = hg.hg_probe_pairs(t, hg.to_device(q[light]))
    eb, ep, et = oracle.probe_pairs(keys, q[light], kb)
    b, p = hg.to_numpy(b, np.uint32)[:et], hg.to_numpy(p, np.uint32)[:et]
    o = np.lexsort((b, p))
    assert tot == et and np.array_equal(p[o], ep) and np.array_equal(b[o], eb)
    del g
    t.free()


def test_table_dropped_during_capture_is_freed_after(hg):
    # a table whose last reference goes away inside a torch.cuda.graph block
    # (as when the garbage collector runs there) is not freed during the
    # capture: freeing device memory would invalidate it
    n = 50000
    keys = workloads.uniform_keys(n, 32, seed=81)
    q = workloads.probe_queries(keys, n, 0.5, seed=82)
    dk, dq = hg.to_device(keys), hg.to_device(q)
    t = hg.Table.create(n, n, 32)
    counts = torch.empty(n, dtype=torch.int32, device="cuda")
    t.rebuild(dk, n, seed=5)
    hg.hg_probe(t, dq, counts=True, out=counts)
    doomed = hg.hg_build(hg.to_device(workloads.uniform_keys(1000, 32, seed=83)), 1000)
    torch.cuda.synchronize()
    before = len(hg._deferred)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        t.rebuild(dk, n, seed=5)
        del doomed
        hg.hg_probe(t, dq, counts=True, out=counts)
    assert len(hg._deferred) == before + 1
    counts.fill_(-1)
    g.replay()
    torch.cuda.synchronize()
    assert np.array_equal(hg.to_numpy(counts, np.uint32), oracle.probe_counts(keys, q)[0])
    hg.flush_deferred_releases()
    assert not hg._deferred
    t.free()
