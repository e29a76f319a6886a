"""Batched build + probe (one hipGraph launch) against the CPU oracle.

Every table of the batch must equal the oracle's stable table bit for bit and
its probe counts must equal the oracle's counts.  The captured graph is
replayed several times with eager library work and synchronisations in
between, and every replay is checked (the inputs are changed between replays
so that a stale replay cannot pass).
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


def make_tables(kb, seed, count=120):
    rng = np.random.default_rng(seed)
    sizes = list(np.floor(np.exp2(rng.uniform(0, 16, count))).astype(np.int64))
    # edge tables: empty, single key, V = 1, a one-bin table above the LDS
    # capacity (goes through the oversize-bin path), V >> n, duplicates, skew
    specials = [(0, 7), (1, 1), (5000, 1), (4000, 3), (3072, 3072), (3073, 4096), (300, 100000),
                (70000, 65536), (20000, 20000)]
    tabs = []
    for i, n in enumerate(sizes):
        tabs.append((int(n), max(1, int(n)), i))
    for j, (n, V) in enumerate(specials):
        tabs.append((n, V, 1000 + j))
    out = []
    for n, V, s in tabs:
        if s == 1000 + 6:
            k = workloads.duplicate_keys(n, 8.0, kb, seed=s)
        elif s == 1000 + 8:
            k = workloads.zipf_keys(n, 1.3, distinct=1 << 10, seed=s).astype(
                np.uint64 if kb == 64 else np.uint32)
        else:
            k = workloads.uniform_keys(n, kb, seed=s + 17 * seed)
        q = workloads.probe_queries(k if n else workloads.uniform_keys(3, kb, 1), max(n, 5), 0.5,
                                    seed=s + 3, key_bits=kb)
        out.append((k, q, V, s * 7 + 1))
    return out


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("autotune", [True, False])
def test_batch_matches_oracle_over_replays(hg, kb, autotune):
    print("[case] batch", kb, autotune, flush=True)
    data = make_tables(kb, seed=1)
    tabs = []
    for k, q, V, seed in data:
        tabs.append({"keys": hg.to_device(k), "queries": hg.to_device(q), "hash_range": V,
                     "seed": seed})
    b = hg.Batch(tabs, key_bits=kb, autotune=autotune)
    assert b.info()["bin_target"] in (1024, 2048)
    dt = np.uint64 if kb == 64 else np.uint32
    for rep in range(3):
        flip = dt((rep * 0x9E3779B1) & 0xFFFFFFFF)
        if rep:
            # new contents in the same buffers, plus unrelated eager work
            for (k, q, V, seed), t in zip(data, b.tables):
                if k.size:
                    k2 = (k ^ flip).astype(dt)
                    t["keys"].copy_(hg.to_device(k2))
            data = [(((k ^ flip).astype(dt) if k.size else k), q, V, s)
                    for (k, q, V, s) in data]
            e = hg.hg_build(hg.to_device(workloads.uniform_keys(5000, kb, rep)), 777)
            hg.hg_probe(e, hg.to_device(workloads.uniform_keys(100, kb, rep)))
            torch.cuda.synchronize()
        b.run()
        torch.cuda.synchronize()
        for (k, q, V, seed), t in zip(data, b.tables):
            n = k.size
            off = hg.to_numpy(t["offsets"], np.uint32)
            o_off, o_ids, o_ek = oracle.build_table(k, V, seed, kb)
            assert np.array_equal(off, o_off), (rep, n, V)
            assert np.array_equal(hg.to_numpy(t["ids"], np.uint32)[:n], o_ids), (rep, n, V)
            assert np.array_equal(hg.to_numpy(t["ekeys"], dt)[:n], o_ek), (rep, n, V)
            c = hg.to_numpy(t["counts"], np.uint32)[:q.size]
            assert np.array_equal(c, oracle.probe_counts(k, q, kb)[0]), (rep, n, V)
    b.free()


def test_batch_equals_per_table_loop(hg):
    data = make_tables(32, seed=5, count=60)
    tabs = [{"keys": hg.to_device(k), "queries": hg.to_device(q), "hash_range": V, "seed": s}
            for k, q, V, s in data]
    b = hg.Batch(tabs, key_bits=32, autotune=False, bin_target=1024)
    b.run()
    for (k, q, V, s), t in zip(data, b.tables):
        tb = hg.hg_build(t["keys"], V, seed=s)
        off, ids, ek = tb.export()
        c, _ = hg.hg_probe(tb, t["queries"])
        torch.cuda.synchronize()
        n = k.size
        assert torch.equal(off, t["offsets"])
        assert torch.equal(ids[:n], t["ids"][:n]) and torch.equal(ek[:n], t["ekeys"][:n])
        assert torch.equal(c, t["counts"][:q.size])


@pytest.mark.parametrize("kb", [32, 64])
def test_batch_any_order_matches_oracle_as_multisets(hg, kb):
    print("[case] batch any order", kb, flush=True)
    data = make_tables(kb, seed=3, count=80)
    tabs = [{"keys": hg.to_device(k), "queries": hg.to_device(q), "hash_range": V, "seed": s}
            for k, q, V, s in data]
    b = hg.Batch(tabs, key_bits=kb, autotune=False, any_order=True)
    dt = np.uint64 if kb == 64 else np.uint32
    for rep in range(2):
        b.run()
        torch.cuda.synchronize()
        for (k, q, V, seed), t in zip(data, b.tables):
            n = k.size
            off = hg.to_numpy(t["offsets"], np.uint32)
            ids = hg.to_numpy(t["ids"], np.uint32)[:n]
            ek = hg.to_numpy(t["ekeys"], dt)[:n]
            o_off, o_ids, _ = oracle.build_table(k, V, seed, kb)
            assert np.array_equal(off, o_off), (rep, n, V)
            seg = np.searchsorted(off.astype(np.int64), np.arange(n), side="right") - 1
            order = np.lexsort((ids, seg))
            assert np.array_equal(ids[order], o_ids), (rep, n, V)
            assert np.array_equal(ek, k[ids]), (rep, n, V)
            c = hg.to_numpy(t["counts"], np.uint32)[:q.size]
            assert np.array_equal(c, oracle.probe_counts(k, q, kb)[0]), (rep, n, V)
    b.free()


def test_batch_rejects_bad_items(hg):
    k = hg.to_device(workloads.uniform_keys(10, 32, 1))
    with pytest.raises(hg.HGError):
        hg.Batch([{"keys": k, "queries": None, "hash_range": 0, "seed": 0}])
