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
    # the tuner keeps the fastest candidate of each dimension: 1024, 2048 or
    # (32-bit keys) 4096 keys per bin, 8 or 16 keys per partition thread, one
    # of four probe shapes; without tuning the defaults are 2048, 16, 256x4
    info = b.info()
    if autotune:
        assert info["bin_target"] in ((1024, 2048, 4096) if kb == 32 else (1024, 2048))
        assert info["part_items"] in (8, 16)
        assert info["probe_shape"] in ((256, 4), (256, 8), (512, 2), (128, 8))
    else:
        assert (info["bin_target"], info["part_items"], info["probe_shape"]) == (2048, 16, (256, 4))
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


@pytest.fixture(scope="module")
def config_shape():
    """320 tables shaped like the benchmark's batch (sizes floor(2^U), U
    uniform in [8, 20], V = n, per-table seed, as many 50%-hit queries as
    keys), so that about a quarter of them hold 2^17 to 2^20 keys, plus the
    largest size itself; the oracle's stable table and counts of every one."""
    sizes = [int(x) for x in workloads.batched_sizes(320, 8.0, 20.0, seed=41)] + [1 << 20]
    data = []
    for i, n in enumerate(sizes):
        k = workloads.uniform_keys(n, 32, seed=50_000 + i)
        q = workloads.probe_queries(k, n, 0.5, seed=60_000 + i)
        off, ids, ek = oracle.build_table(k, n, i)
        data.append((k, q, n, i, off, ids, oracle.probe_counts(k, q)[0]))
    assert sum(1 for d in data if d[2] > (1 << 17)) >= 60
    return data


@pytest.mark.parametrize("any_order", [True, False])
@pytest.mark.parametrize("bin_target", [1024, 2048, 4096])
def test_batch_config_shape_every_bin_target(hg, config_shape, bin_target, any_order):
    """The batched configuration's table sizes (up to 2^20 keys, whose
    partition has up to 1024 digits) with each bin size the tuner can pick,
    in both layouts: offsets and counts equal the oracle's for every table;
    stable tables equal the oracle's table entry for entry, any-order tables
    as multisets per bucket (ids sorted inside each bucket)."""
    print("[case] batch config shape", bin_target, any_order, flush=True)
    tabs = [{"keys": hg.to_device(k), "queries": hg.to_device(q), "hash_range": V, "seed": s}
            for k, q, V, s, _, _, _ in config_shape]
    b = hg.Batch(tabs, key_bits=32, autotune=False, bin_target=bin_target, any_order=any_order)
    assert b.info()["bin_target"] == bin_target
    for rep in range(2):
        b.run()
        torch.cuda.synchronize()
        for (k, q, V, s, o_off, o_ids, o_cnt), t in zip(config_shape, b.tables):
            n = k.size
            off = t["offsets"].to(torch.int64) & 0xFFFFFFFF
            assert torch.equal(off, torch.from_numpy(o_off.astype(np.int64)).cuda()), (rep, n)
            ids = t["ids"][:n].to(torch.int64) & 0xFFFFFFFF
            ek = t["ekeys"][:n]
            assert torch.equal(ek, t["keys"][ids]), (rep, n)
            if any_order:
                seg = torch.repeat_interleave(torch.arange(V, device=ids.device),
                                              off[1:] - off[:-1], output_size=n)
                ids = ids[torch.argsort(seg * (1 << 32) + ids)]
            assert torch.equal(ids, torch.from_numpy(o_ids.astype(np.int64)).cuda()), (rep, n)
            c = t["counts"][:q.size].to(torch.int64) & 0xFFFFFFFF
            assert torch.equal(c, torch.from_numpy(o_cnt.astype(np.int64)).cuda()), (rep, n)
    b.free()


@pytest.mark.parametrize("part_items,probe_shape,any_order",
                         [(8, (256, 8), False), (8, (512, 2), True), (16, (128, 8), False),
                          (16, (256, 8), True), (8, (256, 4), False)])
def test_batch_config_shape_every_tile_shape(hg, config_shape, part_items, probe_shape, any_order):
    """The launch shapes the tuner can pick besides the bin target (keys per
    partition thread, probe workgroup shape) at the batched configuration's
    table sizes: offsets, counts and (stable) tables equal the oracle's."""
    print("[case] batch tile shape", part_items, probe_shape, any_order, flush=True)
    tabs = [{"keys": hg.to_device(k), "queries": hg.to_device(q), "hash_range": V, "seed": s}
            for k, q, V, s, _, _, _ in config_shape]
    b = hg.Batch(tabs, key_bits=32, autotune=False, bin_target=2048, any_order=any_order,
                 part_items=part_items, probe_shape=probe_shape)
    info = b.info()
    assert (info["part_items"], info["probe_shape"]) == (part_items, probe_shape)
    b.run()
    torch.cuda.synchronize()
    for (k, q, V, s, o_off, o_ids, o_cnt), t in zip(config_shape, b.tables):
        n = k.size
        off = t["offsets"].to(torch.int64) & 0xFFFFFFFF
        assert torch.equal(off, torch.from_numpy(o_off.astype(np.int64)).cuda()), n
        ids = t["ids"][:n].to(torch.int64) & 0xFFFFFFFF
        assert torch.equal(t["ekeys"][:n], t["keys"][ids]), n
        if any_order:
            seg = torch.repeat_interleave(torch.arange(V, device=ids.device),
                                          off[1:] - off[:-1], output_size=n)
            ids = ids[torch.argsort(seg * (1 << 32) + ids)]
        assert torch.equal(ids, torch.from_numpy(o_ids.astype(np.int64)).cuda()), n
        c = t["counts"][:q.size].to(torch.int64) & 0xFFFFFFFF
        assert torch.equal(c, torch.from_numpy(o_cnt.astype(np.int64)).cuda()), n
    # the reported configuration plans the same graph again, without tuning
    b2 = hg.Batch(tabs, key_bits=32, autotune=True, bin_target=info["bin_target"],
                  any_order=any_order, part_items=info["part_items"],
                  probe_shape=info["probe_shape"])
    assert b2.info() == info
    b2.free()
    b.free()
