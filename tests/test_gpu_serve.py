"""Serving loop: every result is the same alone and in the mix.

A fixed list of build and probe requests is run twice: once alone (one
request in flight, no merging: submit, wait, next) and once as a mix (all
submitted back to back with Poisson-like pauses, four streams, merging on).
Tables (offsets, ids, keys) and probe counts must be bit-identical between
the two runs and equal to the CPU oracle.  Further tests cover eviction under
a small memory budget, pinning of tables with pending probes, and the error
paths.
"""
import time

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


def make_requests(seed=3, nbuild=24, nprobe=56):
    rng = np.random.default_rng(seed)
    builds = []
    for b in range(nbuild):
        n = int(np.floor(np.exp2(rng.uniform(8, 17))))
        k = workloads.uniform_keys(n, 32, seed=100 + b)
        builds.append((k, max(1, n), 1000 + b))
    reqs = [("build", b) for b in range(nbuild)]
    for p in range(nprobe):
        b = int(rng.integers(0, nbuild))
        m = int(np.floor(np.exp2(rng.uniform(6, 15))))
        q = workloads.probe_queries(builds[b][0], m, 0.5, seed=500 + p)
        first = reqs.index(("build", b)) + 1  # after its build
        pos = int(rng.integers(first, len(reqs) + 1))
        reqs.insert(pos, ("probe", (b, q)))
    return builds, reqs


def run(hg, builds, reqs, alone, workers=0):
    if alone:
        srv = hg.Server(streams=1, max_inflight=1, merge_max=1)
    else:
        srv = hg.Server(streams=8 if workers > 2 else 4, max_inflight=16, merge_max=64,
                        merge_keys=1 << 16, workers=workers)
    dk = [hg.to_device(k) for k, _, _ in builds]
    tids, counts, qs = {}, [], []
    rng = np.random.default_rng(9)
    for kind, arg in reqs:
        if kind == "build":
            k, V, seed = builds[arg]
            tid, rid = srv.submit_build(dk[arg], V, seed)
            tids[arg] = tid
        else:
            b, q = arg
            dq = hg.to_device(q)
            rid, c = srv.submit_probe(tids[b], dq)
            counts.append(c)
            qs.append((b, q))
        if alone:
            assert srv.wait(rid) == hg.HG_OK
        elif rng.random() < 0.2:
            time.sleep(rng.exponential(0.0005))
    srv.drain()
    torch.cuda.synchronize()
    tables = {}
    for b, tid in tids.items():
        ex = srv.export(tid)
        assert ex is not None
        tables[b] = tuple(hg.to_numpy(x, np.uint32) for x in ex)
    cnts = [hg.to_numpy(c[:q.size], np.uint32) for c, (b, q) in zip(counts, qs)]
    st = srv.stats()
    srv.close()
    return tables, cnts, qs, st


@pytest.mark.parametrize("workers", [1, 2, 4])
def test_results_same_alone_and_in_mix(hg, workers):
    # the mix runs with one, two or four threads launching device work
    builds, reqs = make_requests()
    print("[case] serve alone", flush=True)
    t_alone, c_alone, qs, st_alone = run(hg, builds, reqs, alone=True)
    print("[case] serve mix, workers", workers, flush=True)
    t_mix, c_mix, _, st_mix = run(hg, builds, reqs, alone=False, workers=workers)
    assert st_alone["merged_requests"] == 0
    assert st_mix["completed"] == len(reqs) and st_mix["failed"] == 0
    for b in t_alone:
        for x, y in zip(t_alone[b], t_mix[b]):
            assert np.array_equal(x, y), b
        k, V, seed = builds[b]
        o = oracle.build_table(k, V, seed)
        assert np.array_equal(t_alone[b][0], o[0]) and np.array_equal(t_alone[b][1], o[1])
        assert np.array_equal(t_alone[b][2], o[2])
    for x, y, (b, q) in zip(c_alone, c_mix, qs):
        assert np.array_equal(x, y)
        assert np.array_equal(x, oracle.probe_counts(builds[b][0], q)[0])
    assert st_mix["p50_ms"] <= st_mix["p99_ms"] <= st_mix["max_ms"]


def test_budget_eviction_and_pinning(hg):
    # each table: 40000 keys, V = 40000 -> about 480 KB; budget fits ~4
    srv = hg.Server(budget_bytes=2_000_000, streams=2, max_inflight=4)
    keys = [hg.to_device(workloads.uniform_keys(40000, 32, seed=i)) for i in range(10)]
    tids = []
    for i, k in enumerate(keys):
        tid, rid = srv.submit_build(k, 40000, i)
        assert srv.wait(rid) == hg.HG_OK
        tids.append(tid)
    st = srv.stats()
    assert st["evictions"] >= 5 and st["peak_bytes"] <= 2_000_000
    # the oldest tables are gone, the newest resident
    assert srv.export(tids[0]) is None
    assert srv.export(tids[-1]) is not None
    with pytest.raises(hg.HGError) as e:
        srv.submit_probe(tids[0], keys[0][:10])
    assert e.value.status == hg.HG_ERR_NOT_FOUND
    # a probe pins its table: queue many builds behind it, the table survives
    # until the probe completes and its counts are right
    q = keys[-1][:1000]
    rid, c = srv.submit_probe(tids[-1], q)
    for i in range(3):
        srv.submit_build(keys[i], 40000, 77 + i)
    assert srv.wait(rid) == hg.HG_OK
    exp = oracle.probe_counts(hg.to_numpy(keys[-1], np.uint32),
                              hg.to_numpy(q, np.uint32))[0]
    assert np.array_equal(hg.to_numpy(c[:1000], np.uint32), exp)
    # a table larger than the whole budget is rejected
    big = hg.to_device(workloads.uniform_keys(300000, 32, 5))
    tid, rid = srv.submit_build(big, 300000, 1)
    assert srv.wait(rid) == hg.HG_ERR_BUDGET
    srv.drain()
    assert srv.stats()["rejected"] >= 1
    srv.close()


def test_server_options_validated(hg):
    for kw in ({"streams": 2, "workers": 3}, {"workers": 9, "streams": 16}, {"streams": 17}):
        with pytest.raises(hg.HGError) as e:
            hg.Server(**kw)
        assert e.value.status == hg.HG_ERR_INVALID_ARG


def test_request_records_released(hg):
    # one stream, one launch in flight: requests complete in submission order
    srv = hg.Server(streams=1, max_inflight=1, merge_max=1)
    k_np = workloads.uniform_keys(30000, 32, seed=21)
    q_np = workloads.probe_queries(k_np, 5000, 0.5, seed=22)
    dk, dq = hg.to_device(k_np), hg.to_device(q_np)
    tid, _ = srv.submit_build(dk, 30000, 4, want_id=False)
    outs = [srv.submit_probe(tid, dq, want_id=False)[1] for _ in range(3)]
    rid, c = srv.submit_probe(tid, dq)
    assert srv.wait(rid) == hg.HG_OK
    # the id-less requests left no record; the waited one was released
    assert srv.stats()["held_requests"] == 0
    with pytest.raises(hg.HGError) as e:
        srv.wait(rid)
    assert e.value.status == hg.HG_ERR_NOT_FOUND
    exp = oracle.probe_counts(k_np, q_np)[0]
    for x in outs + [c]:
        assert np.array_equal(hg.to_numpy(x[:q_np.size], np.uint32), exp)
    # records with ids are kept until drain releases them
    rids = [srv.submit_probe(tid, dq)[0] for _ in range(4)]
    srv.drain()
    assert srv.stats()["held_requests"] == 0
    with pytest.raises(hg.HGError) as e:
        srv.wait(rids[0])
    assert e.value.status == hg.HG_ERR_NOT_FOUND
    st = srv.stats()
    assert st["completed"] == 9 and st["failed"] == 0
    srv.close()


def test_failed_build_releases_its_table(hg):
    # a build larger than the budget fails; its table is forgotten, probes
    # queued behind it fail, and the budget accounting is unchanged
    srv = hg.Server(budget_bytes=4_000_000, streams=1, max_inflight=1, merge_max=1)
    small = hg.to_device(workloads.uniform_keys(20000, 32, seed=31))
    tid_ok, rid = srv.submit_build(small, 20000, 1)
    assert srv.wait(rid) == hg.HG_OK
    before = srv.stats()["resident_bytes"]
    big = hg.to_device(workloads.uniform_keys(500000, 32, seed=32))  # about 20 MB
    tid_big, rid_big = srv.submit_build(big, 500000, 2)
    try:
        rid_p, _ = srv.submit_probe(tid_big, big[:100])
    except hg.HGError as e:  # the build was already rejected
        assert e.status == hg.HG_ERR_NOT_FOUND
        rid_p = None
    assert srv.wait(rid_big) == hg.HG_ERR_BUDGET
    if rid_p is not None:
        assert srv.wait(rid_p) == hg.HG_ERR_NOT_FOUND
    with pytest.raises(hg.HGError) as e:
        srv.submit_probe(tid_big, big[:100])
    assert e.value.status == hg.HG_ERR_NOT_FOUND
    st = srv.stats()
    assert st["resident_bytes"] == before and st["resident_tables"] == 1
    assert srv.export(tid_ok) is not None and srv.export(tid_big) is None
    srv.close()
