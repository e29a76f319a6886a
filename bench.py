#!/usr/bin/env python3
"""Benchmark of the HashGraph hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu-baseline]

One step = one pass of the hot path over one batch: a V2 HashGraph build of
n = 2^28 uniform uint32 keys with hash_range V = 2^28 (load 1), followed by
HashGraph-Probe-Standard of m = 2^28 queries (half drawn from the keys), with
per-query match counts written to device memory.  Inputs are resident in HBM
before the timed region; the table and workspace are preallocated, so nothing
is allocated while timing.  value = (n + m) / step time, in G keys/s.

The JSON line also carries:
  roofline      the dominant kernel's algorithmic bytes per launch (the
                method's own passes; for the probe its compulsory bytes:
                query, two offsets, the bucket's keys, the count) divided by
                its average launch time (HIP events around each launch, on the
                stream the library launches on), against 8 TB/s;
  cpu_baseline  the CPU oracle on this host's cores: its multi-core variant
                on the step's own arrays, and the sequential oracle on a
                bounded sample;
  phases        per-kernel times, the V1 build, the hash-range sweep
                {2^26, 2^28, 2^30}, the 64-bit-key variant and Probe-New.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "build & probe Gkeys/s + % HBM peak at 2^28 uint32 keys; batched/served p99"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# sources of the kernels the timed step launches (build, index, probe, scans)
STEP_KERNEL_SOURCES = ("hg_device.h", "hg_internal.h", "hg_v2_device.h", "hg_v2.hip",
                       "hg_probe.hip", "hg_scan.hip", "hg_runs.hip")


def src_digest() -> str:
    """Digest of the step's kernel sources: HBM counters stored with another
    digest were taken on other kernels and are not reported."""
    h = hashlib.sha256()
    for name in STEP_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1907_02900_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def micro_roofline(hg):
    """Random-transaction rates (G accesses/s) over L2-, MALL- and HBM-sized
    footprints: 4-byte and 16-byte reads and 4-byte atomic adds."""
    out = {}
    for label, fp in (("4MiB", 1 << 22), ("128MiB", 1 << 27), ("4GiB", 1 << 32)):
        out[label] = {
            "read4_G_per_s": round(hg.random_access_rate(hg.MICRO_READ4, fp, 1 << 27) / 1e9, 2),
            "read16_G_per_s": round(hg.random_access_rate(hg.MICRO_READ16, fp, 1 << 27) / 1e9, 2),
            "atomic4_G_per_s": round(hg.random_access_rate(hg.MICRO_ATOMIC4, fp, 1 << 26) / 1e9,
                                     2)}
    return out


def timed(fn, reps, torch):
    """Median milliseconds of `reps` runs of fn() (events on the current stream)."""
    out = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        out.append(e0.elapsed_time(e1))
    return float(np.median(out))


def kernel_bytes(name, n, m, V, kb, sum_len, plan):
    """Algorithmic bytes one launch of `name` must move (reads + writes), by
    the method's own passes (Sec. 3.3 phases; the probe's compulsory bytes):

      probe_count     a query reads its key, the two offsets of its bucket and
                      every key of the bucket, and writes its count:
                      m*kb + 8m + kb*sum(|bucket|) + 4m (about 22 B per query
                      at load 1 with 50% hits);
      v2_local_build  phase 3 reads and writes every (key, id) and writes the
                      offsets: 2n(kb+4) + 4(V+1);
      v2_partition_*  phase 2: the first pass reads keys and writes (key, id),
                      a second pass reads and writes (key, id); plus the
                      tile x digit bases it reads;
      v2_tile_hist_*  phase 1: reads the keys, writes the tile histograms.

    When the probe first groups its queries by bucket range (hg_probe does at
    this size), three passes of the same kind as the build's come with it:

      probe_group_hist  reads the queries, writes their tile histograms;
      probe_group       reads the queries and the tile bases, writes the
                        queries and their input positions in grouped order;
      probe_ungroup     reads positions and counts in grouped order and two
                        rows of bases per four tiles, writes the counts.

    The per-bucket probe index is this design's addition and is not counted
    here (index_bytes gives the bytes with it)."""
    gm = group_matrix_bytes(m, V)
    if name == "probe_count":
        return m * kb + 8 * m + kb * sum_len + 4 * m
    if name == "probe_group_hist":
        return m * kb + gm
    if name == "probe_group":
        return m * kb + gm + m * kb + 4 * m
    if name == "probe_ungroup":
        return 4 * m + 4 * m + 4 * m + gm // 2
    if name == "v2_local_build":
        return 2 * n * (kb + 4) + (V + 1) * 4
    if name == "v2_partition_t1":
        return n * kb + n * (kb + 4) + plan["m1_bytes"]
    if name == "v2_partition_t2":
        return 2 * n * (kb + 4) + plan["m2_bytes"]
    if name == "v2_tile_hist_t1":
        return n * kb + plan["m1_bytes"]
    if name == "v2_tile_hist_t2":
        return n * kb + plan["m2_bytes"]
    return None


def group_matrix_bytes(m, V):
    """Tile x range matrix of the probe's query grouping: 4096 queries per
    tile, 2^min(9, ceil(log2 V)) ranges (at least 2), 4 bytes each."""
    kv = max(int(V - 1).bit_length(), 0)
    bits = 9 if kv >= 9 else max(kv, 1)
    return -(-m // 4096) * (1 << bits) * 4


def index_bytes(name, n, m, V, kb, sum_tail):
    """Bytes the kernels move with the per-bucket probe index: the probe reads
    one 16-byte entry per query and only the keys the entry does not account
    for (sum_tail); the per-bin build also writes 16 bytes per bucket."""
    if name == "probe_count":
        return m * kb + m * 16 + kb * sum_tail + m * 4
    if name == "v2_local_build":
        return 2 * n * (kb + 4) + (V + 1) * 4 + V * 16
    return None


def v2_plan_bytes(hg, n, V, kb=4):
    """Tile x digit matrix bytes of each partition pass, from the library's
    own plan (hg_build_plan)."""
    p = hg.build_plan(n, V, 8 * kb)
    m1 = p["tiles"][0] * (1 << p["digit_bits"][0]) * 4
    m2 = p["tiles"][1] * (1 << p["digit_bits"][1]) * 4 if p["passes"] == 2 else 0
    return {"m1_bytes": m1, "m2_bytes": m2, "plan": p}


def load_traffic(kernel, digest):
    """Measured HBM bytes per launch from profiles/pmc_traffic.json, if it was
    taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        with open(p) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get("kernels", {}).get(kernel)
    if not e or d.get("source_digest") != digest:
        return None
    return e.get("hbm_bytes_per_launch")


def run_batched(hg, workloads, torch, tables=4096, reps=5, log=print, any_order=True):
    """4096 tables, sizes floor(2^U), U ~ U[8, 20], V = n, m = n queries with
    50% hits: one graph launch per run vs a per-table loop of hg_table_build
    + hg_probe into preallocated tables."""
    sizes = workloads.batched_sizes(tables, 8.0, 20.0, seed=7)
    keys, qs = [], []
    for i, n in enumerate(sizes):
        k = workloads.uniform_keys(int(n), 32, seed=10_000 + i)
        keys.append(hg.to_device(k))
        qs.append(hg.to_device(workloads.probe_queries(k, int(n), 0.5, seed=20_000 + i)))
    tot = int(sizes.sum()) * 2
    t0 = time.perf_counter()
    b = hg.Batch([{"keys": keys[i], "queries": qs[i], "hash_range": int(sizes[i]),
                   "seed": i} for i in range(tables)], key_bits=32, autotune=True,
                 any_order=any_order)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    t_graph = timed(b.run, reps, torch)
    # per-table loop of the plain entry points, tables preallocated
    loop_tabs = [hg.Table.create(int(n), int(n), 32) for n in sizes]
    outs = [t["counts"] for t in b.tables]

    def loop():
        # the same work as the graph: V2 tables without the probe index
        for i in range(tables):
            loop_tabs[i].rebuild(keys[i], int(sizes[i]), seed=i, index=False,
                                 any_order=any_order)
            hg.hg_probe(loop_tabs[i], qs[i], counts=True, out=outs[i])

    t_loop = timed(loop, 2, torch)
    info = b.info()
    for t in loop_tabs:
        t.free()
    b.free()
    log("batched: graph %.3f ms, loop %.3f ms" % (t_graph, t_loop))
    return {"tables": tables, "keys_plus_queries": tot, "graph_ms": round(t_graph, 3),
            "graph_Gkeys": round(tot / t_graph / 1e6, 2), "loop_ms": round(t_loop, 3),
            "loop_Gkeys": round(tot / t_loop / 1e6, 2), "speedup": round(t_loop / t_graph, 2),
            "bin_target": info["bin_target"], "part_items": info["part_items"],
            "probe_shape": list(info["probe_shape"]), "plan_create_s": round(create_s, 2)}


SERVING_RATES = (2e3, 5e3, 1e4, 1.5e4, 2e4, 3e4, 5e4, 1e6)


def run_serving(hg, workloads, torch, requests=2000, rates=SERVING_RATES, log=print):
    """Poisson stream, 30% builds (n log-uniform in [2^10, 2^24]) and 70%
    probes (m log-uniform in [2^10, 2^22]) against resident tables, 64 GB
    budget; the arrival rate is swept from well below to beyond saturation,
    `requests` requests per rate; the server runs 4 launching threads over 8
    streams with up to 32 launches in flight.  Keys come from one device pool of uniform
    keys; a probe takes half its queries from its table's key range (hits) and
    half from elsewhere.  The baseline is a sequential loop of the plain
    entry points over the saturated stream, doing the same work the server
    does: tables preallocated before the clock (a ring of 64 tables of the
    largest size, so nothing is allocated or synchronised per request),
    stable V2 builds with the probe index, counts into preallocated outputs."""
    pool_n = 1 << 26
    pool = hg.to_device(workloads.uniform_keys(pool_n, 32, seed=99))
    qpool = hg.to_device(workloads.uniform_keys(pool_n, 32, seed=98))
    rng = np.random.default_rng(5)

    def build_slice(n):
        o = int(rng.integers(0, pool_n - n))
        return pool[o:o + n], o

    out = {"rates": [], "requests_per_rate": requests}
    srv = hg.Server(budget_bytes=64 << 30, streams=8, max_inflight=32, workers=4)
    tables = []
    for _ in range(64):  # warm-up: resident tables
        n = int(np.exp2(rng.uniform(10, 24)))
        k, o = build_slice(n)
        tid, _ = srv.submit_build(k, n, seed=len(tables))
        tables.append((tid, o, n))
    srv.drain()

    def make_plan(nreq, rate, seed):
        # every input is made (and finished) before the clock starts: probe
        # queries, half from the target table's keys and half from elsewhere
        arr, isb, size, _ = workloads.serving_stream(nreq, rate, seed=seed)
        plan, qs = [], []
        for b_, s in zip(isb, size):
            s = int(s)
            if b_:
                plan.append(("b",) + build_slice(s) + (s,))
            else:
                j = int(rng.integers(0, 64))
                tid, o, n = tables[j]
                half = min(s // 2, n)
                q = torch.cat([pool[o:o + half], qpool[:s - half]])
                plan.append(("p", j, q))
                qs.append(s)
        outc = torch.empty(max(sum(qs), 1), dtype=torch.int32, device="cuda")
        return arr, plan, outc

    def one_run(rate, nreq, seed):
        arr, plan, outc = make_plan(nreq, rate, seed)
        torch.cuda.synchronize()
        srv.reset_stats()
        t0 = time.perf_counter()
        mo = 0
        for a, item in zip(arr, plan):
            while time.perf_counter() - t0 < a:
                pass
            if item[0] == "b":
                _, k, o, s = item
                srv.submit_build(k, s, seed=s)
            else:
                _, j, q = item
                srv.submit_probe(tables[j][0], q, outc[mo:mo + q.numel()])
                mo += q.numel()
        srv.drain()
        wall = time.perf_counter() - t0
        st = srv.stats()
        return {"rate_per_s": rate, "requests": nreq,
                "achieved_rate_per_s": round(nreq / wall, 1),
                "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                "Gkeys": round(st["keys"] / max(st["busy_s"], 1e-9) / 1e9, 2),
                "merged_requests": st["merged_requests"], "launches": st["launches"],
                "evictions": st["evictions"], "failed": st["failed"]}

    for rate in rates:
        r = one_run(rate, requests, seed=int(rate) % 1000 + 1)
        out["rates"].append(r)
        log("serving rate %g: p50 %.3f ms p99 %.3f ms %.2f Gkeys/s (%.0f req/s)" % (
            rate, r["p50_ms"], r["p99_ms"], r["Gkeys"], r["achieved_rate_per_s"]))
    srv.close()
    # the knee: the first offered rate the server no longer keeps up with
    # (achieved below 90% of offered) or whose p99 is over twice the p99 at
    # the lowest rate
    base = out["rates"][0]["p99_ms"]
    knee = None
    for r in out["rates"]:
        if r["achieved_rate_per_s"] < 0.9 * r["rate_per_s"] or r["p99_ms"] > 2.0 * base:
            knee = r["rate_per_s"]
            break
    out["knee_rate_per_s"] = knee
    out["saturation_Gkeys"] = out["rates"][-1]["Gkeys"]

    # the sequential loop over the saturated stream
    ring = [hg.Table.create(1 << 24, 1 << 24, 32) for _ in range(64)]
    for i, (tid, o, n) in enumerate(tables[:64]):
        ring[i].rebuild(pool[o:o + n], n, seed=i)
    arr, plan, outc = make_plan(requests, rates[-1], seed=int(rates[-1]) % 1000 + 1)
    torch.cuda.synchronize()
    nxt, keys_done, mo = 0, 0, 0
    t0 = time.perf_counter()
    for item in plan:
        if item[0] == "b":
            _, k, o, s = item
            ring[nxt].rebuild(k, s, seed=s)
            nxt = (nxt + 1) % len(ring)
            keys_done += s
        else:
            _, j, q = item
            hg.hg_probe(ring[j], q, counts=True, out=outc[mo:mo + q.numel()])
            mo += q.numel()
            keys_done += q.numel()
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    for t in ring:
        t.free()
    out["loop_Gkeys"] = round(keys_done / t_loop / 1e9, 2)
    out["loop"] = ("sequential hg_table_build (stable, probe index) + hg_probe over %d "
                   "requests of the saturated stream, 64 preallocated 2^24-key tables"
                   % requests)
    out["speedup_at_saturation"] = round(out["saturation_Gkeys"] / max(out["loop_Gkeys"], 1e-9), 2)
    log("serving loop %.2f Gkeys/s; knee %s req/s" % (out["loop_Gkeys"], knee))
    return out


def copy_gbps(torch, nbytes=1 << 30, reps=5):
    """Achievable stream bandwidth: an elementwise kernel reading and writing
    1 GiB each (read + write bytes over its time; a plain tensor copy goes to
    the copy engines, which are slower)."""
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    t = timed(lambda: torch.bitwise_xor(src, 1, out=dst), reps, torch)
    del src, dst
    return 2 * nbytes / (t / 1000.0) / 1e9


def hbm_fractions(build_ms, probe_ms, n, m, V, kb, sum_len, digest, copy, grouped=False):
    """Per phase of the step: HBM bytes the counters saw (profiles/
    pmc_traffic.json, same kernel sources) over the phase time, against the
    8 TB/s peak and the measured copy bandwidth; and the compulsory bytes
    (build: read keys, write keys + ids + offsets; probe: read the query, two
    offsets and its bucket's keys, write the count) over the same time."""
    tr = {k: load_traffic(k, digest) for k in ("v2_tile_hist", "v2_partition_t1",
                                               "v2_partition_t2", "v2_local_build",
                                               "probe_count")}
    grp = {k: load_traffic(k, digest) for k in ("probe_group_hist", "probe_group",
                                                "probe_ungroup")}
    b_min = {"build": n * kb + n * (kb + 4) + 4 * (V + 1),
             "probe": m * kb + 8 * m + kb * sum_len + 4 * m}
    ms = {"build": build_ms, "probe": probe_ms}
    meas = None
    if all(tr.values()) and (not grouped or all(grp.values())):
        meas = {"build": 2 * tr["v2_tile_hist"] + tr["v2_partition_t1"] +
                tr["v2_partition_t2"] + tr["v2_local_build"],
                "probe": tr["probe_count"] + (sum(grp.values()) if grouped else 0)}
    out = {"peak_GBps": HBM_PEAK_GBS, "copy_GBps": round(copy, 1)}
    for ph in ("build", "probe"):
        t = ms[ph] / 1000.0
        e = {"ms": round(ms[ph], 3), "compulsory_bytes": b_min[ph],
             "compulsory_pct_peak": round(100 * b_min[ph] / t / 1e9 / HBM_PEAK_GBS, 1)}
        if meas:
            g = meas[ph] / t / 1e9
            e.update({"hbm_bytes": int(meas[ph]), "hbm_GBps": round(g, 1),
                      "hbm_pct_peak": round(100 * g / HBM_PEAK_GBS, 1),
                      "hbm_pct_copy": round(100 * g / copy, 1)})
        out[ph] = e
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(keys, queries, V, log2_sample=24):
    """The CPU oracle on this host: its multi-core variant (OpenMP, the same
    definitions, bit-identical output) on the step's own arrays -- the stable
    build of all keys, then the counts of all queries -- and the sequential
    oracle on a bounded sample of the same workload."""
    import oracle
    from paper_1907_02900_amd import workloads
    n, m = keys.size, queries.size
    threads = oracle.omp_threads()
    times = []
    for _ in range(2):
        t0 = time.perf_counter()
        oracle.build_table_omp(keys, V, 0)
        oracle.probe_counts_omp(keys, queries)
        times.append(time.perf_counter() - t0)
    t = float(np.min(times))
    ns = 1 << log2_sample
    sk = workloads.uniform_keys(ns, 32, seed=0)
    sq = workloads.probe_queries(sk, ns, 0.5, seed=1)
    seq = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.build_table(sk, ns, 0)
        oracle.probe_counts(sk, sq)
        seq.append(time.perf_counter() - t0)
    ts = float(np.median(seq))
    return {"value": round((n + m) / t / 1e9, 5), "unit": "Gkeys/s", "cores": threads,
            "kind": "oracle",
            "host": {"nproc": os.cpu_count(), "model": cpu_model()},
            "sample": "the step's own arrays: stable build of %d uniform uint32 keys, hash_range "
                      "%d, then probe counts of %d queries (50%% hits), by the oracle's "
                      "multi-core variant (OpenMP, %d threads, output identical to the "
                      "sequential oracle), best of 2 (%.2f s)" % (n, V, m, threads, t),
            "sequential": {"value": round(2 * ns / ts / 1e9, 5), "unit": "Gkeys/s", "cores": 1,
                           "sample": "2^%d uniform uint32 keys, hash_range 2^%d, + 2^%d "
                                     "queries: sequential oracle, median of 3 (%.2f s)"
                                     % (log2_sample, log2_sample, log2_sample, ts)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--log2range", type=int, default=28)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--tables", type=int, default=4096)
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--stable", action="store_true",
                    help="time the stable (ids ascending in each bucket) V2 layout")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device-to-device (reference for HBM counters)")
    ap.add_argument("--random-calibration", action="store_true",
                    help="only run the random 16-byte read micro-benchmark over 4 GiB "
                         "(2 launches of 2^27 reads; reference for HBM counters)")
    args = ap.parse_args()
    if args.random_calibration:
        from paper_1907_02900_amd import hg
        rate = hg.random_access_rate(hg.MICRO_READ16, 1 << 32, 1 << 27)
        print(json.dumps({"footprint_bytes": 1 << 32, "reads_per_launch": 1 << 27,
                          "launches": 2, "read16_G_per_s": round(rate / 1e9, 2)}))
        return
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30, "launches": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1907_02900_amd import hg, workloads

    torch.cuda.set_device(0)
    n = 1 << args.log2n
    V = 1 << args.log2range
    m = n
    kb = 4
    log("generating %d keys / %d queries" % (n, m))
    keys_np = workloads.uniform_keys(n, 32, seed=0)
    q_np = workloads.probe_queries(keys_np, m, 0.5, seed=1)
    dk = hg.to_device(keys_np)
    dq = hg.to_device(q_np)
    counts = torch.empty(m, dtype=torch.int32, device="cuda")
    table = hg.Table.create(n, V, 32)
    torch.cuda.synchronize()

    def step():
        table.rebuild(dk, V, seed=0, variant=hg.VARIANT_V2, any_order=not args.stable)
        hg.hg_probe(table, dq, counts=True, total=False, out=counts)

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    hg.profile_reset()
    hg.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    hg.profile_enable(False)
    prof = hg.profile_report()
    hg.profile_reset()
    ms_step = wall * 1000.0 / args.steps
    # the event-instrumented run above also gives the step time; time the
    # same steps once more without instrumentation for the headline value
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall2 = time.perf_counter() - t0
    ms_step = min(ms_step, wall2 * 1000.0 / args.steps)
    value = (n + m) / (ms_step / 1000.0) / 1e9
    log("step %.3f ms -> %.2f Gkeys/s" % (ms_step, value))

    # exact sum of probed bucket lengths (for the probe's algorithmic bytes)
    off, _, ek = table.export()
    h = hg.hg_hash(dq, V, 0).to(torch.int64)
    offl = off.to(torch.int64) & 0xFFFFFFFF
    blen = offl[h + 1] - offl[h]
    sum_len = int(blen.sum().item())
    # a bucket of up to 3 keys is held whole in its index entry; a longer one
    # holds its first key, that key's count and a 24-bit filter of its other
    # keys: a query equal to the first key, or whose filter bit no other key
    # of the bucket sets, needs nothing more; other queries read the rest of
    # the bucket (a bucket of more than 32 keys is counted as read whole)
    eku = ek.to(torch.int64) & 0xFFFFFFFF
    qu = dq.to(torch.int64) & 0xFFFFFFFF
    first = eku[offl[h].clamp(max=n - 1)]
    reads = (blen > 3) & (qu != first)
    sel = torch.nonzero(reads).squeeze(1)
    if sel.numel():
        def fbit(x):  # the entry's filter bit of a key (multiplicative hash)
            return (((x * 0x9E3779B1) & 0xFFFFFFFF) * 24) >> 32
        st, ln = offl[h[sel]], blen[sel]
        pos = st[:, None] + torch.arange(1, int(ln.max().item()), device=st.device)[None, :]
        kk = eku[pos.clamp(max=n - 1)]
        other = (pos < (st + ln)[:, None]) & (kk != first[sel][:, None])
        reads[sel] = (other & (fbit(kk) == fbit(qu[sel])[:, None])).any(1) | (ln > 32)
        del st, ln, pos, kk, other
    sum_tail = int(((blen - 1) * reads).sum().item())
    n_tail = int(reads.sum().item())  # queries that also read the edge array
    del h, offl, off, blen, ek, eku, qu, first, reads, sel

    plan = v2_plan_bytes(hg, n, V, kb)
    kernels = {}
    for name, (launches, tot_ms) in prof.items():
        per = launches / args.steps
        avg = tot_ms / launches
        b = kernel_bytes(name, n, m, V, kb, sum_len, plan)
        bi = index_bytes(name, n, m, V, kb, sum_tail)
        kernels[name] = {"launches_per_step": per, "avg_ms": round(avg, 4),
                         "ms_per_step": round(tot_ms / args.steps, 4),
                         "alg_bytes": b,
                         "alg_GBps": round(b / (avg / 1000.0) / 1e9, 1) if b else None}
        if bi:
            kernels[name]["index_bytes"] = bi
            kernels[name]["index_GBps"] = round(bi / (avg / 1000.0) / 1e9, 1)
    grouped = "probe_ungroup" in kernels
    dom = max((k for k in kernels if kernels[k]["alg_bytes"]),
              key=lambda k: kernels[k]["ms_per_step"])
    dk_ = kernels[dom]
    achieved = dk_["alg_bytes"] / (dk_["avg_ms"] / 1000.0) / 1e9
    digest = src_digest()
    traffic = load_traffic(dom, digest)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": dom,
                "alg_bytes_per_launch": dk_["alg_bytes"], "avg_launch_ms": dk_["avg_ms"],
                # the same kernel's bytes counting the per-bucket probe index
                # it reads (16 B per query) in place of the two offsets
                "index_bytes_per_launch": dk_.get("index_bytes"),
                "index_GBps": dk_.get("index_GBps"),
                # HBM bytes the counters saw per launch, over the same launch time
                "traffic_GBps": (round(traffic / (dk_["avg_ms"] / 1000.0) / 1e9, 1)
                                 if traffic else None)}
    if dom == "probe_count":
        # a random read costs one 128-byte line of HBM traffic: the index
        # entry of every query, plus the edge array for long buckets
        lines = m + n_tail
        roofline["random_lines_per_launch"] = lines
        roofline["line_bytes"] = 128
        roofline["line_GBps"] = round(lines * 128 / (dk_["avg_ms"] / 1000.0) / 1e9, 1)
        # the measured ceiling of independent random 16-byte reads over a
        # 4 GiB footprint (the probe index is 4 GiB at this size)
        micro = micro_roofline(hg)
        rate = micro["4GiB"]["read16_G_per_s"]
        roofline["random_read16_G_per_s_4GiB"] = rate
        roofline["random_lines_G_per_s"] = round(lines / (dk_["avg_ms"] / 1000.0) / 1e9, 2)
        roofline["frac_of_random_read_rate"] = round(
            roofline["random_lines_G_per_s"] / rate, 3)
        roofline["micro_roofline"] = micro
    if grouped:
        # the queries were grouped by bucket range first: each XCD then reads
        # one window of the index at a time and reuses its lines from L2, so
        # the probe can pass the rate of random lines over the whole index
        # (frac_of_random_read_rate above 1); the grouping's own passes are
        # the probe_group* and probe_ungroup kernels
        roofline["probe_order"] = "grouped by bucket range"

    phases = {"kernels": kernels, "source_digest": digest,
              "probe_sum_bucket_len": sum_len, "probe_sum_keys_past_index": sum_tail}
    build_ms = sum(v["ms_per_step"] for k, v in kernels.items()
                   if k.startswith("v2_") or k == "fill")
    # the probe with its query grouping and column scans, when it grouped
    probe_ms = sum(v["ms_per_step"] for k, v in kernels.items() if k.startswith("probe_"))
    phases["build_v2_ms"] = round(build_ms, 3)
    phases["probe_ms"] = round(probe_ms, 3)
    phases["hbm"] = hbm_fractions(build_ms, probe_ms, n, m, V, kb, sum_len, digest,
                                  copy_gbps(torch), grouped)

    if not args.no_extras:
        log("extras")
        reps = 3
        ex = {}
        # hash-range sweep (Fig. 8 style) for V2, V1 and the probe
        big = hg.Table.create(n, 1 << 30, 32)
        for lv in (26, 28, 30):
            Vs = 1 << lv
            t_v2 = timed(lambda: big.rebuild(dk, Vs, 0, variant=hg.VARIANT_V2), reps, torch)
            t_pr = timed(lambda: hg.hg_probe(big, dq, counts=True, out=counts), reps, torch)
            t_v2a = timed(lambda: big.rebuild(dk, Vs, 0, variant=hg.VARIANT_V2, any_order=True),
                          reps, torch)
            t_v2x = timed(lambda: big.rebuild(dk, Vs, 0, variant=hg.VARIANT_V2, index=False),
                          reps, torch)
            t_prx = timed(lambda: hg.hg_probe(big, dq, counts=True, out=counts), reps, torch)
            t_v1p = timed(lambda: big.rebuild(dk, Vs, 0, variant=hg.VARIANT_V1, v1_plain=True), 2,
                          torch)
            t_v1 = timed(lambda: big.rebuild(dk, Vs, 0, variant=hg.VARIANT_V1), 2, torch)
            t_pr1 = timed(lambda: hg.hg_probe(big, dq, counts=True, out=counts), reps, torch)
            ex["V=2^%d" % lv] = {"build_v2_ms": round(t_v2, 3),
                                 "build_v2_Gkeys": round(n / t_v2 / 1e6, 2),
                                 "build_v2_noindex_ms": round(t_v2x, 3),
                                 "build_v2_any_order_ms": round(t_v2a, 3),
                                 "build_v1_ms": round(t_v1, 3),
                                 "build_v1_Gkeys": round(n / t_v1 / 1e6, 2),
                                 "build_v1_plain_ms": round(t_v1p, 3),
                                 "probe_ms": round(t_pr, 3),
                                 "probe_Gkeys": round(m / t_pr / 1e6, 2),
                                 "probe_noindex_ms": round(t_prx, 3),
                                 "probe_v1table_ms": round(t_pr1, 3)}
            log("V=2^%d v2 %.3f (any order %.3f, no index %.3f) ms v1 %.3f ms probe %.3f "
                "(no index %.3f, v1 table %.3f) ms" % (lv, t_v2, t_v2a, t_v2x, t_v1, t_pr, t_prx,
                                                       t_pr1))
        big.free()
        del big
        # all matching pairs of the step's probe (two passes: counts and
        # offsets, then the pairs)
        _, _, npairs = hg.hg_probe_pairs(table, dq, capacity=0)
        t_pairs = timed(lambda: hg.hg_probe_pairs(table, dq, capacity=npairs), reps, torch)
        ex["probe_pairs_2^28"] = {"ms": round(t_pairs, 3), "pairs": npairs,
                                  "G_pairs_per_s": round(npairs / t_pairs / 1e6, 3)}
        log("pairs: %d in %.3f ms" % (npairs, t_pairs))
        # Probe-New (Alg. 3): build the query table, then intersect (counts)
        tq = hg.Table.create(m, V, 32)
        cb = torch.empty(m, dtype=torch.int32, device="cuda")

        def probe_new():
            tq.rebuild(dq, V, 0)
            hg.hg_intersect(table, tq, counts=True, total=False)

        t_pn = timed(probe_new, reps, torch)

        def probe_new_edges():
            # the query table in any order and Alg. 3's counts in its edge order
            tq.rebuild(dq, V, 0, any_order=True)
            hg.hg_intersect_edges(table, tq, counts=True, total=False, out=cb)

        t_pne = timed(probe_new_edges, reps, torch)
        t_int = timed(lambda: hg.hg_intersect(table, tq, counts=True, total=False), reps, torch)
        # the join size alone: no per-query counts scattered back to input order
        t_tot = timed(lambda: hg.hg_intersect(table, tq, counts=False, total=True), reps, torch)
        # counts in the query table's edge order (Alg. 3's own order, sequential writes)
        t_edge = timed(lambda: hg.hg_intersect_edges(table, tq, counts=True, total=False, out=cb),
                       reps, torch)
        ex["probe_new"] = {"ms": round(t_pn, 3), "Gkeys": round(m / t_pn / 1e6, 2),
                           "intersect_only_ms": round(t_int, 3),
                           "intersect_total_only_ms": round(t_tot, 3),
                           "intersect_edge_order_ms": round(t_edge, 3),
                           "any_order_build_and_edge_order_ms": round(t_pne, 3),
                           "build_share": round(1 - t_int / t_pn, 3)}
        tq.free()
        del tq, cb
        # 64-bit keys: 2^27 keys with uint32 ids, V = 2^27, 2^27 queries
        n64 = n // 2
        k64 = workloads.uniform_keys(n64, 64, seed=3)
        q64 = workloads.probe_queries(k64, n64, 0.5, seed=4)
        dk64, dq64 = hg.to_device(k64), hg.to_device(q64)
        del k64, q64
        t64 = hg.Table.create(n64, n64, 64)
        c64 = torch.empty(n64, dtype=torch.int32, device="cuda")
        tb = timed(lambda: t64.rebuild(dk64, n64, 0), reps, torch)
        tp = timed(lambda: hg.hg_probe(t64, dq64, counts=True, out=c64), reps, torch)
        ex["uint64_2^27"] = {"build_v2_ms": round(tb, 3), "build_Gkeys": round(n64 / tb / 1e6, 2),
                             "probe_ms": round(tp, 3), "probe_Gkeys": round(n64 / tp / 1e6, 2)}
        t64.free()
        del dk64, dq64, c64, t64
        # skewed join: 2^27 Zipf(1.2) build keys over 2^24 values, V = 2^27,
        # 2^28 probe keys from the same law (long buckets use key runs)
        log("zipf join")
        nz = n // 2
        kz = hg.to_device(workloads.zipf_keys(nz, 1.2, 1 << 24, seed=21, map_seed=99))
        qz = hg.to_device(workloads.zipf_keys(m, 1.2, 1 << 24, seed=22, map_seed=99))
        tz = hg.Table.create(nz, nz, 32)
        tb = timed(lambda: tz.rebuild(kz, nz, 9), 2, torch)
        tp = timed(lambda: hg.hg_probe(tz, qz, counts=True, out=counts), 2, torch)
        _, ztot = hg.hg_probe(tz, qz, counts=False, total=True)
        # V1 on the skewed keys: merged per-wave atomics against one per key
        tz1 = timed(lambda: tz.rebuild(kz, nz, 9, variant=hg.VARIANT_V1), 2, torch)
        tz1p = timed(lambda: tz.rebuild(kz, nz, 9, variant=hg.VARIANT_V1, v1_plain=True), 2, torch)
        ex["zipf1.2_join"] = {"build_ms": round(tb, 3), "build_Gkeys": round(nz / tb / 1e6, 2),
                              "probe_ms": round(tp, 3), "probe_Gkeys": round(m / tp / 1e6, 2),
                              "matches": ztot, "build_v1_ms": round(tz1, 3),
                              "build_v1_plain_ms": round(tz1p, 3)}
        log("zipf join build %.3f ms probe %.3f ms, %d matches" % (tb, tp, ztot))
        tz.free()
        del kz, qz, tz
        # erasing keys: 2^22 distinct keys removed from a 2^28 table (about 1.6%
        # of its entries), then a probe of all 2^28 queries
        log("erase")
        te = hg.Table.create(n, V, 32)
        te.rebuild(dk, V, 0)
        gone = hg.to_device(np.unique(keys_np[: 1 << 22]))
        te.erase(gone[:0])  # allocates the length and mark arrays
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        removed = te.erase(gone)
        torch.cuda.synchronize()
        t_er = (time.perf_counter() - t0) * 1e3
        t_pe = timed(lambda: hg.hg_probe(te, dq, counts=True, out=counts), reps, torch)
        ex["erase_2^22_keys_from_2^28"] = {"erase_ms": round(t_er, 3), "removed": removed,
                                           "probe_after_ms": round(t_pe, 3)}
        log("erase %d entries %.3f ms, probe after %.3f ms" % (removed, t_er, t_pe))
        te.free()
        del te, gone
        # build once, intersect many: 2^20 sets shaped like sparse rows (mean
        # 32 keys, Pareto tail 1.5, at most 2^16), columns uniform over 2^20,
        # and 2^24 random set pairs (each set takes part in 32 pairs on average)
        log("collection")
        S = 1 << 20
        kc, oc = workloads.collection_sets(S, 32, 1 << 20, seed=31)
        pc = workloads.set_pairs(1 << 24, S, S, seed=32)
        dkc = hg.to_device(kc)
        doc = torch.from_numpy(oc.astype(np.int32)).cuda()
        dpc = torch.from_numpy(pc.view(np.int32)).cuda()
        walked = int(np.minimum(np.diff(oc)[pc[:, 0]], np.diff(oc)[pc[:, 1]]).sum())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        coll = hg.Collection(dkc, doc, seed=5)
        torch.cuda.synchronize()
        t_cb = (time.perf_counter() - t0) * 1e3
        t_ci = timed(lambda: coll.intersect(coll, dpc, counts=True, total=False), reps, torch)
        hg.profile_reset()
        hg.profile_enable(True)
        coll2 = hg.Collection(dkc, doc, seed=5)
        coll.intersect(coll, dpc, counts=True, total=False)
        torch.cuda.synchronize()
        hg.profile_enable(False)
        pr = hg.profile_report()
        hg.profile_reset()
        k_build = sum(v[1] for k, v in pr.items() if k in ("coll_plan", "coll_groups", "coll_big"))
        info = coll.info()
        ex["collection_2^20_sets_2^24_pairs"] = {
            "keys": int(kc.size), "heavy_set_keys": int(info.heavy_keys),
            "build_ms": round(t_cb, 3), "build_device_ms": round(k_build, 3),
            "build_Gkeys": round(kc.size / k_build / 1e6, 2),
            "intersect_ms": round(t_ci, 3), "pairs_G_per_s": round(len(pc) / t_ci / 1e6, 2),
            "walked_items": walked, "walked_G_per_s": round(walked / t_ci / 1e6, 2),
            "pair_count_kernel_ms": round(pr.get("coll_pair_count", (0, 0.0))[1], 3)}
        log("collection: build %.3f ms (kernels %.3f), intersect %.3f ms" % (t_cb, k_build, t_ci))
        coll.free()
        coll2.free()
        del dkc, doc, dpc, kc, oc, pc
        # 2^30 keys, V = 2^30 (two partition passes of 9 bits each)
        log("2^30 keys")
        n30 = 1 << 30
        k30 = hg.to_device(workloads.uniform_keys(n30, 32, seed=8))
        t30 = hg.Table.create(n30, n30, 32)
        tb30a = timed(lambda: t30.rebuild(k30, n30, 0, any_order=True), 2, torch)
        tb30 = timed(lambda: t30.rebuild(k30, n30, 0), 2, torch)
        ex["keys_2^30"] = {"build_any_order_ms": round(tb30a, 3),
                           "build_any_order_Gkeys": round(n30 / tb30a / 1e6, 2),
                           "build_stable_ms": round(tb30, 3),
                           "build_stable_Gkeys": round(n30 / tb30 / 1e6, 2)}
        log("2^30 keys: build any order %.3f ms, stable %.3f ms" % (tb30a, tb30))
        t30.free()
        del k30, t30
        # the paper's own input: the sequence 1..2^25 at loads 0.5 / 1 / 2 / 4
        # (V = N / load); build, then probe every key (all hits).  The paper
        # reports up to 2.5 Gkeys/s build on a GV100 for this input.
        ns = 1 << 25
        ks = hg.to_device(workloads.sequence_keys(ns, 32))
        cs = torch.empty(ns, dtype=torch.int32, device="cuda")
        seq = {}
        for load in (0.5, 1, 2, 4):
            Vs = int(ns / load)
            ts = hg.Table.create(ns, Vs, 32)
            tb_any = timed(lambda: ts.rebuild(ks, Vs, 0, any_order=True), reps, torch)
            tb_st = timed(lambda: ts.rebuild(ks, Vs, 0), reps, torch)
            tp = timed(lambda: hg.hg_probe(ts, ks, counts=True, out=cs), reps, torch)
            seq["load %g" % load] = {"build_any_order_Gkeys": round(ns / tb_any / 1e6, 2),
                                     "build_stable_Gkeys": round(ns / tb_st / 1e6, 2),
                                     "probe_Gkeys": round(ns / tp / 1e6, 2)}
            ts.free()
        seq["paper_gv100_build_peak_Gkeys"] = 2.5
        ex["sequence_2^25"] = seq
        log("sequence 1..2^25: %s" % seq)
        del ks, cs
        phases["extras"] = ex

    if not args.no_batched:
        log("batched")
        phases["batched"] = run_batched(hg, workloads, torch, tables=args.tables, log=log,
                                        any_order=not args.stable)
    if not args.no_serving:
        log("serving")
        phases["serving"] = run_serving(hg, workloads, torch, requests=args.requests, log=log)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline")
        cpu = cpu_baseline(keys_np, q_np, V)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "single table: V2 build of 2^%d uniform uint32 keys, hash_range "
                               "2^%d (%s), with the per-bucket probe index, then "
                               "Probe-Standard counts of 2^%d queries (50%% drawn from the "
                               "keys)" % (args.log2n, args.log2range,
                                          "stable layout" if args.stable else
                                          "order inside a bucket unspecified, as in the paper",
                                          args.log2n),
                   "n": n, "hash_range": V, "m": m, "key_bits": 32,
                   "bucket_order": "stable" if args.stable else "any"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phases": phases,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
