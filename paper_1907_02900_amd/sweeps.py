"""The paper's parameter sweeps, run on this library's kernels (one GPU).

Sec. 5 varies three things on synthetic keys; each sweep here reuses the
seeded generators and the C ABI, and prints one JSON object:

``appearances``  Sec. 5.1 / Fig. 3, 4, 7: N = 2^25 keys drawn uniformly from a
                 range of N / R values (R appearances per key on average,
                 R = 1/8 ... 32), V = N.  V1 build (per-wave merged and
                 per-key atomics), V2 build (stable; any order with and
                 without the probe index, and with hg_build_tune's choice of
                 bins), Probe-Standard counts and Probe-New (build the query
                 table, intersect: counts in its edge order) with queries from
                 the same range.
``bins``         Fig. 4 / 5: V2 build time over sizes 2^21, 2^23, 2^25 and bin
                 counts 2^10 ... 2^16 (the `bins` option; a bin spans a power
                 of two of at most 2^12 buckets here, so small counts are
                 raised), for R = 1 and R = 32.
``range``        Fig. 8: N = 2^25 uniform keys, V = 2N, N, N/2, N/4: V2 build
                 and Probe-Standard (50% hits).

Times are the median of 3 runs after one warm-up, with events on the current
stream; rates are keys (or queries) per second.

Usage: python3 -m paper_1907_02900_amd.sweeps [appearances|bins|range ...]
"""
import json
import sys

import numpy as np
import torch

from . import hg, workloads


def _timed(fn, reps=3):
    fn()
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


def _rate(count, ms):
    return round(count / ms / 1e6, 3)


def appearances(n=1 << 25):
    rows = []
    counts = torch.empty(n, dtype=torch.int32, device="cuda")
    t = hg.Table.create(n, n, 32)
    tq = hg.Table.create(n, n, 32)
    for R in (0.125, 0.25, 0.5, 1, 2, 4, 8, 16, 32):
        k = hg.to_device(workloads.duplicate_keys(n, R, 32, seed=1))
        q = hg.to_device(workloads.duplicate_keys(n, R, 32, seed=2))
        v1 = _timed(lambda: t.rebuild(k, n, 0, variant=hg.VARIANT_V1))
        v1p = _timed(lambda: t.rebuild(k, n, 0, variant=hg.VARIANT_V1, v1_plain=True))
        v2a = _timed(lambda: t.rebuild(k, n, 0, any_order=True))
        v2x = _timed(lambda: t.rebuild(k, n, 0, any_order=True, index=False))
        kw, _ = hg.build_tune(k, n, 0, any_order=True)
        v2t = _timed(lambda: t.rebuild(k, n, 0, **kw))
        v2 = _timed(lambda: t.rebuild(k, n, 0))
        ps = _timed(lambda: hg.hg_probe(t, q, counts=True, out=counts))

        def probe_new():
            tq.rebuild(q, n, 0)
            hg.hg_intersect_edges(t, tq, counts=True, total=False, out=counts)

        pn = _timed(probe_new)
        rows.append({"R": R, "v1_Gkeys": _rate(n, v1), "v1_per_key_atomics_Gkeys": _rate(n, v1p),
                     "v2_stable_Gkeys": _rate(n, v2), "v2_any_Gkeys": _rate(n, v2a),
                     "v2_any_no_index_Gkeys": _rate(n, v2x), "v2_any_tuned_Gkeys": _rate(n, v2t),
                     "tuned_bins": kw["bins"], "probe_standard_Gq": _rate(n, ps),
                     "probe_new_Gq": _rate(n, pn)})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    t.free()
    tq.free()
    return rows


def bins(sizes=(21, 23, 25), bin_counts=(10, 12, 14, 16), appear=(1, 32)):
    rows = []
    for lg in sizes:
        n = 1 << lg
        t = hg.Table.create(n, n, 32)
        for R in appear:
            k = hg.to_device(workloads.duplicate_keys(n, R, 32, seed=3))
            for lb in bin_counts:
                b = min(1 << lb, n)
                ms = _timed(lambda: t.rebuild(k, n, 0, bins=b))
                rows.append({"log2n": lg, "R": R, "bins": b, "v2_stable_Gkeys": _rate(n, ms)})
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        t.free()
    return rows


def hash_range(n=1 << 25):
    rows = []
    k_np = workloads.uniform_keys(n, 32, seed=4)
    k = hg.to_device(k_np)
    q = hg.to_device(workloads.probe_queries(k_np, n, 0.5, seed=5))
    counts = torch.empty(n, dtype=torch.int32, device="cuda")
    for f in (2.0, 1.0, 0.5, 0.25):
        V = int(n * f)
        t = hg.Table.create(n, V, 32)
        b = _timed(lambda: t.rebuild(k, V, 0))
        ba = _timed(lambda: t.rebuild(k, V, 0, any_order=True))
        p = _timed(lambda: hg.hg_probe(t, q, counts=True, out=counts))
        rows.append({"V_over_N": f, "v2_stable_Gkeys": _rate(n, b), "v2_any_Gkeys": _rate(n, ba),
                     "probe_Gq": _rate(n, p)})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        t.free()
    return rows


def main(argv=None):
    which = (argv if argv is not None else sys.argv[1:]) or ["appearances", "bins", "range"]
    hg.lib()
    fns = {"appearances": appearances, "bins": bins, "range": hash_range}
    out = {w: fns[w]() for w in which}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
