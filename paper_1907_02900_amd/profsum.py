"""Summaries of rocprofv3 output databases (rocpd SQLite, ``*_results.db``).

Two commands, both reading what ``rocprofv3 -d DIR -o run`` wrote:

``trace DB --title T --cmd C``
    Markdown table of per-kernel statistics (calls, total and average
    duration) from a ``--kernel-trace --stats`` run, plus the launch shape of
    each library kernel.

``traffic --fetch DB --write DB --copy-fetch DB --copy-write DB --out JSON
[--rand-fetch DB]``
    HBM bytes per launch of the library's kernels from two ``--pmc`` runs
    (FETCH_SIZE, then WRITE_SIZE; both in KiB per dispatch).  Each counter is
    scaled by what it reads for a plain 1 GiB device-to-device copy (the
    ``bench.py --copy-calibration`` run), so that the figures are in bytes of
    HBM traffic.  With ``--rand-fetch`` (a FETCH_SIZE run of ``bench.py
    --random-calibration``) it also records what the counter reads per random
    16-byte read, raw and scaled.  The JSON carries the digest of the kernel sources it was
    taken on; bench.py reports the traffic only while that digest matches.

``counters DB [DB ...] --title T --cmd C``
    Markdown table of the SQ (shader sequencer) counters of the step's
    kernels from one or more ``--pmc`` runs (per kernel, the mean over its
    dispatches; a counter present in several runs keeps the last run's), with
    the share of wave time spent waiting and per-wave VALU, LDS and LDS
    bank-conflict cycles.

Usage: python3 -m paper_1907_02900_amd.profsum trace|traffic|counters ...
"""
import argparse
import collections
import json
import sqlite3
import sys

# library kernel -> name of the timed range bench.py reports it under
RANGES = [
    ("k_probe_count", "probe_count"),
    # the probe's query grouping before the build's passes of the same code
    ("k_tile_partition<unsigned int, false, false, false, true", "probe_group"),
    ("k_tile_hist<unsigned int, false, true", "probe_group_hist"),
    ("k_ungroup_by_pos", "probe_ungroup"),
    ("k_local_light", "v2_local_build"),
    ("k_local_heavy", "v2_local_heavy"),
    ("k_tile_partition<unsigned int, false", "v2_partition_t1"),
    ("k_tile_partition<unsigned int, true", "v2_partition_t2"),
    ("k_tile_hist", "v2_tile_hist"),
    ("k_hist_global", "v1_hist_global"),
    ("k_scatter_v1", "v1_scatter"),
    ("k_hist_wave", "v1_hist_wave"),
    ("k_scatter_wave", "v1_scatter_wave"),
    ("k_intersect_count", "intersect_count"),
]


def short_name(name):
    s = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
    if "at::native" in s:
        s = "torch:" + s.split("<")[0][-40:]
    return s


def cmd_trace(a):
    c = sqlite3.connect(a.db)
    out = ["# %s" % a.title, "", "Command (from the repository root, one MI355X):", "",
           "    %s" % a.cmd, "", "rocprofv3 kernel statistics (durations in microseconds):", "",
           "| kernel | calls | total us | avg us | % |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in c.execute(
            "select name, total_calls, total_duration, average, percentage from top_kernels"):
        out.append("| %s | %d | %.1f | %.2f | %.2f |" % (short_name(name), calls, tot, avg, pct))
    out += ["", "Launch shapes (grid in threads, workgroup size, LDS bytes, VGPRs):", ""]
    seen = set()
    for r in c.execute("select name, grid_x, workgroup_x, lds_size, vgpr_count from kernels"):
        nm = short_name(r[0])
        if nm in seen or not nm.startswith("hg::"):
            continue
        seen.add(nm)
        out.append("- %s: grid %d, wg %d, lds %d, vgpr %d" % (nm, r[1], r[2], r[3], r[4]))
    text = "\n".join(out) + "\n"
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    sys.stdout.write(text)


def per_kernel(db, counter):
    c = sqlite3.connect(db)
    agg = collections.defaultdict(list)
    for name, cn, cv in c.execute(
            "select name, counter_name, counter_value from pmc_events"):
        if cn == counter:
            agg[name].append(cv)
    return agg


def median(v):
    v = sorted(v)
    return v[len(v) // 2]


def cmd_traffic(a):
    fc, wc = per_kernel(a.copy_fetch, "FETCH_SIZE"), per_kernel(a.copy_write, "WRITE_SIZE")

    def copy_vals(d):
        return [x for k, vs in d.items() if "copy" in k.lower() or "elementwise" in k.lower()
                for x in vs]

    # counters are KiB per dispatch; the calibration copy moves 1 GiB each way
    sf = (1 << 30) / (median(copy_vals(fc)) * 1024.0)
    sw = (1 << 30) / (median(copy_vals(wc)) * 1024.0)
    fb, wb = per_kernel(a.fetch, "FETCH_SIZE"), per_kernel(a.write, "WRITE_SIZE")
    res = {"source_digest": a.digest, "fetch_scale": sf, "write_scale": sw,
           "command": a.cmd, "kernels": {}}
    for full, vals in fb.items():
        s = short_name(full).replace("hg::", "")
        key = next((nm for pat, nm in RANGES if s.startswith(pat)), None)
        if key is None:
            continue
        f = median(vals) * 1024.0 * sf
        w = median(wb.get(full, [0.0])) * 1024.0 * sw
        res["kernels"][key] = {"kernel": s, "fetch_bytes": f, "write_bytes": w,
                               "hbm_bytes_per_launch": f + w, "dispatches": len(vals)}
    if a.rand_fetch:
        # random 16-byte reads of known count: bytes the counter sees per read
        rv = [x for k, vs in per_kernel(a.rand_fetch, "FETCH_SIZE").items()
              if "k_rand_read16" in k for x in vs]
        raw = median(rv) * 1024.0 / float(a.rand_accesses)
        res["random_read16"] = {"reads_per_dispatch": int(a.rand_accesses),
                                "dispatches": len(rv),
                                "fetch_bytes_per_read_raw": raw,
                                "fetch_bytes_per_read_scaled": raw * sf}
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


SQ_COLS = ["SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_LDS",
           "SQ_INSTS_LDS", "SQ_ACTIVE_INST_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_VALU"]
SQ_KERNELS = ("k_tile_hist", "k_tile_partition", "k_local_light", "k_probe_count",
              "k_ungroup_by_pos")


def cmd_counters(a):
    rows = collections.OrderedDict()
    for db in a.dbs:
        c = sqlite3.connect(db)
        agg = collections.defaultdict(lambda: collections.defaultdict(list))
        for name, cn, cv in c.execute("select name, counter_name, counter_value from pmc_events"):
            if any(k in name for k in SQ_KERNELS):
                agg[short_name(name)][cn].append(cv)
        for k in sorted(agg):
            rows.setdefault(k, {}).update({cn: sum(v) / len(v) for cn, v in agg[k].items()})
    cols = [c for c in SQ_COLS if any(c in d for d in rows.values())]
    out = ["# %s" % a.title, "", "Commands (from the repository root, one MI355X):", "",
           "    %s" % a.cmd, "",
           "Per kernel, the mean over its dispatches of each counter (as rocprofv3 reports "
           "them; cycle counters of the sampled shader engines).  wait = SQ_WAIT_ANY / "
           "SQ_WAVE_CYCLES; per wave = counter / SQ_WAVES.", "",
           "| kernel | " + " | ".join(cols) + " | wait | per wave: VALU / LDS / LDS bank-conflict |",
           "|---|" + "---|" * (len(cols) + 2)]
    for k, d in rows.items():
        w = d.get("SQ_WAVES", 0) or 1
        wait = d.get("SQ_WAIT_ANY", 0) / (d.get("SQ_WAVE_CYCLES", 0) or 1)
        out.append("| %s | %s | %.2f | %.0f / %.0f / %.0f |" % (
            k, " | ".join("%.0f" % d.get(c, 0) for c in cols), wait,
            d.get("SQ_ACTIVE_INST_VALU", 0) / w, d.get("SQ_ACTIVE_INST_LDS", 0) / w,
            d.get("SQ_LDS_BANK_CONFLICT", 0) / w))
    text = "\n".join(out) + "\n"
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    sys.stdout.write(text)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="profsum")
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--title", required=True)
    t.add_argument("--cmd", required=True)
    t.add_argument("--out")
    t.set_defaults(fn=cmd_trace)
    p = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "out", "digest", "cmd"):
        p.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    p.add_argument("--rand-fetch", dest="rand_fetch", default=None)
    p.add_argument("--rand-accesses", dest="rand_accesses", type=int, default=1 << 27)
    p.set_defaults(fn=cmd_traffic)
    q = sub.add_parser("counters")
    q.add_argument("dbs", nargs="+")
    q.add_argument("--title", required=True)
    q.add_argument("--cmd", required=True)
    q.add_argument("--out")
    q.set_defaults(fn=cmd_counters)
    a = ap.parse_args(argv)
    a.fn(a)


if __name__ == "__main__":
    main()
