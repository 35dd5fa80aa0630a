"""Summaries of rocprofv3 result databases (kernel durations and PMC counters).

Used to turn the SQLite output of ``rocprofv3 --kernel-trace --stats`` and
``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs into the short text summaries kept
under profiles/.  Command line:

  python -m paper_2211_15308_amd.profile_tools stats  <results.db> [name filter]
  python -m paper_2211_15308_amd.profile_tools pmc    <results.db> <counter> <name filter>
  python -m paper_2211_15308_amd.profile_tools csvstats <kernel_stats.csv>
  python -m paper_2211_15308_amd.profile_tools csvpmc <counter_collection.csv>
  python -m paper_2211_15308_amd.profile_tools csvtrace <kernel_trace.csv> <name> <split_us>
  python -m paper_2211_15308_amd.profile_tools csvgrid <kernel_trace.csv> [rows]
  python -m paper_2211_15308_amd.profile_tools traffic <fetch.csv> <write.csv> <kernel> <out.json>
  python -m paper_2211_15308_amd.profile_tools traffic_batched <fetch.csv> <write.csv> <kernel> <out.json>

`traffic` turns a FETCH_SIZE run and a WRITE_SIZE run of ``bench.py --pmc-mode`` (which also
copies 256 MiB device-to-device once, as the calibration of known size) into HBM bytes per
working launch of one kernel; bench.py reads the record while its sources are unchanged.
"""
import csv
import collections
import sqlite3
import sys


def _rows(db, table):
    con = sqlite3.connect(db)
    cur = con.cursor()
    cols = [r[1] for r in cur.execute(f"pragma table_info({table})")]
    return cols, cur.execute(f"select * from {table}").fetchall()


def kernel_stats(db, name_filter=None):
    """{kernel name: (calls, total_us, avg_us)} from the kernel trace."""
    cols, rows = _rows(db, "kernels")
    ci = {c: i for i, c in enumerate(cols)}
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in rows:
        nm = r[ci["name"]]
        if name_filter and name_filter not in nm:
            continue
        d = (r[ci["end"]] - r[ci["start"]]) / 1e3
        agg[nm][0] += 1
        agg[nm][1] += d
    return {k: (v[0], v[1], v[1] / v[0]) for k, v in agg.items()}


def pmc_per_dispatch(db, counter, name_filter):
    """Per-dispatch values of one counter for kernels whose name contains name_filter."""
    con = sqlite3.connect(db)
    cur = con.cursor()
    cols = [r[1] for r in cur.execute("pragma table_info(counters_collection)")]
    rows = cur.execute("select * from counters_collection").fetchall()
    ci = {c: i for i, c in enumerate(cols)}
    name_col = "kernel_name" if "kernel_name" in ci else "name"
    val_col = "value" if "value" in ci else "counter_value"
    cname_col = "counter_name" if "counter_name" in ci else "counter"
    out = collections.defaultdict(float)
    for r in rows:
        if name_filter not in str(r[ci[name_col]]) or r[ci[cname_col]] != counter:
            continue
        key = r[ci["dispatch_id"]] if "dispatch_id" in ci else r[ci["id"]]
        out[key] += float(r[ci[val_col]])
    return list(out.values())


def short_name(name):
    """A kernel's name without its argument list ("(anonymous namespace)" is kept)."""
    base = name.replace("(anonymous namespace)::", "")
    return base.split("(")[0].strip()


def csv_kernel_stats(path):
    """Rows of a rocprofv3 *_kernel_stats.csv, sorted by total time."""
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        out.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]) / 1e3,
                    float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    return sorted(out, key=lambda t: -t[2])


def csv_pmc(path):
    """{kernel name: (dispatches, counter name, per-dispatch values)} of a counter CSV."""
    agg = collections.defaultdict(list)
    cname = {}
    disp = collections.defaultdict(float)
    for r in csv.DictReader(open(path)):
        key = (r["Kernel_Name"], r["Dispatch_Id"])
        disp[key] += float(r["Counter_Value"])
        cname[r["Kernel_Name"]] = r["Counter_Name"]
    for (k, _), v in disp.items():
        agg[k].append(v)
    return {k: (len(v), cname[k], v) for k, v in agg.items()}


def csv_trace_split(path, name, split_us):
    """Durations (us) of the dispatches of one kernel from a kernel_trace.csv, split at split_us."""
    durs = []
    for r in csv.DictReader(open(path)):
        if short_name(r["Kernel_Name"]) == short_name(name):
            durs.append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    long = [d for d in durs if d >= split_us]
    return durs, long


def csv_grid_groups(path):
    """Rows (kernel, threads of the grid, calls, average us, total us) of a kernel_trace.csv grouped
    by kernel and grid size (for multigrid kernels: by level), sorted by total time."""
    groups = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        threads = 1
        for ax in ("X", "Y", "Z"):
            threads *= int(r.get(f"Grid_Size_{ax}", "1") or 1)
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        groups[(short_name(r["Kernel_Name"]), threads)].append(dur)
    out = [(k, t, len(v), sum(v) / len(v), sum(v)) for (k, t), v in groups.items()]
    return sorted(out, key=lambda row: -row[4])


def traffic_record(fetch_csv, write_csv, kernel, copy_bytes=256 << 20):
    """HBM bytes per working dispatch of `kernel`, each counter scaled by the copy's reading."""
    fet, wri = csv_pmc(fetch_csv), csv_pmc(write_csv)

    def pick(table, name):
        for k, (n, cn, vals) in table.items():
            if k.split("(")[0].strip() == name:
                return vals
        raise KeyError(name)

    def copy_reading(table):
        best = 0.0
        for k, (n, cn, vals) in table.items():
            if "copyBuffer" in k or "elementwise" in k:
                best = max(best, max(vals))
        return best

    def working(vals):
        big = [v for v in vals if v > 0.1 * max(vals)]
        return sum(big) / len(big)

    cf, cw = copy_reading(fet), copy_reading(wri)
    ff = copy_bytes / 1024.0 / cf
    wf = copy_bytes / 1024.0 / cw
    f_kib, w_kib = working(pick(fet, kernel)), working(pick(wri, kernel))
    return {"kernel": kernel, "fetch_kib_per_working_dispatch": f_kib,
            "write_kib_per_working_dispatch": w_kib, "copy_bytes": float(copy_bytes),
            "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_factor": ff, "write_factor": wf,
            "traffic_bytes_per_launch": 1024.0 * (f_kib * ff + w_kib * wf)}


def main(argv):
    if argv[0] == "stats":
        st = kernel_stats(argv[1], argv[2] if len(argv) > 2 else None)
        tot = sum(v[1] for v in st.values())
        print(f"{'total_us':>12} {'pct':>6} {'calls':>7} {'avg_us':>9}  kernel")
        for k, (c, t, a) in sorted(st.items(), key=lambda kv: -kv[1][1]):
            print(f"{t:12.1f} {100 * t / tot:6.1f} {c:7d} {a:9.2f}  {k.split('(')[0]}")
    elif argv[0] == "csvstats":
        print(f"{'total_us':>12} {'pct':>6} {'calls':>7} {'avg_us':>9}  kernel")
        for name, calls, tot, avg, pct in csv_kernel_stats(argv[1]):
            print(f"{tot:12.1f} {pct:6.2f} {calls:7d} {avg:9.2f}  {short_name(name)}")
    elif argv[0] == "csvgrid":
        rows = csv_grid_groups(argv[1])
        total = sum(r[4] for r in rows)
        print(f"total kernel time {total / 1e3:.1f} ms")
        print(f"{'kernel':40s} {'threads':>9} {'calls':>7} {'avg_us':>8} {'pct':>6}")
        for name, threads, calls, avg, tot in rows[:int(argv[2]) if len(argv) > 2 else 30]:
            print(f"{name[:40]:40s} {threads:9d} {calls:7d} {avg:8.2f} {100 * tot / total:6.2f}")
    elif argv[0] == "csvpmc":
        for k, (n, cn, vals) in sorted(csv_pmc(argv[1]).items(), key=lambda kv: -sum(kv[1][2])):
            big = [v for v in vals if v > 0.1 * max(vals)]
            print(f"{cn} dispatches {n:6d} working {len(big):6d} avg_working_KiB "
                  f"{sum(big) / max(len(big), 1):14.1f} max_KiB {max(vals):14.1f}  {short_name(k)}")
    elif argv[0] == "csvtrace":
        durs, long = csv_trace_split(argv[1], argv[2], float(argv[3]))
        print(f"{argv[2]}: dispatches {len(durs)} avg_us {sum(durs) / max(len(durs), 1):.2f}; "
              f">= {argv[3]} us: {len(long)} avg_us {sum(long) / max(len(long), 1):.2f}")
    elif argv[0] in ("traffic", "traffic_batched"):
        import json
        import os
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        import bench
        rec = traffic_record(argv[1], argv[2], argv[3])
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        if argv[0] == "traffic":
            rec["kernel_sources_sha256"] = bench.kernel_source_sha(root)
            rec["workload"] = "2D n=1024 finest level (1023^2 interior points), FP32"
            mode, out = "--pmc-mode", "profiles/down0_traffic.json"
        else:
            rec["kernel_sources_sha256"] = bench.kernel_source_sha(
                root, ("kernels_batch.hip", "mg_device.h", "fdd_internal.h"))
            rec["workload"] = ("32 instances at n=1024 (32 x 1023^2 interior points), FP32, every "
                               "instance's finest level in one launch")
            mode, out = "--only-batched --pmc-mode", "profiles/kb_down0_traffic.json"
        rec["commands"] = [
            f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d /tmp/pmc_fetch -o pmc -- python3 bench.py {mode}",
            f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d /tmp/pmc_write -o pmc -- python3 bench.py {mode}",
            f"python3 -m paper_2211_15308_amd.profile_tools {argv[0]} /tmp/pmc_fetch/pmc_counter_collection.csv "
            f"/tmp/pmc_write/pmc_counter_collection.csv '{argv[3]}' {out}"]
        json.dump(rec, open(argv[4], "w"), indent=1)
        print(json.dumps(rec))
    elif argv[0] == "pmc":
        vals = pmc_per_dispatch(argv[1], argv[2], argv[3])
        nz = [v for v in vals if v > 0]
        print(f"{argv[2]} {argv[3]}: dispatches {len(vals)} nonzero {len(nz)} "
              f"avg_nonzero {sum(nz) / max(len(nz), 1):.1f} max {max(vals) if vals else 0:.1f}")


if __name__ == "__main__":
    main(sys.argv[1:])
