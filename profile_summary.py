"""Summarise rocprofv3 output of bench.py runs into profiles/.

Reads
  --stats DIR    output of `rocprofv3 --kernel-trace --stats --output-format csv`
  --fetch CSV    counter_collection.csv of a `--pmc FETCH_SIZE` run
  --write CSV    counter_collection.csv of a `--pmc WRITE_SIZE` run
and writes
  profiles/<kernel>_<workload>.md          per-kernel durations + traffic
  profiles/<kernel>_<workload>_traffic.json DRAM-side bytes per launch of the
                                            row-accumulation kernel, tagged with
                                            the hash of its source
Counter runs include a plain 1 GiB device copy (bench.py --calibrate-copy);
its FETCH_SIZE / WRITE_SIZE readings against 1 GiB give the scale factor
applied to the kernel's readings.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

COPY_BYTES = 1 << 30


def _counter_rows(path):
    with open(path) as f:
        return list(csv.DictReader(f))


def _per_kernel(rows, name_filter):
    vals = [float(r["Counter_Value"]) for r in rows if name_filter(r["Kernel_Name"])]
    return vals


def _is_accum(name):
    return "k_accum" in name


def _is_copy(name):
    return "copyBuffer" in name


def counter_bytes(path, last=0):
    """(kernel KiB per launch mean, copy KiB mean, launches) from one counter CSV;
    with last > 0 only the last `last` accumulation launches (the timed sweeps,
    after any tuning trials) are averaged."""
    rows = _counter_rows(path)
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    acc = _per_kernel(rows, _is_accum)
    if last > 0:
        acc = acc[-last:]
    # the calibration: bench.py --calibrate-copy runs three 1 GiB copies back
    # to back, i.e. three consecutive copy dispatches with equal readings
    cps = [(int(r["Dispatch_Id"]), float(r["Counter_Value"])) for r in rows if _is_copy(r["Kernel_Name"])]
    cp = []
    for q in range(len(cps) - 2):
        ids = [cps[q + t][0] for t in range(3)]
        vals = [cps[q + t][1] for t in range(3)]
        if ids == [ids[0], ids[0] + 1, ids[0] + 2] and min(vals) > 0 and max(vals) / min(vals) < 1.01:
            cp = vals
            break
    return (statistics.mean(acc) if acc else None, statistics.mean(cp) if cp else None, len(acc))


def kernel_stats(stats_dir):
    paths = glob.glob(os.path.join(stats_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not paths:
        raise SystemExit(f"no kernel_stats.csv under {stats_dir}")
    with open(paths[0]) as f:
        return list(csv.DictReader(f))


def timed_launches(stats_dir, n):
    """Mean duration (us) of the last n accumulation launches in the kernel trace
    of the stats run (the timed sweeps, after tuning trials and warm-up)."""
    paths = glob.glob(os.path.join(stats_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not paths:
        return None
    with open(paths[0]) as f:
        rows = [r for r in csv.DictReader(f) if "k_accum" in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    last = rows[-n:]
    if not last:
        return None
    return sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in last) / len(last) / 1e3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--stats-cmd", required=True)
    ap.add_argument("--fetch-cmd", default="")
    ap.add_argument("--write-cmd", default="")
    ap.add_argument("--bench-json", default=None, help="bench.py output line of the same build")
    ap.add_argument("--tcc", default=None,
                    help="counter_collection.csv of a `--pmc TCC_HIT_sum TCC_MISS_sum` run")
    ap.add_argument("--tcc-cmd", default="")
    ap.add_argument("--timed", type=int, default=0,
                    help="accumulation launches of the timed sweeps in the stats run")
    ap.add_argument("--last", type=int, default=0,
                    help="average only the last N accumulation launches of each counter run")
    args = ap.parse_args()

    from bench import kernel_source_hash

    stats = kernel_stats(args.stats)
    total = sum(float(r["TotalDurationNs"]) for r in stats)
    lines = [f"# Row-accumulation kernels on {args.workload}", "",
             "Per-kernel durations from `rocprofv3 --kernel-trace --stats` (times in microseconds).",
             "", f"Command: `{args.stats_cmd}`", "",
             "| kernel | calls | avg us | min us | max us | share |", "|---|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:14]:
        lines.append(f"| `{r['Name'][:80]}` | {r['Calls']} | {float(r['AverageNs'])/1e3:.1f} | "
                     f"{float(r['MinNs'])/1e3:.1f} | {float(r['MaxNs'])/1e3:.1f} | "
                     f"{100*float(r['TotalDurationNs'])/total:.1f}% |")
    acc = [r for r in stats if "k_accum" in r["Name"]]
    calls = sum(int(r["Calls"]) for r in acc)
    avg_us = sum(float(r["TotalDurationNs"]) for r in acc) / max(calls, 1) / 1e3
    lines += ["", f"All accumulation launches (k_accum*): {calls} calls, average {avg_us:.1f} us per launch "
              "(tuning trials included)."]
    if args.timed:
        t_us = timed_launches(args.stats, args.timed)
        if t_us is not None:
            lines += ["", f"Timed sweeps of the same run (the last {args.timed} accumulation launches of "
                      f"its kernel trace): average {t_us:.1f} us per launch."]

    traffic = None
    if args.fetch and args.write:
        fk, fc, nf = counter_bytes(args.fetch, args.last)
        wk, wc, nw = counter_bytes(args.write, args.last)
        ffac = (COPY_BYTES / 1024) / fc if fc else 1.0
        wfac = (COPY_BYTES / 1024) / wc if wc else 1.0
        fbytes = fk * 1024 * ffac
        wbytes = wk * 1024 * wfac
        traffic = {"kernel_source_sha": kernel_source_hash(), "workload": args.workload,
                   "fetch_bytes_per_launch": fbytes, "write_bytes_per_launch": wbytes,
                   "bytes_per_launch": fbytes + wbytes, "launches_sampled": nf,
                   "copy_fetch_kib": fc, "copy_write_kib": wc,
                   "fetch_scale": ffac, "write_scale": wfac}
        lines += ["", "## HBM-side traffic of the accumulation kernels (rocprofv3 --pmc)", "",
                  f"FETCH_SIZE command: `{args.fetch_cmd}`", "",
                  f"WRITE_SIZE command: `{args.write_cmd}`", "",
                  "A 1 GiB device copy (`__amd_rocclr_copyBuffer`) in the same runs calibrates the "
                  f"counters: FETCH_SIZE read {fc:.0f} KiB (scale {ffac:.4f}), WRITE_SIZE read "
                  f"{wc:.0f} KiB (scale {wfac:.4f}) for 1048576 KiB moved.", "",
                  f"per accumulation launch (mean of the last {nf} launches, the timed sweep): "
                  f"fetch {fbytes/1e9:.3f} GB, "
                  f"write {wbytes/1e9:.3f} GB, total {(fbytes+wbytes)/1e9:.3f} GB."]
        tpath = os.path.join(ROOT, "profiles", f"k_accum_{args.workload}_traffic.json")
        with open(tpath, "w") as f:
            json.dump(traffic, f, indent=1)
    if args.tcc:
        rows = _counter_rows(args.tcc)
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        per = {}
        for r in rows:
            if _is_accum(r["Kernel_Name"]):
                per.setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
        ids = sorted(per)[-args.last:] if args.last > 0 else sorted(per)
        hit = sum(per[i].get("TCC_HIT_sum", 0.0) for i in ids)
        miss = sum(per[i].get("TCC_MISS_sum", 0.0) for i in ids)
        lines += ["", "## L2 (TCC) hit rate of the accumulation kernels", "",
                  f"Command: `{args.tcc_cmd}`", "",
                  f"last {len(ids)} launches (the timed sweep): {hit:.4g} hits, {miss:.4g} misses, "
                  f"hit rate {100 * hit / max(hit + miss, 1):.1f}%."]
    if args.bench_json:
        with open(args.bench_json) as f:
            b = json.loads([l for l in f if l.startswith("{")][-1])
        rf = b["roofline"]
        lines += ["", "## bench.py line of the same build", "",
                  f"value {b['value']:.4g} {b['unit']}, {b['ms_per_step']:.1f} ms per sweep; "
                  f"accumulation kernels: average launch {rf['avg_launch_ms']:.3f} ms (HIP events), "
                  f"{rf['alg_bytes_per_launch']/1e9:.3f} GB algorithmic per launch, "
                  f"achieved {rf['achieved']:.0f} GB/s = {100*rf['frac']:.1f}% of 8 TB/s."]
    out = os.path.join(ROOT, "profiles", f"k_accum_{args.workload}.md")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out)


if __name__ == "__main__":
    main()
