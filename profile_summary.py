"""Summarise rocprofv3 output of bench.py runs into profiles/.

Reads
  --stats DIR    output of `rocprofv3 --kernel-trace --stats --output-format csv`
  --fetch CSV    counter_collection.csv of a `--pmc FETCH_SIZE` run
  --write CSV    counter_collection.csv of a `--pmc WRITE_SIZE` run
  --reads CSV    counter_collection.csv of a `--pmc TCC_EA0_RDREQ_32B_sum
                 TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum` run
  --writes CSV   counter_collection.csv of a `--pmc TCC_EA0_WRREQ_sum
                 TCC_EA0_WRREQ_64B_sum TCC_HIT_sum TCC_MISS_sum` run
  --dram CSV     counter_collection.csv of a `--pmc TCC_EA0_RDREQ_DRAM_32B_sum
                 TCC_EA0_WRREQ_WRITE_DRAM_32B_sum` run (the requests the L2
                 sends towards DRAM, in 32-byte units)
or, with --ceiling FILE (the JSON line of `bench.py --gather-ceiling`),
writes profiles/gather_ceiling.{json,md} and nothing else; with --serving
FILE (the JSON line of `bench.py --serve-full`), profiles/serving_<workload>.md; with
--kernels DIR --name NAME, a table of the kernels matching --match;
otherwise writes
  profiles/k_accum_<workload>.md          per-kernel durations and traffic
  profiles/k_accum_<workload>_traffic.json bytes per launch of the row-
                                           accumulation kernels, tagged with
                                           the hash of their source
HBM-side bytes are the L2's requests to memory by size: read requests of 32,
64 and 128 bytes, write requests of 32 and 64 bytes.  FETCH_SIZE and
WRITE_SIZE (the counters' own byte formulas) are reported beside them, each
scaled by what it reads for a plain 1 GiB device copy in the same run
(bench.py --calibrate-copy).  Both are L2-miss traffic: requests the 256 MB
last-level cache serves are counted too.
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


def _rows(path):
    with open(path) as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows


def _per_dispatch(path, want):
    """{dispatch id: {counter: value}} for the dispatches whose kernel name passes `want`."""
    per = {}
    for r in _rows(path):
        if want(r["Kernel_Name"]):
            per.setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
    return per


def _is_accum(name):
    return "k_accum" in name


def _is_copy(name):
    return "copyBuffer" in name


def _last(per, n):
    ids = sorted(per)
    return [per[i] for i in (ids[-n:] if n > 0 else ids)]


def _copy_reading(path, counter):
    """The counter's reading for the calibration copy: three consecutive copy
    dispatches with equal readings (bench.py --calibrate-copy)."""
    cps = sorted((i, v.get(counter, 0.0)) for i, v in _per_dispatch(path, _is_copy).items())
    for q in range(len(cps) - 2):
        ids = [cps[q + t][0] for t in range(3)]
        vals = [cps[q + t][1] for t in range(3)]
        if ids == [ids[0], ids[0] + 1, ids[0] + 2] and min(vals) > 0 and max(vals) / min(vals) < 1.01:
            return statistics.mean(vals)
    return None


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


def write_ceiling(path, cmd):
    """The random-gather ceiling (tf_probe_gather by table size) as JSON for
    bench.py and as a short table."""
    with open(path) as f:
        c = json.loads([l for l in f if l.startswith("{")][-1])["gather_ceiling"]
    c["command"] = cmd
    with open(os.path.join(ROOT, "profiles", "gather_ceiling.json"), "w") as f:
        json.dump(c, f, indent=1)
    lines = ["# Random 128-byte row gathers by table size (tf_probe_gather)", "",
             f"Command: `{cmd}`", "",
             f"{c['waves']} wavefronts, {c['rows_per_half_wave']} rows per half-wavefront, one "
             "coalesced 128-byte load per row and half-wavefront, rows drawn by a counter-based "
             "hash (no index stream); median of 5 timed launches after one warm-up.", "",
             "| table | median ms | G lines/s | GB/s |", "|---|---|---|---|"]
    for r in c["tables"]:
        lines.append(f"| {r['table_mb']} MB | {r['median_ms']:.2f} | {r['glines_s']:.1f} | "
                     f"{r['gbytes_s']:.0f} |")
    lines += ["", f"Ceiling used for the row passes' L2-miss line rate: {c['ceiling_glines_s']:.1f} "
              f"G lines/s ({c['ceiling_table']} table: far above the 8 x 4 MB of L2 and the "
              "256 MB last-level cache)."]
    if c.get("hit_ceiling_glines_s"):
        lines += ["", f"Rate of requests served by L2: {c['hit_ceiling_glines_s']:.1f} G lines/s "
                  f"({c['hit_table']} table: a quarter of one XCD's 4 MB L2)."]
    with open(os.path.join(ROOT, "profiles", "gather_ceiling.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print(os.path.join(ROOT, "profiles", "gather_ceiling.md"))


def write_serving(path, cmd):
    """Fold-in serving latency per method and arrival rate, and the oracle's
    offline solve rate, as a short table."""
    with open(path) as f:
        d = json.loads([l for l in f if l.startswith("{")][-1])
    lines = [f"# Fold-in serving on {d['workload']} factors", "", f"Command: `{cmd}`", "",
             "Poisson arrivals; latency = submit to the row on the host; requests of the first "
             "5 s of each schedule are not counted.", "",
             "| method | rate /s | requests | p50 us | p90 us | p99 us | p99.9 us | solves/s | "
             "mean batch | failed |", "|---|---|---|---|---|---|---|---|---|---|"]
    for r in d["serving_full"]:
        lines.append(f"| {r['method']} | {r['rate_req_s']} | {r['requests']} | {r['p50_us']:.0f} | "
                     f"{r['p90_us']:.0f} | {r['p99_us']:.0f} | {r['p999_us']:.0f} | "
                     f"{r['solves_per_s']:.0f} | {r['mean_batch']:.1f} | {r['failed']} |")
    cpu = d.get("cpu_baseline")
    if cpu:
        lines += ["", f"The oracle (FP64, offline, {cpu['sample']}; host {cpu['host'].get('Model name')}, "
                  f"{cpu['host'].get('nproc')} threads):", ""]
        for k, v in cpu.items():
            if isinstance(v, dict) and "solves_per_s" in v:
                lines.append(f"* {k}: {v['one_thread_solves_per_s']:.0f} solves/s on 1 thread, "
                             f"{v['solves_per_s']:.0f} on {v['cores']}")
    out = os.path.join(ROOT, "profiles", f"serving_{d['workload']}.md")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out)


def write_kernels(stats_dir, name, cmd, pattern):
    """Per-kernel durations of a `--kernel-trace --stats` run, the kernels
    whose name contains `pattern` first, as a short table."""
    stats = kernel_stats(stats_dir)
    total = sum(float(r["TotalDurationNs"]) for r in stats)
    sel = [r for r in stats if pattern in r["Name"]]
    lines = [f"# Kernels matching `{pattern}`", "", f"Command: `{cmd}`", "",
             "Per-kernel durations from `rocprofv3 --kernel-trace --stats` (microseconds; share of "
             "all kernel time in the run).", "",
             "| kernel | calls | avg us | min us | max us | share |", "|---|---|---|---|---|---|"]
    for r in sorted(sel, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs'])/1e3:.1f} | "
                     f"{float(r['MinNs'])/1e3:.1f} | {float(r['MaxNs'])/1e3:.1f} | "
                     f"{100*float(r['TotalDurationNs'])/total:.2f}% |")
    out = os.path.join(ROOT, "profiles", f"{name}.md")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ceiling", default=None)
    ap.add_argument("--serving", default=None)
    ap.add_argument("--kernels", default=None, help="stats dir: write a table of matching kernels")
    ap.add_argument("--name", default=None)
    ap.add_argument("--match", default="k_fold")
    ap.add_argument("--cmd", default="")
    ap.add_argument("--serving-cmd", default="python3 bench.py --workload sals-3way-1m-fp32 --serve-full")
    ap.add_argument("--ceiling-cmd", default="python3 bench.py --gather-ceiling")
    ap.add_argument("--stats")
    ap.add_argument("--workload")
    ap.add_argument("--stats-cmd")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--fetch-cmd", default="")
    ap.add_argument("--write-cmd", default="")
    ap.add_argument("--reads")
    ap.add_argument("--writes")
    ap.add_argument("--reads-cmd", default="")
    ap.add_argument("--dram")
    ap.add_argument("--dram-cmd", default="")
    ap.add_argument("--writes-cmd", default="")
    ap.add_argument("--bench-json", default=None, help="bench.py output line of the same build")
    ap.add_argument("--timed", type=int, default=0,
                    help="accumulation launches of the timed sweeps in the stats run")
    ap.add_argument("--last", type=int, default=0,
                    help="average only the last N accumulation launches of each counter run")
    args = ap.parse_args()
    if args.ceiling:
        write_ceiling(args.ceiling, args.ceiling_cmd)
        return
    if args.serving:
        write_serving(args.serving, args.serving_cmd)
        return
    if args.kernels:
        write_kernels(args.kernels, args.name or "kernels", args.cmd, args.match)
        return
    if not (args.stats and args.workload and args.stats_cmd):
        ap.error("--stats, --workload and --stats-cmd are required without --ceiling")

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
    lines += ["", f"All accumulation launches (k_accum*): {calls} calls, average {avg_us:.1f} us per "
              "launch (tuning trials included)."]
    t_us = None
    if args.timed:
        t_us = timed_launches(args.stats, args.timed)
        if t_us is not None:
            lines += ["", f"Timed sweeps of the same run (the last {args.timed} accumulation launches "
                      f"of its kernel trace): average {t_us:.1f} us per launch."]

    traffic = {"kernel_source_sha": kernel_source_hash(), "workload": args.workload}
    if args.reads and args.writes:
        rd = _last(_per_dispatch(args.reads, _is_accum), args.last)
        wr = _last(_per_dispatch(args.writes, _is_accum), args.last)
        rbytes = statistics.mean(d.get("TCC_EA0_RDREQ_32B_sum", 0) * 32 + d.get("TCC_EA0_RDREQ_64B_sum", 0) * 64
                                 + d.get("TCC_EA0_RDREQ_128B_sum", 0) * 128 for d in rd)
        wbytes = statistics.mean(d.get("TCC_EA0_WRREQ_64B_sum", 0) * 64 +
                                 (d.get("TCC_EA0_WRREQ_sum", 0) - d.get("TCC_EA0_WRREQ_64B_sum", 0)) * 32
                                 for d in wr)
        hits = statistics.mean(d.get("TCC_HIT_sum", 0) for d in wr)
        miss = statistics.mean(d.get("TCC_MISS_sum", 0) for d in wr)
        r128 = statistics.mean(d.get("TCC_EA0_RDREQ_128B_sum", 0) for d in rd)
        rall = statistics.mean(d.get("TCC_EA0_RDREQ_32B_sum", 0) + d.get("TCC_EA0_RDREQ_64B_sum", 0)
                               + d.get("TCC_EA0_RDREQ_128B_sum", 0) for d in rd)
        # the same counters for the calibration copy: 1 GiB each way
        crd = _copy_reading(args.reads, "TCC_EA0_RDREQ_128B_sum")
        traffic.update({"read_bytes_per_launch": rbytes, "write_bytes_per_launch": wbytes,
                        "bytes_per_launch": rbytes + wbytes, "launches_sampled": len(rd),
                        "l2_hits_per_launch": hits, "l2_misses_per_launch": miss,
                        "hit_rate": hits / max(hits + miss, 1.0),
                        "read_requests_128b_share": r128 / max(rall, 1.0),
                        "copy_128b_read_requests": crd})
        lines += ["", "## HBM-side traffic of the accumulation kernels (rocprofv3 --pmc)", "",
                  "Bytes are the L2's read requests of 32, 64 and 128 bytes and write requests of "
                  "32 and 64 bytes (TCC_EA0_*), i.e. lines that miss L2 (the 256 MB last-level "
                  "cache's hits included).", "",
                  f"Read-request command: `{args.reads_cmd}`", "",
                  f"Write-request / hit-rate command: `{args.writes_cmd}`", "",
                  f"Per accumulation launch (mean of the last {len(rd)} launches, the timed sweep): "
                  f"read {rbytes/1e9:.3f} GB, write {wbytes/1e9:.3f} GB, total {(rbytes+wbytes)/1e9:.3f} GB; "
                  f"{100 * r128 / max(rall, 1.0):.1f}% of read requests are whole 128-byte lines.",
                  "", f"L2 (TCC): {hits:.4g} hits, {miss:.4g} misses per launch, hit rate "
                  f"{100 * hits / max(hits + miss, 1):.1f}%."]
        if crd:
            lines += ["", f"Check: the 1 GiB calibration copy makes {crd:.4g} 128-byte read requests "
                      f"({crd * 128 / COPY_BYTES:.3f} GiB)."]
        if t_us:
            lines += ["", f"At the timed launches' average ({t_us:.1f} us): "
                      f"{(rbytes + wbytes) / 1e3 / t_us:.0f} GB/s of HBM-side traffic "
                      f"({100 * (rbytes + wbytes) / 1e3 / t_us / 8000:.1f}% of 8 TB/s), "
                      f"{miss / 1e3 / t_us:.1f} G L2-miss lines/s."]
    if args.dram:
        dr = _last(_per_dispatch(args.dram, _is_accum), args.last)
        drd = statistics.mean(d.get("TCC_EA0_RDREQ_DRAM_32B_sum", 0) * 32 for d in dr)
        dwr = statistics.mean(d.get("TCC_EA0_WRREQ_WRITE_DRAM_32B_sum", 0) * 32 for d in dr)
        traffic.update({"dram_destined_read_bytes_per_launch": drd,
                        "dram_destined_write_bytes_per_launch": dwr,
                        "dram_destined_bytes_per_launch": drd + dwr})
        lines += ["", "## Requests destined for DRAM", "", f"Command: `{args.dram_cmd}`", "",
                  f"Per accumulation launch: read {drd/1e9:.3f} GB, write {dwr/1e9:.3f} GB towards "
                  "DRAM (the memory controllers). The 256 MB last-level cache sits on that side, so "
                  "its hits are still counted: no counter here separates the bytes HBM itself moves."]
        if "bytes_per_launch" in traffic:
            lines += ["", f"Against the request-size count above: {(drd + dwr) / traffic['bytes_per_launch']:.4f} "
                      "of it is DRAM-destined."]
    if args.fetch and args.write:
        fk = statistics.mean(d["FETCH_SIZE"] for d in _last(_per_dispatch(args.fetch, _is_accum), args.last))
        wk = statistics.mean(d["WRITE_SIZE"] for d in _last(_per_dispatch(args.write, _is_accum), args.last))
        fc = _copy_reading(args.fetch, "FETCH_SIZE")
        wc = _copy_reading(args.write, "WRITE_SIZE")
        ffac = (COPY_BYTES / 1024) / fc if fc else 1.0
        wfac = (COPY_BYTES / 1024) / wc if wc else 1.0
        traffic.update({"fetch_size_bytes_per_launch": fk * 1024 * ffac + wk * 1024 * wfac,
                        "fetch_scale": ffac, "write_scale": wfac})
        lines += ["", "## FETCH_SIZE / WRITE_SIZE, calibrated", "",
                  f"FETCH_SIZE command: `{args.fetch_cmd}`", "", f"WRITE_SIZE command: `{args.write_cmd}`",
                  "", f"A 1 GiB device copy in the same runs reads FETCH_SIZE {fc} KiB (scale "
                  f"{ffac:.4f}) and WRITE_SIZE {wc} KiB (scale {wfac:.4f}); per accumulation launch: "
                  f"fetch {fk * 1024 * ffac / 1e9:.3f} GB, write {wk * 1024 * wfac / 1e9:.3f} GB "
                  "(the fetch scale is taken from a streaming copy of whole lines; applied to a "
                  "kernel whose reads are also whole 128-byte lines it agrees with the request count "
                  "above)."]
    if "bytes_per_launch" in traffic:
        with open(os.path.join(ROOT, "profiles", f"k_accum_{args.workload}_traffic.json"), "w") as f:
            json.dump(traffic, f, indent=1)
    if args.bench_json:
        with open(args.bench_json) as f:
            b = json.loads([l for l in f if l.startswith("{")][-1])
        rf = b["roofline"]
        lines += ["", "## bench.py line of the same build", "",
                  f"value {b['value']:.4g} {b['unit']}, {b['ms_per_step']:.1f} ms per sweep; "
                  f"accumulation kernels: average launch {rf['avg_launch_ms']:.3f} ms (HIP events), "
                  f"{rf['alg_bytes_per_launch']/1e9:.3f} GB algorithmic per launch "
                  f"({rf['alg_achieved']:.0f} GB/s, {100*rf['alg_frac']:.1f}% of 8 TB/s without cache credit)."]
        if rf.get("achieved"):
            lines += ["", f"Its bounded roofline: {rf['achieved']:.0f} GB/s of HBM-side traffic, frac "
                      f"{rf['frac']:.3f}; L2-miss lines at {rf['l2_miss_line_rate']['achieved_glines_s']:.1f} "
                      f"G/s, {rf['l2_miss_line_rate'].get('frac', 0):.2f} of the gather ceiling."]
            rm = rf.get("l2_request_model")
            if rm:
                lines += ["", f"Its L2 requests at the gather probe's rates ({rm['hits_per_launch']:.4g} "
                          f"hits at {rm['hit_glines_s']:.1f} G/s, {rm['misses_per_launch']:.4g} misses "
                          f"at {rm['miss_glines_s']:.1f} G/s) take {rm['model_ms']:.2f} ms: "
                          f"{rm['frac']:.2f} of the measured launch."]
    out = os.path.join(ROOT, "profiles", f"k_accum_{args.workload}.md")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out)


if __name__ == "__main__":
    main()
