"""Throughput of SALS sweeps on one MI355X (gfx950).

One step is one sweep (outer iteration of Algorithm 1, arXiv:1410.5209) over
the whole synthetic tensor: ceil(K/C) splits x T_in inner iterations x N mode
passes.  The metric is nnz*C updates per second: every sweep folds each
(observed entry, column) pair into its row's update T_in times per mode, i.e.
nnz * K * T_in * N updates per sweep.

Default workload (the headline): the skewed 5-way tensor, mode lengths 1M,
5e8 Zipf(1.0) draws (4.99e8 entries after dropping repeated tuples), rank-20
ground truth plus N(0, 0.25^2) noise; K = 1000, lambda = 1, T_in = 1, C tuned
over {16, 32}; FP32 factors, residual and Gram accumulation, FP64 Cholesky
(a scaled version of the paper's synthetic S4, Table 5).  Inputs are
generated on the host and resident in HBM before timing starts.

Besides the fields of the JSON line, it reports:
  roofline     for the row-accumulation kernels (the ones that gather factor
               rows and build the Gram matrices): HBM-side bytes per launch
               from the committed rocprofv3 counter summary of the same
               kernel source (read, write and L2-miss requests by size), over
               the average launch time measured here with HIP events on the
               library's stream, against 8 TB/s; beside it the design-neutral
               algorithmic bytes (no cache credit) over the same time, and the
               L2-miss line rate against the measured random-gather ceiling
  cpu_baseline the FP64 oracle timed on the host cores (all of them, and one
               thread on a smaller sample) on one split of the same recipe
  extra        the 3-way workload (mode lengths 1M, 1e8 uniform entries,
               K = 100, C = 10, T_in = 2: the paper's S2 shape) timed the same way
  serving      fold-in of new mode-1 rows against the trained 3-way factors
               under Poisson arrivals: p50/p99 latency and solves/s, full rank
               (C = K) and CDTF x 3
Other modes: --gather-ceiling (the random 128-byte gather rate by table size),
--serve-full (>= 1e5 requests per rate after a 5 s warm-up), --als (C = K
sweeps), --c-sweep / --tin-sweep, --precision-compare.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "nnz·C updates/s per SALS/CDTF sweep, % HBM roofline; fold-in p50/p99 latency"
HEADLINE = "sals-5way-zipf-fp32"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1410_5209_amd/csrc/k_rows.inc.h", "paper_1410_5209_amd/csrc/k_rows_wide.inc.h",
                  "paper_1410_5209_amd/csrc/dev_common.h", "paper_1410_5209_amd/csrc/tf_internal.h",
                  "paper_1410_5209_amd/csrc/tf_api.hip"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _profile_json(name):
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def counters_for(workload: str):
    """The committed counter summary of the accumulation kernels on this
    workload, if it was taken from the current kernel source; else None."""
    t = _profile_json(f"k_accum_{workload}_traffic.json")
    if t is None or t.get("kernel_source_sha") != kernel_source_hash():
        return None
    return t


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info():
    info = {"nproc": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "NUMA node(s)", "Socket(s)", "Core(s) per socket",
                             "L3 cache"):
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(w, scale, C, reg_mode=0, scale_1t=None):
    """The oracle as it stands, on one split of the same recipe at 1/scale
    size (mode lengths and entries both divided by `scale`, so rows keep the
    full workload's mean length; K, C, T_in, lambda unchanged), with all host
    threads, and on a 1/scale_1t sample with one thread."""
    import synth
    from oracle import oracle as orc

    def one(sc, threads):
        r = w.replica(w.I // sc, w.nnz // sc, C=C)
        idx, x = synth.make_tensor(r)[:2]
        orc.set_threads(threads)
        o = orc.Oracle(r.dims, idx, x, r.K, r.lam, reg_mode)
        o.init_factors(2, True)
        cols = list(range(min(r.C, r.K)))
        t0 = time.perf_counter()
        o.split(cols, r.T_in)
        dt = time.perf_counter() - t0
        upd = idx.shape[0] * len(cols) * r.T_in * r.N
        del o
        return upd / dt, upd, dt, r, idx.shape[0]

    allc = os.cpu_count() or 1
    v, upd, dt, r, n = one(scale, allc)
    out = {"value": v, "unit": "nnz·C updates/s", "cores": allc, "kind": "oracle",
           "sample": f"one split (C={min(r.C, r.K)}, T_in={r.T_in}) of the same recipe at 1/{scale} size "
                     f"(mode lengths {r.dims[0]}, {n} entries, K={r.K}): {upd} updates in {dt:.2f} s "
                     f"on {allc} threads",
           "host": host_info()}
    if scale_1t:
        v1, upd1, dt1, r1, n1 = one(scale_1t, 1)
        out["one_thread"] = {"value": v1, "cores": 1,
                             "sample": f"one split at 1/{scale_1t} size ({n1} entries): {upd1} updates "
                                       f"in {dt1:.2f} s"}
    return out


def foldin_cpu_baseline(m, w, nreq=2000, sweeps=3):
    """The oracle's fold-in (full rank and CDTF x sweeps) on `nreq` requests of
    the serving recipe against the same trained factors, with one thread and
    with one request per host thread at a time (the oracle's fold-in is serial
    and reads the context only)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import synth
    from oracle import oracle as orc

    orc.set_threads(1)
    # a one-entry tensor of the same shape carries the trained factors
    o = orc.Oracle(w.dims, np.zeros((1, w.N), dtype=np.int32), np.ones(1), w.K, w.lam)
    for n in range(w.N):
        o.set_factor(n, m.factor(n))
    ptr, oidx, vals = synth.make_requests(w.dims, w.R, nreq, seed=synth.SEED_REQ + 7)
    reqs = [(oidx[ptr[q]:ptr[q + 1]], vals[ptr[q]:ptr[q + 1]]) for q in range(nreq)]
    allc = os.cpu_count() or 1
    out = {"kind": "oracle", "host": host_info(),
           "sample": f"{nreq} requests of the serving recipe (mean {ptr[-1] / nreq:.0f} entries), "
                     "solved offline (no arrival process)"}
    for name, fn in (("full-rank", lambda r: o.foldin_full(0, r[0], r[1])),
                     (f"cdtf x{sweeps}", lambda r: o.foldin_cdtf(0, r[0], r[1], sweeps))):
        t0 = time.perf_counter()
        for r in reqs[: max(nreq // 8, 1)]:
            fn(r)
        one = max(nreq // 8, 1) / (time.perf_counter() - t0)
        t0 = time.perf_counter()
        with ThreadPoolExecutor(allc) as ex:
            list(ex.map(fn, reqs))
        many = nreq / (time.perf_counter() - t0)
        out[name] = {"solves_per_s": many, "cores": allc, "one_thread_solves_per_s": one}
        log(f"oracle fold-in {name}: {one:.0f} solves/s on 1 thread, {many:.0f} on {allc}")
    del o
    return out


def roofline(ks, dt_s, workload, C):
    """Bounded HBM figure (counter bytes / live launch time), the algorithmic
    figure beside it, and the L2-miss line rate against the gather ceiling."""
    avg_ms = ks.total_ms / max(ks.launches, 1)
    alg_bpl = ks.alg_bytes / max(ks.launches, 1)
    alg_gbs = alg_bpl / 1e9 / (avg_ms / 1e3) if avg_ms > 0 else 0.0
    t = counters_for(workload)
    out = {"bound": "hbm",
           "kernel": ("k_accum_wide (gather + matrix-core Gram accumulation)" if C > 16 else
                      "k_accum (gather + Gram accumulation)"),
           "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None, "traffic": None,
           "launches": ks.launches, "avg_launch_ms": avg_ms,
           "kernel_share_of_sweep": ks.total_ms / (dt_s * 1000.0),
           "alg_bytes_per_launch": alg_bpl, "alg_achieved": alg_gbs,
           "alg_frac": alg_gbs / HBM_PEAK_GBS,
           "note": ("achieved = HBM-side bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, each "
                    "scaled by its reading for a 1 GiB copy; the L2's requests counted by size "
                    "agree; committed summary of this kernel source: lines that miss L2, so they "
                    "include the 256 MB last-level cache's hits) / average launch time measured "
                    "here; alg_* = design-neutral algorithmic bytes (every gathered factor row, "
                    "index and residual counted at its size each use, no cache credit) / the same "
                    "time, which exceeds the HBM peak when hot rows are served by L2")}
    if t is None:
        out["note"] += "; counter summary missing or from another kernel source: achieved unknown"
        return out
    # FETCH_SIZE + WRITE_SIZE per launch, each scaled by its reading for a
    # 1 GiB device copy; the L2's requests counted by size agree with it
    bpl = t.get("fetch_size_bytes_per_launch") or t["bytes_per_launch"]
    gbs = bpl / 1e9 / (avg_ms / 1e3)
    out.update({"achieved": gbs, "frac": gbs / HBM_PEAK_GBS, "traffic": bpl,
                "traffic_requests_by_size": t.get("bytes_per_launch"),
                "traffic_read": t.get("read_bytes_per_launch"),
                "traffic_write": t.get("write_bytes_per_launch"),
                "traffic_dram_destined": t.get("dram_destined_bytes_per_launch"),
                "l2_hit_rate": t.get("hit_rate")})
    ceil = _profile_json("gather_ceiling.json")
    miss = t.get("l2_misses_per_launch")
    if miss:
        rate = miss / (avg_ms / 1e3) / 1e9
        lr = {"achieved_glines_s": rate}
        if ceil:
            c = ceil["ceiling_glines_s"]
            lr.update({"ceiling_glines_s": c, "frac": rate / c, "ceiling_table": ceil["ceiling_table"]})
        out["l2_miss_line_rate"] = lr
    hits = t.get("l2_hits_per_launch")
    if miss and hits and ceil and ceil.get("hit_ceiling_glines_s"):
        # each L2 request charged at the probe's rate for its kind: a launch
        # that is bound by line requests takes hits / R_hit + misses / R_miss
        rh, rm = ceil["hit_ceiling_glines_s"], ceil["ceiling_glines_s"]
        model_ms = (hits / rh + miss / rm) / 1e9 * 1e3
        out["l2_request_model"] = {
            "hits_per_launch": hits, "misses_per_launch": miss, "hit_glines_s": rh,
            "miss_glines_s": rm, "model_ms": model_ms, "frac": model_ms / avg_ms,
            "note": "time the launch's L2 requests take at the gather probe's rates (hits at the "
                    "1 MiB table's, misses at the 1 GiB table's), over the measured launch time"}
    return out


def serve_bench(m, w, rates, seconds=2.0, min_requests=0, warmup_s=None, streams=4, max_batch=512):
    """Fold-in serving against the trained, resident factors: Poisson arrivals
    (exponential gaps) at each rate; request sizes Zipf(1.1) on [1, 5000];
    other-mode indices uniform; values from the training ground truth.
    Latency = submit -> row on the host.  Requests of the warm-up part of each
    schedule (the first 10%, or the first `warmup_s` seconds) are not counted."""
    import numpy as np

    import synth
    from paper_1410_5209_amd import tf

    out = []
    for method, name in ((tf.TF_FOLDIN_FULL, "full-rank"), (tf.TF_FOLDIN_CDTF, "cdtf x3")):
        srv = tf.tf_serve_open(m.ctx, tf.tf_serve_default_options(
            method=method, sweeps=3, streams=streams, max_batch=max_batch, mem_budget=2 << 30))
        for rate in rates:
            nw = int(rate * warmup_s) if warmup_s else int(rate * seconds) // 10
            nmeas = max(int(rate * seconds) - (0 if warmup_s else nw), int(min_requests))
            nreq = nw + nmeas
            ptr, oidx, vals = synth.make_requests(w.dims, w.R, nreq, seed=synth.SEED_REQ + int(rate))
            keep = [(np.ascontiguousarray(oidx[ptr[q]:ptr[q + 1]]),
                     np.ascontiguousarray(vals[ptr[q]:ptr[q + 1]])) for q in range(nreq)]
            reqs = [tf.make_request(a, b) for a, b in keep]
            arrival = np.cumsum(synth.exponential(synth.SEED_REQ, 100 + int(rate), nreq, float(rate)))
            t = tf.tf_serve_replay(srv, arrival[:nw], reqs[:nw])
            for q in t:
                tf.tf_serve_wait(srv, int(q), w.K)
            tf.tf_serve_reset_stats(srv)
            t = tf.tf_serve_replay(srv, arrival[nw:] - arrival[nw], reqs[nw:])
            for q in t:
                tf.tf_serve_wait(srv, int(q), w.K)
            r = tf.tf_serve_report(srv)
            out.append({"method": name, "rate_req_s": rate, "requests": int(r.completed),
                        "warmup_requests": nw, "p50_us": r.p50_us, "p90_us": r.p90_us,
                        "p99_us": r.p99_us, "p999_us": r.p999_us, "max_us": r.max_us,
                        "solves_per_s": r.solves_per_s, "mean_batch": r.mean_batch,
                        "busy_rejects": int(r.busy_rejects), "failed": int(r.failed),
                        "mean_request_nnz": float(np.diff(ptr[nw:]).mean())})
            log(f"serve {name} {rate}/s: {int(r.completed)} requests, p50 {r.p50_us:.0f} us "
                f"p99 {r.p99_us:.0f} us {r.solves_per_s:.0f} solves/s batch {r.mean_batch:.1f}")
        tf.tf_serve_close(srv)
    return out


def make_model(w, data, strategy=1, lane_nnz=2, reg_mode=0, col_order="fixed", prec=None,
               graph=False):
    from paper_1410_5209_amd import tf
    from paper_1410_5209_amd.model import SparseCP
    order_opt = tf.TF_ORDER_RANDOM if col_order == "random" else tf.TF_ORDER_FIXED
    return SparseCP(w.dims, data[0], data[1], w.K, w.lam, precision=prec or w.prec,
                    strategy=strategy, lane_nnz=lane_nnz, reg_mode=reg_mode, col_order=order_opt,
                    graph=graph)


def timed_sweeps(m, C, T_in, steps, warmup, label, events=True):
    """`steps` sweeps after `warmup` untimed ones; with `events`, every
    accumulation launch is also bracketed by HIP events (not possible inside
    a captured sweep graph)."""
    import torch
    for s in range(warmup):
        m.sweep(C, T_in)
        log(f"{label}: warmup sweep {s} done")
    torch.cuda.synchronize()
    m.profile(events)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        m.sweep(C, T_in)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ks = m.profile_read()
    m.profile(False)
    return dt, ks


def tune(m, w, cands):
    r = m.autotune(w.T_in, cands, tune_tiles=True)
    info = {"candidates": list(cands), "est_sweep_ms": [r.est_sweep_ms[q] for q in range(r.ncand)],
            "chosen_C": int(r.best_C), "lane_nnz": list(r.lane_nnz)[:w.N],
            "chunk_nnz": list(r.chunk_nnz)[:w.N], "persistent": list(r.persistent)[:w.N],
            "tune_ms": r.tune_ms}
    return int(r.best_C), info


def run_workload(w, args, steps, warmup, serve=False):
    """Generate, build, tune, time; returns the record and the serving list."""
    import torch

    import synth
    t0 = time.perf_counter()
    data = synth.make_tensor(w)
    log(f"{w.name}: generated {data[0].shape[0]} entries in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    m = make_model(w, data, args.strategy, args.lane_nnz, args.reg_mode, args.col_order,
                   graph=args.graph)
    torch.cuda.synchronize()
    log(f"{w.name}: tf_init {time.perf_counter() - t0:.1f} s")
    del data
    cands = [int(c) for c in args.autotune.split(",")] if args.autotune else \
        ([16, 32] if w.name == HEADLINE else [w.C])
    C, tinfo = (w.C, None) if args.no_tune else tune(m, w, cands)
    log(f"{w.name}: C={C}" + (f" (tuned in {tinfo['tune_ms']:.0f} ms)" if tinfo else ""))
    dt, ks = timed_sweeps(m, C, w.T_in, steps, warmup, w.name, events=not args.graph)
    loss, rmse = m.loss()
    ms = dt * 1000.0 / steps
    updates = m.nnz * w.K * w.T_in * w.N
    log(f"{w.name}: timed {steps} sweeps in {dt:.3f} s ({ms:.1f} ms/sweep); loss {loss:.6g} rmse {rmse:.6g}")
    rec = {"workload": w.name, "N": w.N, "dims": w.dims, "nnz": m.nnz, "K": w.K, "C": C,
           "T_in": w.T_in, "lambda": w.lam, "precision": w.prec, "autotune": tinfo,
           "strategy": args.strategy, "graph": bool(args.graph),
           "steps": steps, "warmup": warmup, "ms_per_step": ms, "value": updates / (ms / 1000.0),
           "roofline": (roofline(ks, dt, w.name, C) if not args.graph else
                        {"note": "not measured with --graph: a captured sweep holds no per-kernel "
                                 "events", "graph_sweeps": ks.graph_sweeps}),
           "loss_after": loss, "train_rmse_after": rmse}
    serving = None
    if serve and w.N == 3 and w.K <= 128:
        serving = serve_bench(m, w, [1000, 10000, 50000], args.serve_seconds,
                              streams=args.serve_streams, max_batch=args.serve_max_batch)
    m.close()
    del m
    torch.cuda.empty_cache()
    return rec, serving, C


def gather_ceiling():
    """Random 128-byte row gathers by table size (tf_probe_gather): the rate
    at which the GPU serves line requests that miss (large tables) or hit
    (4 MB, one XCD's L2) its L2."""
    import numpy as np
    import torch

    from paper_1410_5209_amd import tf
    waves, steps = 8192, 4096
    out = torch.empty(waves * 64, dtype=torch.float32, device="cuda")
    res = []
    for mb in (1, 2, 4, 32, 128, 256, 1024, 4096):
        rows = mb * (1 << 20) // 128
        table = torch.rand(rows * 32, dtype=torch.float32, device="cuda")
        tf.tf_probe_gather(table, rows, waves, steps, 1, out)     # warm-up (TLB, caches)
        t = [tf.tf_probe_gather(table, rows, waves, steps, 2 + r, out) for r in range(5)]
        ms = float(np.median(t))
        g = waves * 2 * steps / (ms / 1e3) / 1e9
        res.append({"table_mb": mb, "median_ms": ms, "glines_s": g, "gbytes_s": g * 128})
        log(f"gather {mb} MB table: {g:.1f} G lines/s ({g * 128:.0f} GB/s)")
        del table
    big = [r for r in res if r["table_mb"] == 1024][0]
    small = [r for r in res if r["table_mb"] == 1][0]
    return {"probe": "tf_probe_gather", "waves": waves, "rows_per_half_wave": steps,
            "tables": res, "ceiling_glines_s": big["glines_s"], "ceiling_table": "1 GiB",
            "hit_ceiling_glines_s": small["glines_s"], "hit_table": "1 MiB",
            "note": "random 128-byte rows, one coalesced load per half-wavefront, no index stream; "
                    "the 1 GiB table (far above the 8 x 4 MB of L2, above the 256 MB last-level "
                    "cache) gives the L2-miss line-request ceiling, the 1 MiB table (a quarter of "
                    "one XCD's L2) the rate of requests that hit L2"}


def c_tin_sweep(w, data, cs, tins, sweeps):
    """The split width C and inner-iteration count T_in varied on one
    workload: for each pair, a fresh model from the same seeded start (row
    tiles tuned for that C, not timed), `sweeps` timed sweeps, then the
    regularised loss and training RMSE."""
    import numpy as np
    import torch

    out = []
    for T_in in tins:
        for C in cs:
            if C > w.K or C > 128:
                continue
            m = make_model(w, data)
            if C <= 32:
                m.autotune(T_in, [C], tune_tiles=True)
            times = []
            for _ in range(sweeps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                m.sweep(C, T_in)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            loss, rmse = m.loss()
            med = float(np.median(times))
            rec = {"C": C, "T_in": T_in, "median_sweep_ms": 1e3 * med,
                   "upd_per_s": len(data[1]) * w.K * T_in * w.N / med,
                   "sweeps": sweeps, "loss": loss, "train_rmse": rmse}
            out.append(rec)
            log(f"C={C} T_in={T_in}: {1e3 * med:.1f} ms/sweep, train RMSE {rmse:.5f}")
            m.close()
            del m
            torch.cuda.empty_cache()
    return out


def precision_compare(w, data, sweeps):
    """Held-out test RMSE and sweep time of the plain FP32 form (one wavefront
    per row, default tiles) against the batched forms (skew-aware plan, tuned
    row tiles) in FP32 and BF16 storage, at the workload's C and at a tuned C.
    Every form trains from the same seeded start for `sweeps` sweeps; times
    are the median sweep."""
    import numpy as np
    import torch

    from paper_1410_5209_amd import tf
    from paper_1410_5209_amd.model import SparseCP

    idx, x, idx_t, x_t = data
    forms = (("fp32-plain", "f32", tf.TF_STRATEGY_PLAIN, None),
             ("fp32-batched", "f32", tf.TF_STRATEGY_SKEW, [w.C]),
             ("bf16-batched", "bf16", tf.TF_STRATEGY_SKEW, [w.C]),
             ("fp32-batched-tunedC", "f32", tf.TF_STRATEGY_SKEW, [w.C, 16, 32]),
             ("bf16-batched-tunedC", "bf16", tf.TF_STRATEGY_SKEW, [w.C, 16, 32]))
    out = {}
    for name, prec, strat, cands in forms:
        m = SparseCP(w.dims, idx, x, w.K, w.lam, precision=prec, strategy=strat)
        C = w.C
        if cands is not None:
            C = m.autotune(w.T_in, cands, tune_tiles=True).best_C
        times = []
        for _ in range(sweeps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m.sweep(C, w.T_in)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        pred = m.predict(idx_t)
        rmse = float(np.sqrt(np.mean((pred - x_t) ** 2)))
        loss, train_rmse = m.loss()
        med = float(np.median(times))
        out[name] = {"C": C, "test_rmse": rmse, "train_rmse": train_rmse, "loss": loss,
                     "median_sweep_ms": 1e3 * med, "sweeps": sweeps,
                     "upd_per_s": len(x) * w.K * w.T_in * w.N / med}
        log(f"{name}: C={C} test RMSE {rmse:.6f}, median sweep {1e3 * med:.1f} ms")
        m.close()
        del m
        torch.cuda.empty_cache()
    base = out["fp32-plain"]
    for v in out.values():
        v["speedup_vs_fp32_plain"] = base["median_sweep_ms"] / v["median_sweep_ms"]
        v["test_rmse_minus_fp32_plain"] = v["test_rmse"] - base["test_rmse"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--strategy", type=int, default=1, choices=[0, 1, 2, 3],
                    help="row plan: 0 plain, 1 skew-aware, 2 skew-aware with tiles timed, 3 persistent")
    ap.add_argument("--lane-nnz", type=int, default=2)
    ap.add_argument("--graph", action="store_true",
                    help="sweeps captured as HIP graphs and replayed (tf_options.graph)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", default=None,
                    help="comma-separated candidate C values (default: 16,32 for the 5-way "
                         "workload, the workload's C otherwise)")
    ap.add_argument("--cpu-scale", type=int, default=0,
                    help="oracle sample at 1/scale size (default 40 for the 5-way workload, else 4)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 3-way workload and its serving runs after the headline")
    ap.add_argument("--extra-steps", type=int, default=10)
    ap.add_argument("--no-serve", action="store_true", help="skip the fold-in serving runs")
    ap.add_argument("--no-tune", action="store_true", help="use the default row tiles and C")
    ap.add_argument("--reg-mode", type=int, default=0, choices=[0, 1],
                    help="1: weighted lambda (lambda times the row's entry count)")
    ap.add_argument("--col-order", default="fixed", choices=["fixed", "random"],
                    help="random: a seeded column permutation per sweep")
    ap.add_argument("--c-sweep", default=None,
                    help="comma-separated C values: time and accuracy per (C, T_in) pair")
    ap.add_argument("--tin-sweep", default="1", help="comma-separated T_in values for --c-sweep")
    ap.add_argument("--precision-compare", action="store_true",
                    help="with a held-out workload: BF16 vs FP32 test RMSE and sweep time")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-max-batch", type=int, default=512)
    ap.add_argument("--serve-full", action="store_true",
                    help="serving only, on the 3-way workload: >= 1e5 requests per rate after a "
                         "5 s warm-up at that rate")
    ap.add_argument("--gather-ceiling", action="store_true",
                    help="the random 128-byte gather rate by table size")
    ap.add_argument("--als", action="store_true",
                    help="sweeps with C = K (the ALS row solve, eq. (ALS)) on the workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the row-sharded multi-GPU design is described, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth

    torch.cuda.set_device(0)
    if args.gather_ceiling:
        print(json.dumps({"gather_ceiling": gather_ceiling()}), flush=True)
        return
    w = synth.WORKLOADS[args.workload]
    if args.c_sweep or args.precision_compare or args.serve_full or args.als:
        t0 = time.perf_counter()
        data = synth.make_tensor(w)
        log(f"generated {data[0].shape[0]} entries in {time.perf_counter() - t0:.1f} s")
        if args.c_sweep:
            res = c_tin_sweep(w, data, [int(c) for c in args.c_sweep.split(",")],
                              [int(t) for t in args.tin_sweep.split(",")], w.sweeps)
            print(json.dumps({"workload": w.name, "dims": w.dims, "nnz": int(len(data[1])), "K": w.K,
                              "lambda": w.lam, "c_tin_sweep": res}), flush=True)
        elif args.precision_compare:
            if len(data) != 4:
                raise SystemExit("--precision-compare needs a workload with a held-out split")
            print(json.dumps({"workload": w.name,
                              "precision_compare": precision_compare(w, data, w.sweeps)}), flush=True)
        elif args.als:
            m = make_model(w, data)
            del data
            dt, ks = timed_sweeps(m, w.K, 1, args.steps, args.warmup, f"{w.name} ALS")
            loss, rmse = m.loss()
            ms = dt * 1000.0 / args.steps
            print(json.dumps({"workload": w.name, "als": {"C": w.K, "T_in": 1, "ms_per_sweep": ms,
                                                          "upd_per_s": m.nnz * w.K * w.N / (ms / 1e3),
                                                          "loss": loss, "train_rmse": rmse}}),
                  flush=True)
            m.close()
        else:
            m = make_model(w, data)
            del data
            C = w.C
            m.autotune(w.T_in, [C], tune_tiles=True)
            for s in range(4):
                m.sweep(C, w.T_in)
            log("trained 4 sweeps; serving")
            res = serve_bench(m, w, [1000, 10000, 50000], seconds=0.0, min_requests=100_000,
                              warmup_s=5.0, streams=args.serve_streams, max_batch=args.serve_max_batch)
            cpu = foldin_cpu_baseline(m, w)
            print(json.dumps({"workload": w.name, "serving_full": res, "cpu_baseline": cpu}),
                  flush=True)
            m.close()
        return

    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    head, serving, C = run_workload(w, args, args.steps, args.warmup,
                                    serve=(not args.no_serve and w.name != HEADLINE))
    extra = None
    if w.name == HEADLINE and not args.no_extra:
        w3 = synth.WORKLOADS["sals-3way-1m-fp32"]
        extra, serving, _ = run_workload(w3, args, args.extra_steps, 2, serve=not args.no_serve)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on one split")
        scale = args.cpu_scale or (40 if w.N == 5 else 4)
        cpu = cpu_baseline(w, scale, C, args.reg_mode, scale_1t=scale * 10)

    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "nnz·C updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "bf16": "bf16-storage/f32"}[w.prec],
        "data": "synthetic",
        "config": {"workload": w.name, "N": w.N, "dims": w.dims, "nnz": head["nnz"], "K": w.K,
                   "C": head["C"], "autotune": head["autotune"], "T_in": w.T_in, "lambda": w.lam,
                   "precision": w.prec, "reg_mode": args.reg_mode, "col_order": args.col_order,
                   "strategy": {0: "plain", 1: "skew", 2: "auto", 3: "persistent"}[args.strategy],
                   "parallelism": "single-gpu"},
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "extra": {extra["workload"]: extra} if extra else None,
        "serving": serving,
        "loss_after": head["loss_after"],
        "train_rmse_after": head["train_rmse_after"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
