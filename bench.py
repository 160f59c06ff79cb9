"""Throughput of SALS sweeps on one MI355X (gfx950).

One step is one sweep (outer iteration of Algorithm 1, arXiv:1410.5209) over
the whole synthetic tensor: ceil(K/C) splits x T_in inner iterations x N mode
passes.  The metric is nnz*C updates per second: every sweep folds each
(observed entry, column) pair into its row's update T_in times per mode, i.e.
nnz * K * T_in * N updates per sweep.

Default workload: 3-way tensor, 1M x 1M x 1M, 1e8 uniform entries (the shape
of the paper's synthetic S2), rank-20 ground truth mapped to [1, 5] plus
N(0, 0.25^2) noise; K = 100, lambda = 1, C = 10, T_in = 2; FP32 factors,
residual and Gram accumulation, FP64 Cholesky.  Inputs are generated on the
host and resident in HBM before timing starts.

Besides the JSON line fields the driver needs, it reports:
  serving      fold-in of new mode-0 rows against the trained factors under
               Poisson arrivals at 1k, 10k and 50k requests/s: p50/p99
               latency and solves/s, full rank (C = K) and CDTF x 3
  roofline     achieved algorithmic GB/s of the row-accumulation kernel (HIP
               events around each launch on the library's stream) vs 8 TB/s;
               traffic = DRAM bytes per launch from rocprofv3 counters when the
               counter file matches the current kernel source, else null
  cpu_baseline the FP64 oracle timed on the host cores (rank 0 only) on one
               split of the same recipe at quarter size (same row lengths)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "nnz·C updates/s per SALS/CDTF sweep, % HBM roofline; fold-in p50/p99 latency"
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


def traffic_per_launch(workload: str):
    """DRAM bytes per accumulation launch from the committed counter summary,
    if it was taken from the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"k_accum_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(w, scale=4, C=None, reg_mode=0):
    """The oracle as it stands, on one split of the same recipe at 1/scale size
    (mode lengths and entries both divided by `scale`, so every row keeps the
    full workload's mean length; K, C, T_in, lambda unchanged)."""
    import synth
    from oracle import oracle as orc
    r = w.replica(w.I // scale, w.nnz // scale, C=C or w.C)
    idx, x = synth.make_tensor(r)[:2]
    t0 = time.perf_counter()
    o = orc.Oracle(r.dims, idx, x, r.K, r.lam, reg_mode)
    o.init_factors(2, True)
    t_setup = time.perf_counter() - t0
    cols = list(range(min(r.C, r.K)))
    t0 = time.perf_counter()
    o.split(cols, r.T_in)
    dt = time.perf_counter() - t0
    updates = idx.shape[0] * len(cols) * r.T_in * r.N
    del o
    return {"value": updates / dt, "unit": "nnz·C updates/s", "cores": orc.get_threads(),
            "kind": "oracle",
            "sample": f"one split (C={len(cols)}, T_in={r.T_in}) of the same recipe at 1/{scale} size "
                      f"(mode lengths {r.dims}, {idx.shape[0]} entries, K={r.K}): {updates} updates in "
                      f"{dt:.2f} s; setup {t_setup:.1f} s untimed"}


def serve_bench(m, w, rates, seconds, streams, max_batch):
    """Fold-in serving against the trained, resident factors: Poisson arrivals
    (exponential gaps) at each rate; request sizes Zipf(1.1) on [1, 5000];
    other-mode indices uniform; values from the training ground truth.
    Latency = submit -> row on the host.  The first 10% of each schedule warms
    up and is not counted."""
    import numpy as np

    import synth
    from paper_1410_5209_amd import tf

    dims = w.dims
    out = []
    for method, name in ((tf.TF_FOLDIN_FULL, "full-rank"), (tf.TF_FOLDIN_CDTF, "cdtf x3")):
        srv = tf.tf_serve_open(m.ctx, tf.tf_serve_default_options(
            method=method, sweeps=3, streams=streams, max_batch=max_batch,
            mem_budget=2 << 30))
        for rate in rates:
            nreq = int(rate * seconds)
            ptr, oidx, vals = synth.make_requests(dims, w.R, nreq, seed=synth.SEED_REQ + int(rate))
            keep = [(np.ascontiguousarray(oidx[ptr[q]:ptr[q + 1]]),
                     np.ascontiguousarray(vals[ptr[q]:ptr[q + 1]])) for q in range(nreq)]
            reqs = [tf.make_request(a, b) for a, b in keep]
            arrival = np.cumsum(synth.exponential(synth.SEED_REQ, 100 + int(rate), nreq, float(rate)))
            nw = nreq // 10
            t = tf.tf_serve_replay(srv, arrival[:nw], reqs[:nw])
            for q in t:
                tf.tf_serve_wait(srv, int(q), w.K)
            tf.tf_serve_reset_stats(srv)
            t = tf.tf_serve_replay(srv, arrival[nw:] - arrival[nw], reqs[nw:])
            for q in t:
                tf.tf_serve_wait(srv, int(q), w.K)
            r = tf.tf_serve_report(srv)
            out.append({"method": name, "rate_req_s": rate, "requests": int(r.completed),
                        "p50_us": r.p50_us, "p90_us": r.p90_us, "p99_us": r.p99_us,
                        "p999_us": r.p999_us, "max_us": r.max_us, "solves_per_s": r.solves_per_s,
                        "mean_batch": r.mean_batch, "busy_rejects": int(r.busy_rejects),
                        "mean_request_nnz": float(np.diff(ptr).mean())})
            log(f"serve {name} {rate}/s: p50 {r.p50_us:.0f} us p99 {r.p99_us:.0f} us "
                f"{r.solves_per_s:.0f} solves/s batch {r.mean_batch:.1f}")
        tf.tf_serve_close(srv)
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
    dims = w.dims
    forms = (("fp32-plain", "f32", tf.TF_STRATEGY_PLAIN, None),
             ("fp32-batched", "f32", tf.TF_STRATEGY_SKEW, [w.C]),
             ("bf16-batched", "bf16", tf.TF_STRATEGY_SKEW, [w.C]),
             ("fp32-batched-tunedC", "f32", tf.TF_STRATEGY_SKEW, [w.C, 16, 32]),
             ("bf16-batched-tunedC", "bf16", tf.TF_STRATEGY_SKEW, [w.C, 16, 32]))
    out = {}
    for name, prec, strat, cands in forms:
        m = SparseCP(dims, idx, x, w.K, w.lam, precision=prec, strategy=strat)
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


def c_tin_sweep(w, data, cs, tins, sweeps):
    """The split width C and inner-iteration count T_in varied on one
    workload: for each pair, a fresh model from the same seeded start (row
    tiles tuned for that C, not timed), `sweeps` timed sweeps, then the
    regularised loss and training RMSE.  Columns above 32 per split are not
    run (the kernels take at most 32)."""
    import numpy as np
    import torch

    from paper_1410_5209_amd.model import SparseCP

    idx, x = data[0], data[1]
    out = []
    for T_in in tins:
        for C in cs:
            if C > w.K or C > 32:
                continue
            m = SparseCP(w.dims, idx, x, w.K, w.lam, precision=w.prec)
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
                   "upd_per_s": len(x) * w.K * T_in * w.N / med,
                   "sweeps": sweeps, "loss": loss, "train_rmse": rmse}
            out.append(rec)
            log(f"C={C} T_in={T_in}: {1e3 * med:.1f} ms/sweep, train RMSE {rmse:.5f}")
            m.close()
            del m
            torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sals-3way-1m-fp32")
    ap.add_argument("--strategy", type=int, default=1)
    ap.add_argument("--lane-nnz", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", default=None,
                    help="comma-separated candidate C values; the sweep then uses the tuned C "
                         "(default for the 5-way Zipf workload: 16,32)")
    ap.add_argument("--cpu-scale", type=int, default=0,
                    help="oracle sample at 1/scale size (default 4; 40 for the 5-way workload)")
    ap.add_argument("--no-serve", action="store_true", help="skip the fold-in serving runs")
    ap.add_argument("--no-tune", action="store_true", help="use the default row tiles")
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
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the row-sharded multi-GPU design is described, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1410_5209_amd import tf
    from paper_1410_5209_amd.model import SparseCP

    w = synth.WORKLOADS[args.workload]
    dims = w.dims
    t0 = time.perf_counter()
    data = synth.make_tensor(w)
    idx, x = data[0], data[1]
    log(f"generated {idx.shape[0]} entries in {time.perf_counter() - t0:.1f} s")

    torch.cuda.set_device(0)
    if args.c_sweep:
        res = c_tin_sweep(w, data, [int(c) for c in args.c_sweep.split(",")],
                          [int(t) for t in args.tin_sweep.split(",")], w.sweeps)
        print(json.dumps({"workload": w.name, "dims": w.dims, "nnz": int(len(data[1])), "K": w.K,
                          "lambda": w.lam, "c_tin_sweep": res}), flush=True)
        return
    if args.precision_compare:
        if len(data) != 4:
            raise SystemExit("--precision-compare needs a workload with a held-out split")
        res = precision_compare(w, data, w.sweeps)
        print(json.dumps({"workload": w.name, "precision_compare": res}), flush=True)
        return
    t0 = time.perf_counter()
    # random order: the library draws the columns of every sweep without
    # replacement (Algorithm 1), a seeded permutation per sweep
    order_opt = tf.TF_ORDER_RANDOM if args.col_order == "random" else tf.TF_ORDER_FIXED
    m = SparseCP(dims, idx, x, w.K, w.lam, precision=w.prec, strategy=args.strategy,
                 lane_nnz=args.lane_nnz, reg_mode=args.reg_mode, col_order=order_opt)
    torch.cuda.synchronize()
    log(f"tf_init {time.perf_counter() - t0:.1f} s")

    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # the tuner always picks the row tiles per mode; it also picks C when the
    # workload leaves C open (the 5-way Zipf workload)
    cands = None if args.no_tune else args.autotune or ("16,32" if w.name == "sals-5way-zipf-fp32" else str(w.C))
    C = w.C
    tune = None
    if cands:
        r = m.autotune(w.T_in, [int(c) for c in cands.split(",")], tune_tiles=True)
        C = r.best_C
        tune = {"candidates": [int(c) for c in cands.split(",")],
                "est_sweep_ms": [r.est_sweep_ms[q] for q in range(r.ncand)], "chosen_C": C,
                "lane_nnz": list(r.lane_nnz)[:w.N], "chunk_nnz": list(r.chunk_nnz)[:w.N],
                "tune_ms": r.tune_ms}
        log(f"autotune: C={C} ({r.tune_ms:.0f} ms)")

    def one_sweep(s):
        m.sweep(C, w.T_in)

    for s in range(args.warmup):
        one_sweep(s)
        log(f"warmup sweep {s} done")
    torch.cuda.synchronize()

    m.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        one_sweep(args.warmup + s)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ks = m.profile_read()
    m.profile(False)
    loss, rmse = m.loss()
    log(f"timed {args.steps} sweeps in {dt:.3f} s; loss {loss:.6g} rmse {rmse:.6g}")

    nnz = m.nnz
    ms = dt * 1000.0 / args.steps
    updates = nnz * w.K * w.T_in * w.N
    value = updates / (ms / 1000.0)
    avg_ms = ks.total_ms / max(ks.launches, 1)
    bytes_per_launch = ks.alg_bytes / max(ks.launches, 1)
    achieved = (ks.alg_bytes / 1e9) / (ks.total_ms / 1000.0) if ks.total_ms > 0 else 0.0
    traffic = traffic_per_launch(args.workload)
    serving = None
    if not args.no_serve and w.N == 3 and w.K <= 128:
        serving = serve_bench(m, w, [1000, 10000, 50000], args.serve_seconds, args.serve_streams,
                              args.serve_max_batch)
    m.close()
    del m
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on one split")
        del idx, x
        scale = args.cpu_scale or (40 if w.N == 5 else 4)
        cpu = cpu_baseline(w, scale, C, args.reg_mode)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "nnz·C updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "bf16": "bf16-storage/f32"}[w.prec],
        "data": "synthetic",
        "config": {"workload": w.name, "N": w.N, "dims": w.dims, "nnz": nnz, "K": w.K, "C": C,
                   "autotune": tune,
                   "T_in": w.T_in, "lambda": w.lam, "precision": w.prec,
                   "reg_mode": args.reg_mode, "col_order": args.col_order,
                   "strategy": "skew" if args.strategy == 1 else "plain",
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm",
                     "kernel": ("k_accum_wide (gather + MFMA Gram accumulation)" if C > 16 else
                                "k_accum (gather + Gram accumulation)"),
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_gbs": (traffic / 1e6 / avg_ms) if traffic else None,
                     "note": "achieved = algorithmic bytes (each gathered factor row and each "
                             "residual counted at its size, no cache credit) / kernel time; "
                             "traffic = DRAM-side bytes per launch from FETCH_SIZE + WRITE_SIZE",
                     "launches": ks.launches, "avg_launch_ms": avg_ms,
                     "alg_bytes_per_launch": bytes_per_launch,
                     "kernel_share_of_sweep": ks.total_ms / (dt * 1000.0)},
        "cpu_baseline": cpu,
        "serving": serving,
        "loss_after": loss,
        "train_rmse_after": rmse,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
