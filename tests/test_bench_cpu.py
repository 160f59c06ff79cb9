"""CPU checks of bench.py's roofline arithmetic on stubbed counter summaries:
the bounded figure is counter bytes over the measured launch time, the line
rate is misses over that time, and the request model charges hits and misses
at the gather probe's two rates."""
import types

import pytest

import bench


def _ks(total_ms, launches, alg_bytes):
    return types.SimpleNamespace(total_ms=total_ms, launches=launches, alg_bytes=alg_bytes)


def test_roofline_from_counter_summary(monkeypatch):
    traffic = {"fetch_size_bytes_per_launch": 4.0e9, "bytes_per_launch": 4.1e9,
               "read_bytes_per_launch": 3.9e9, "write_bytes_per_launch": 0.2e9,
               "dram_destined_bytes_per_launch": 4.09e9, "hit_rate": 0.25,
               "l2_hits_per_launch": 1.0e7, "l2_misses_per_launch": 3.0e7}
    ceil = {"ceiling_glines_s": 50.0, "ceiling_table": "1 GiB", "hit_ceiling_glines_s": 200.0,
            "hit_table": "1 MiB"}
    monkeypatch.setattr(bench, "counters_for", lambda w: traffic)
    monkeypatch.setattr(bench, "_profile_json", lambda name: ceil)
    # 10 launches of 1 ms each, in a 20 ms sweep
    r = bench.roofline(_ks(10.0, 10, 10 * 6.0e9), 0.020, "w", 32)
    assert r["avg_launch_ms"] == pytest.approx(1.0)
    assert r["kernel_share_of_sweep"] == pytest.approx(0.5)
    assert r["achieved"] == pytest.approx(4000.0)                # 4 GB in 1 ms
    assert r["frac"] == pytest.approx(4000.0 / 8000.0)
    assert r["traffic"] == 4.0e9
    assert r["alg_achieved"] == pytest.approx(6000.0) and r["alg_frac"] == pytest.approx(0.75)
    lr = r["l2_miss_line_rate"]
    assert lr["achieved_glines_s"] == pytest.approx(30.0)         # 3e7 lines in 1 ms
    assert lr["frac"] == pytest.approx(0.6)
    rm = r["l2_request_model"]
    # 1e7 hits at 200 G/s = 0.05 ms, 3e7 misses at 50 G/s = 0.6 ms
    assert rm["model_ms"] == pytest.approx(0.65)
    assert rm["frac"] == pytest.approx(0.65)


def test_roofline_without_summary_reports_unknown(monkeypatch):
    monkeypatch.setattr(bench, "counters_for", lambda w: None)
    r = bench.roofline(_ks(4.0, 2, 8.0e9), 0.010, "w", 10)
    assert r["achieved"] is None and r["frac"] is None and r["traffic"] is None
    assert "l2_request_model" not in r and "l2_miss_line_rate" not in r
    assert r["alg_achieved"] == pytest.approx(2000.0)               # 4 GB per 2 ms launch
