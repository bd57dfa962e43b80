"""Host logic of bench.py, without a GPU.

- The roofline entry of the dominant projector: achieved = algorithmic bytes
  (nnz x element size + outputs x element size) over the launch time, frac =
  achieved / 8000 GB/s, bound "hbm"; the committed rocprofv3 summary adds
  the measured traffic, the VALU issue rate, the gather pipe and the
  busiest limiter, but only while the profiled kernel source and launch-shape
  code match the current ones (digests).
- The exact workload counts it divides by are the oracle's (stored by
  tests/golden/make_workload_stats.py).
- More than one GPU is refused with a message, before anything touches a
  device.
"""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def stats():
    return json.load(open(os.path.join(ROOT, "tests", "golden", "workload_stats.json")))


def _counters(wl):
    return json.load(open(os.path.join(ROOT, "profiles", f"{wl}_counters.json")))


@pytest.mark.parametrize("wl,kname,es", [("muct1500", "forward", 2), ("muct1500", "backward", 2),
                                         ("medical256", "forward", 4), ("medical256", "backward", 4)])
def test_roofline_entry_arithmetic(bench, stats, wl, kname, es):
    s = stats[wl]
    n_out = s["rays"] if kname == "forward" else s["voxels"]
    units = s["nnz"] if kname == "forward" else s["voxel_views"]
    ms = 1234.5
    r = bench.roofline_entry(wl, kname, ms, s["nnz"], n_out, es, units)
    alg = s["nnz"] * es + n_out * es
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["algorithmic_bytes_per_launch"] == alg
    assert r["achieved"] == pytest.approx(alg / (ms / 1000.0) / 1e9, abs=0.05)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)
    # The counter fields, while the committed summary matches the current
    # kernel source and launch-shape code (after a kernel change the summary
    # is stale until the workload is profiled again).
    k = _counters(wl)["kernels"][kname]
    fresh = bench.counter_entry(wl, kname, bench.src_digest("proj_fwd.hip" if kname == "forward" else "proj_bwd.hip"))
    if fresh is None:
        assert r["traffic"] is None and "limiter" not in r
        pytest.skip(f"the {wl} {kname} counter summary predates the current sources")
    assert r["traffic"] == k["hbm_bytes_per_launch"]
    assert r["valu"]["insts_per_unit"] == pytest.approx(k["valu_insts_per_unit"], abs=1e-4)
    assert r["valu"]["frac"] == pytest.approx(k["valu_insts_per_unit"] * units / (ms / 1000.0) / 1e9 / 614.4,
                                              abs=1e-4)
    assert r["limiter"]["name"] in ("hbm", "valu_issue", "vector_memory_pipe")
    busiest = max(r["hbm_gbs_measured"] / 8000.0, r["valu"]["frac"], r["gather_pipe"]["td_busy"])
    assert r["limiter"]["busy"] == pytest.approx(busiest, abs=1e-4)


def test_stale_counters_are_not_reported(bench, stats, monkeypatch):
    """A summary taken on another kernel source or launch-shape code gives no
    traffic and no limiter."""
    s = stats["muct1500"]
    real = bench.src_digest
    monkeypatch.setattr(bench, "src_digest", lambda *names: "0" * 16 if names == ("api.hip",) else real(*names))
    r = bench.roofline_entry("muct1500", "forward", 2500.0, s["nnz"], s["rays"], 2, s["nnz"])
    assert r["traffic"] is None and "limiter" not in r and "valu" not in r
    assert bench.counter_entry("no_such_workload", "forward", "x") is None


def test_workload_counts_are_consistent(stats):
    """The stored counts hold together: every hit ray has at least one
    nonzero, voxel-views are voxels x angles, and the micro-CT workload's
    figures match its geometry (1571 angles of 2000^2 pixels, 1500^3 voxels)."""
    m = stats["muct1500"]
    assert m["rays"] == 1571 * 2000 * 2000 and m["voxels"] == 1500 ** 3
    assert m["voxel_views"] == m["voxels"] * 1571
    for s in stats.values():
        assert s["hit_rays"] <= s["rays"] and s["nnz"] >= s["hit_rays"]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert "one GPU only" in (r.stdout + r.stderr)
