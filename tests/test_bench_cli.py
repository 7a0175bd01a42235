"""bench.py's command-line contract, checked without a GPU: it measures one
GPU only and says so for any other count."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_rejects_a_graph_chunk_out_of_range():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--graph-chunk", "0"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "--graph-chunk" in r.stderr
    assert r.stdout == ""


def test_bench_help_lists_the_workloads():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    assert "turbulence256" in r.stdout and "batch256" in r.stdout and "d3q39_192" in r.stdout


def test_traffic_counters_apply_only_to_the_sources_they_were_taken_on(tmp_path, monkeypatch):
    """bench.traffic_per_launch returns the committed FETCH+WRITE bytes only
    while the kernel sources hash to the value recorded with them."""
    import json

    import bench

    f = tmp_path / "traffic.json"
    json.dump({"source_hash": "abc", "traffic_bytes_per_launch": 123.0}, open(f, "w"))
    monkeypatch.setattr(bench, "traffic_file", lambda kernel, workload="turbulence256", dtype="fp32": str(f))
    monkeypatch.setattr(bench, "source_hash", lambda: "abc")
    assert bench.traffic_per_launch("scalar")[0] == 123.0
    monkeypatch.setattr(bench, "source_hash", lambda: "def")
    value, why = bench.traffic_per_launch("scalar")
    assert value is None and "changed" in why
    monkeypatch.setattr(bench, "traffic_file", lambda kernel, workload="turbulence256", dtype="fp32": str(tmp_path / "none.json"))
    assert bench.traffic_per_launch("scalar")[0] is None


def test_source_hash_covers_the_device_sources():
    import bench

    names = bench._kernel_sources()
    assert "csrc/step.hpp" in names and "csrc/step_batch.hpp" in names and "csrc/collide.hpp" in names
    assert "build.py" in names and "csrc/api.hip" not in names
    assert len(bench.source_hash()) == 16


def test_counted_traffic_rate_counts_every_step_of_a_launch():
    """bench.counted_rate divides a launch's counted bytes by the time of one
    launch: ms_per_step times the steps a launch takes (two for the two-step
    kernel), so the rate does not double when a launch covers two steps."""
    import bench

    one = {"ms_per_step": 0.5, "steps_per_launch": 1}
    two = {"ms_per_step": 0.25, "steps_per_launch": 2}
    gbs1, frac1 = bench.counted_rate(one, 2.0e9)
    gbs2, frac2 = bench.counted_rate(two, 2.0e9)
    assert abs(gbs1 - 4000.0) < 1e-9 and abs(gbs2 - 4000.0) < 1e-9
    assert abs(frac1 - 0.5) < 1e-12 and abs(frac2 - 0.5) < 1e-12
    assert bench.counted_rate(one, None) == (None, None)
