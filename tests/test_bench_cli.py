"""bench.py's command line on the CPU: more than one GPU is refused with a
message before anything touches a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "only --gpus 1" in (r.stdout + r.stderr)


def test_traffic_reported_only_for_the_measured_kernel(tmp_path):
    """A counter summary gives the line's `traffic` only while it names this
    workload and carries the hash of the kernel sources it was measured on."""
    import json
    sys.path.insert(0, ROOT)
    import bench

    path = tmp_path / "traffic.json"
    summary = {"config": "mid", "kernel_source_sha256_16": bench.kernel_source_hash(),
               "fetch_bytes_per_launch": 6.0e9, "write_bytes_per_launch": 2.0e9}
    path.write_text(json.dumps(summary))
    rate, t = bench.measured_traffic("mid", 1.0, str(path))
    assert rate == 8000.0 and t["config"] == "mid"   # 8 GB in 1 ms
    assert bench.measured_traffic("large", 1.0, str(path)) == (None, None)
    path.write_text(json.dumps(dict(summary, kernel_source_sha256_16="0" * 16)))
    assert bench.measured_traffic("mid", 1.0, str(path)) == (None, None)
    assert bench.measured_traffic("mid", 1.0, str(tmp_path / "missing.json")) == (None, None)


def test_committed_counter_summaries_name_their_workload():
    """Every committed summary parses and names a workload and a source hash."""
    import glob
    import json
    paths = glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json"))
    assert paths
    for p in paths:
        with open(p) as f:
            t = json.load(f)
        assert t["config"] and len(t["kernel_source_sha256_16"]) == 16
        assert t["fetch_bytes_per_launch"] > 0 and t["write_bytes_per_launch"] > 0
