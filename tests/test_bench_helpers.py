"""Host-side pieces of bench.py (no GPU): the one-GPU guard and the lookup of
HBM traffic recorded per schedule for the current kernel sources."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_traffic_lookup_by_schedule_and_source_hash(tmp_path):
    h = bench.kernel_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    rec = {"read_bytes": 2.0e9, "write_bytes": 1.0e8, "algorithmic_bytes": 4.0e8,
           "kernel_source_hash": h}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps({"strided_perm": {"f64": {"by_schedule": {
        "12": rec, "33": dict(rec, kernel_source_hash="0" * 16)}}}}))
    got = bench.load_traffic(str(path), "strided_perm", "f64", 12)
    assert got == {"read_bytes": 2.0e9, "write_bytes": 1.0e8, "algorithmic_bytes": 4.0e8,
                   "unit": "bytes/launch"}
    assert bench.load_traffic(str(path), "strided_perm", "f64", 14) is None   # not profiled
    assert bench.load_traffic(str(path), "strided_perm", "f64", 33) is None   # kernel changed
    assert bench.load_traffic(str(path), "strided_perm", "f32", 12) is None
    assert bench.load_traffic(str(path), "cc", "f64", 12) is None             # other workload
    assert bench.load_traffic(str(tmp_path / "missing.json"), "strided_perm", "f64", 12) is None
