"""CPU checks of the benchmark's contract pieces that need no GPU.

* More than one GPU is refused with a message and a non-zero exit (this build
  runs on one GPU).
* The HBM-traffic figure is reported only while the kernel sources hash to the
  value recorded with the counters, and is null otherwise.
"""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_traffic_only_for_the_profiled_kernel(tmp_path, monkeypatch):
    rec = json.load(open(bench.TRAFFIC_FILE))
    assert rec["kernel_source_hash"] == bench.kernel_source_hash()  # the committed record is current
    assert bench.traffic_entry() == rec["bytes_per_launch"]
    stale = dict(rec, kernel_source_hash="0" * 16)
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.traffic_entry() is None
