"""Host-side checks of bench.py's contract (no GPU needed).

* ``--gpus N`` with N > 1 exits with status 2 and a message, before touching
  torch or the GPU (one GPU only).
* ``roofline.traffic`` comes from the committed counter summary only while the
  dense kernel's source matches the sha256 recorded with the counters.
"""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_multi_gpu_exits_with_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_traffic_only_for_the_profiled_source(tmp_path, monkeypatch):
    src = tmp_path / "paper_2605_30267_amd" / "csrc" / "accsk_dense.hip"
    src.parent.mkdir(parents=True)
    src.write_text("// kernel source as profiled\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    (prof / "dense_solve_gmm8192_traffic.json").write_text(
        json.dumps({"source_sha256": sha, "hbm_bytes_per_launch": 1.5e10}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    traffic, info = bench.traffic_from_profile()
    assert traffic == 1.5e10 and info["source_sha256"] == sha
    src.write_text("// kernel source changed since the counters were taken\n")
    assert bench.traffic_from_profile() == (None, None)
    (prof / "dense_solve_gmm8192_traffic.json").unlink()
    assert bench.traffic_from_profile() == (None, None)
