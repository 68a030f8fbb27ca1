"""Host-side logic of bench.py: the counter-summary reader and the one-GPU guard."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_summary_tied_to_xengine_source(tmp_path):
    src = os.path.join(ROOT, "paper_1305_5639_amd", "csrc", "xengine.hip")
    h = bench.source_hash(src)
    f = tmp_path / "t.txt"
    f.write_text(f"xengine_source_sha256_16 = {h}\n"
                 "traffic_bytes_per_launch w/fp32 = 123456.0\n")
    assert bench.read_traffic(str(f), "w/fp32") == 123456.0
    assert bench.read_traffic(str(f), "w/fp16") is None
    f.write_text("xengine_source_sha256_16 = 0000000000000000\n"
                 "traffic_bytes_per_launch w/fp32 = 123456.0\n")
    assert bench.read_traffic(str(f), "w/fp32") is None          # stale: kernel changed
    assert bench.read_traffic(str(tmp_path / "missing.txt"), "w/fp32") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
