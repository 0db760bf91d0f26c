"""Host-side logic of bench.py (no GPU): the one-GPU contract and the traffic table."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_figures_follow_their_kernel_source(tmp_path, monkeypatch):
    key = ("block_mr", "8x8x8x8", "mixed")
    assert key in bench.TRAFFIC
    entry = dict(bench.TRAFFIC[key])
    src = os.path.join(ROOT, "paper_1204_1306_amd", "csrc", entry["source"])
    assert os.path.exists(src)
    # a figure whose recorded hash does not match the source reads as unmeasured
    monkeypatch.setitem(bench.TRAFFIC, key, dict(entry, sha256="0" * 64))
    assert bench.traffic_for(*key) is None
    # an unknown key is unmeasured too
    assert bench.traffic_for("no_such_family", "8x8x8x8", "mixed") is None
