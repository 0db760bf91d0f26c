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
    key = ("block_mr", "32x32x32x32", "mixed_bf16")
    assert key in bench.TRAFFIC
    entry = dict(bench.TRAFFIC[key])
    src = os.path.join(ROOT, "paper_1204_1306_amd", "csrc", entry["source"])
    assert os.path.exists(src)
    # a figure whose recorded hash does not match the source reads as unmeasured
    monkeypatch.setitem(bench.TRAFFIC, key, dict(entry, sha256="0" * 64))
    assert bench.traffic_for(*key) is None
    # an unknown key is unmeasured too
    assert bench.traffic_for("no_such_family", "8x8x8x8", "mixed") is None


def test_block_sweep_flops_counts_the_in_block_hops():
    """The sweep flop model against hops counted site by site on a small geometry."""
    import itertools

    L, b = (8, 4, 4, 8), (4, 2, 2, 4)
    n_in = n_out = 0
    for x in itertools.product(*(range(v) for v in L)):
        for mu in range(4):
            for d in (+1, -1):
                y = (x[mu] + d) % L[mu]
                if y // b[mu] == x[mu] // b[mu] and abs(y - x[mu]) == 1:
                    n_in += 1
                else:
                    n_out += 1
    V = 8 * 4 * 4 * 8
    cycles, iters, nprop, nrhs = 3, 5, 2, 3
    n = (iters + 1) // 2
    face = (2 * cycles - 1) / (2 * cycles)
    per_site = (bench.HOP_FLOPS * n_in / V * (n + 1) + 192.0 * n + bench.HOP_FLOPS * n_out / V * face)
    want = V / 2 * nprop * nrhs * per_site
    got = bench.block_sweep_flops(L, b, nprop, nrhs, cycles, iters)
    assert abs(got - want) <= 1e-9 * want
