"""The benchmark's contract on the CPU: one GPU only (other counts exit with a message), the
algorithmic operation count of the shading kernel, and the traffic summary taken only when it
was measured on the current kernel sources."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_ops_per_fragment():
    # per fragment: base 104 ops + 1 transcendental; each light adds its lobes and 15 transcendentals
    ops, trans = bench.alg_ops(1, 0, 0)
    assert (ops, trans) == (104, 1)
    ops, trans = bench.alg_ops(10, 1, 1)
    assert ops == 10 * (104 + 171 + 186) and trans == 10 * (1 + 2 * 15)
    # the figure the bench reports for the 1080p frame (25,244,783 fragments, one light of each kind)
    ops, trans = bench.alg_ops(25_244_783, 1, 1)
    assert int(ops + bench.TRANS_WEIGHT * trans) == 14_768_198_055


def test_traffic_only_for_the_measured_sources(tmp_path, monkeypatch):
    good = tmp_path / "good.txt"
    good.write_text(f"kernel = k\nkernel_hash = {bench.kernel_hash()}\nbytes_per_launch = 1234\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(good))
    assert bench.read_traffic() == 1234.0
    stale = tmp_path / "stale.txt"
    stale.write_text("kernel = k\nkernel_hash = 0000000000000000\nbytes_per_launch = 1234\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    assert bench.read_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.read_traffic() is None

