"""CPU checks of bench.py's reporting contract: one GPU only, and HBM
traffic reported only while the committed counters match the W-build
sources they were taken on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_follows_the_source_hash(monkeypatch):
    t = bench.measured_traffic("wbuild_kernel<fp64>", "o40_v400")
    assert t is not None and 4.92e9 <= t <= 2 * 4.92e9   # at least the algorithmic bytes
    monkeypatch.setattr(bench, "wbuild_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("wbuild_kernel<fp64>", "o40_v400") is None
    assert bench.measured_traffic("wbuild_kernel<fp64>", "o99_v999") is None


def test_source_hash_covers_the_w_build_files(tmp_path, monkeypatch):
    h = bench.wbuild_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    csrc = tmp_path / "paper_2512_01055_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("te_device.h", "te_wbuild.hip"):
        (csrc / f).write_bytes(open(os.path.join(ROOT, "paper_2512_01055_amd", "csrc", f), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.wbuild_source_hash() == h
    (csrc / "te_wbuild.hip").write_bytes((csrc / "te_wbuild.hip").read_bytes() + b"\n")
    assert bench.wbuild_source_hash() != h
