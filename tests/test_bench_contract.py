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


def _fake_tree(tmp_path, hash_):
    """A copy of the W-build sources and a counter summary taken on them."""
    csrc = tmp_path / "paper_2512_01055_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("te_device.h", "te_wbuild.hip"):
        (csrc / f).write_bytes(open(os.path.join(ROOT, "paper_2512_01055_amd", "csrc", f), "rb").read())
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "x.md").write_text(
        "traffic_bytes_per_launch: 6.1e9 kernel: wbuild_kernel<fp64> workload: o40_v400 "
        f"source_sha256_16: {hash_}\n")
    return csrc


def test_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    csrc = _fake_tree(tmp_path, bench.wbuild_source_hash())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("wbuild_kernel<fp64>", "o40_v400") == 6.1e9
    assert bench.measured_traffic("wbuild_kernel<fp64>", "o99_v999") is None
    (csrc / "te_wbuild.hip").write_bytes((csrc / "te_wbuild.hip").read_bytes() + b"\n")
    assert bench.measured_traffic("wbuild_kernel<fp64>", "o40_v400") is None


def test_committed_traffic_is_at_least_the_algorithmic_bytes():
    """Per W launch of the benchmark: ceil(65536 / tiles per triple) triples
    (3 GEMMs x ceil(v^2 / 128) x ceil(v / 80) tiles of 128 x 80), each with
    4.92e9 algorithmic bytes (six X slice reads, t2 panels, three W shares)."""
    v = 400
    tiles = 3 * -(-v * v // 128) * -(-v // 80)
    per_launch = -(-65536 // tiles)
    assert per_launch == 4
    t = bench.measured_traffic("wbuild_kernel<fp64>", "o40_v400")
    if t is not None:                      # counters taken on the current sources
        assert per_launch * 4.92e9 <= t <= 2 * per_launch * 4.92e9


def test_step_plan_covers_each_triple_once():
    """The timed steps are contiguous pieces of the triple list that together
    cover every triple exactly once, in order, for the driver's step counts
    and for degenerate ones."""
    for n, steps in ((11440, 20), (11440, 1), (11440, 7), (5, 5), (3, 8)):
        pieces = bench.step_slices(n, steps)
        assert len(pieces) == steps
        assert pieces[0][0] == 0 and pieces[-1][1] == n
        assert all(a <= b for a, b in pieces)
        assert all(pieces[q][1] == pieces[q + 1][0] for q in range(steps - 1))
        covered = [t for a, b in pieces for t in range(a, b)]
        assert covered == list(range(n))
    sizes = [b - a for a, b in bench.step_slices(11440, 20)]
    assert max(sizes) - min(sizes) <= 1


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
