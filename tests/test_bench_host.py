"""Host logic of bench.py (CPU only): the traffic figure read back from a
profile summary, and the one-GPU guard."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _tree(tmp_path, src=b"kernel v1", traffic="123456", note=" (a.hip)"):
    csrc = tmp_path / "paper_1903_10959_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "a.hip").write_bytes(src)
    prof = tmp_path / "profiles"
    prof.mkdir()
    h = hashlib.sha256(src).hexdigest()[:16]
    (prof / "k.md").write_text(f"# summary\n\ntraffic_bytes_per_launch: {traffic}\n"
                               f"kernel_source_sha256_16: {h}{note}\n")
    return csrc


def test_traffic_read_while_the_source_is_unchanged(tmp_path, monkeypatch):
    _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profiled_traffic("k", ("a.hip",)) == 123456.0
    # the note naming the hashed files is optional
    monkeypatch.setattr(bench, "ROOT", str(tmp_path / "x"))
    _tree(tmp_path / "x", note="")
    assert bench.profiled_traffic("k", ("a.hip",)) == 123456.0


def test_traffic_dropped_once_the_source_changes(tmp_path, monkeypatch):
    csrc = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (csrc / "a.hip").write_bytes(b"kernel v2")
    assert bench.profiled_traffic("k", ("a.hip",)) is None


def test_traffic_missing_profile_or_value(tmp_path, monkeypatch):
    _tree(tmp_path, traffic="n/a")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profiled_traffic("k", ("a.hip",)) is None
    assert bench.profiled_traffic("absent", ("a.hip",)) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
