"""Host logic of bench.py (no GPU): the one-GPU guard and the reader of the
stored traffic counters."""

import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_stored_traffic_follows_the_source(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    src = tmp_path / "k.hip"
    src.write_bytes(b"__global__ void k() {}\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    (tmp_path / "profiles" / "k_demo_traffic.txt").write_text(
        "# demo\nsource_sha256: %s\ntraffic_bytes: 12345\n" % sha)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.stored_traffic("k_demo", "k.hip") == 12345.0
    # no summary for the kernel
    assert bench.stored_traffic("k_other", "k.hip") is None
    # the kernel's source changed since the counters were taken
    src.write_bytes(b"__global__ void k() { }\n")
    assert bench.stored_traffic("k_demo", "k.hip") is None


def test_committed_traffic_summary_names_its_source():
    path = os.path.join(ROOT, "profiles", "k_sketch_csr_binned_traffic.txt")
    text = open(path).read()
    assert "source_sha256:" in text and "traffic_bytes:" in text
    assert "rocprofv3" in text  # the command that took the counters
