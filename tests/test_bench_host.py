"""Host-side logic of bench.py (no GPU): the single-GPU contract, the hash
gate that reports the scan's HBM traffic only while the profiled sources are
unchanged, and the CPU share of the oracle baseline."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert not r.stdout.strip().startswith("{")


def _fake_tree(tmp_path, scan_src, hashes):
    csrc = tmp_path / "paper_1403_2136_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "scan.hip").write_bytes(scan_src)
    (csrc / "internal.h").write_bytes(b"// header\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "scan_kernel_toy.md").write_text(
        "# toy\n\n```\nscan sources sha256: %s\ntraffic bytes per launch: 12345\n```\n"
        % " ".join(hashes))


def test_traffic_follows_the_source_hashes(tmp_path, monkeypatch):
    src = b"// scan kernel v1\n"
    hs = [hashlib.sha256(src).hexdigest(), hashlib.sha256(b"// header\n").hexdigest()]
    _fake_tree(tmp_path, src, hs)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("toy") == 12345
    # an edited kernel source: the committed counters no longer describe it
    (tmp_path / "paper_1403_2136_amd" / "csrc" / "scan.hip").write_bytes(b"// scan kernel v2\n")
    assert bench.recorded_traffic("toy") is None
    # no summary for the workload
    assert bench.recorded_traffic("other") is None


def test_cpu_share(monkeypatch):
    info = {"affinity": 16, "cgroup_quota_cpus": 6.0, "nproc": 16}
    monkeypatch.delenv("OMP_NUM_THREADS", raising=False)
    assert bench.cpu_threads(info) == 6
    monkeypatch.setenv("OMP_NUM_THREADS", "4")
    assert bench.cpu_threads(info) == 4
    monkeypatch.delenv("OMP_NUM_THREADS", raising=False)
    assert bench.cpu_threads({"affinity": 8, "cgroup_quota_cpus": None, "nproc": 8}) == 8
