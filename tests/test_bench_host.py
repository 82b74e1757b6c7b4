"""bench.py's host logic, without a GPU: the measured-traffic lookup takes a
committed counter record only for the exact kernel source and workload it was
taken on, and scales the counters as recorded; a run on more than one GPU is
refused before anything touches a device."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KEY = "full/fp32/scale=1.0/steps=20/warmup=5/engine=tiled/dc=0/budget=0/init=relaxed"


def _record(sha, key, fetch=1000.0, ffac=2.0, write=500.0, wfac=1.0, launches=2):
    return (f"traffic-record: kernels.hip sha256 {sha}; workload {key}; fetch KiB {fetch}; "
            f"fetch factor {ffac}; write KiB {write}; write factor {wfac}; launches {launches}\n")


def _setup(tmp_path, monkeypatch, lines):
    src = tmp_path / "kernels.hip"
    src.write_bytes(b"// a kernel source\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k.md").write_text("# a summary\n\n" + "".join(lines(hashlib.sha256(src.read_bytes()).hexdigest())))
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    monkeypatch.setattr(bench, "PROFILES", str(prof))


def test_traffic_from_matching_record(tmp_path, monkeypatch):
    _setup(tmp_path, monkeypatch, lambda sha: [_record(sha, KEY)])
    assert bench.measured_traffic_per_launch(KEY) == (1000.0 * 2.0 + 500.0 * 1.0) * 1024 / 2


def test_traffic_null_for_other_source_or_workload(tmp_path, monkeypatch):
    _setup(tmp_path, monkeypatch, lambda sha: [_record("0" * 64, KEY), _record(sha, KEY.replace("steps=20", "steps=21"))])
    assert bench.measured_traffic_per_launch(KEY) is None


def test_traffic_takes_the_record_of_this_workload(tmp_path, monkeypatch):
    _setup(tmp_path, monkeypatch, lambda sha: [_record(sha, KEY.replace("fp32", "fp16"), fetch=9.0),
                                               _record(sha, KEY, fetch=4.0, launches=1)])
    assert bench.measured_traffic_per_launch(KEY) == (4.0 * 2.0 + 500.0) * 1024


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""
