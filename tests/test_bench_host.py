"""Host-side logic of bench.py, without a GPU: the one-GPU refusal, the
algorithmic-byte count, the staleness rule of the recorded HBM traffic, and
the oracle's CPU-baseline legs."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2605_14743_amd import workloads as W  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr and out.stdout == ""


def test_algorithmic_bytes():
    st = {"sum_DK": 10, "sum_AK": 7, "sum_nK": 3}
    assert bench.algorithmic_bytes(st) == 8 * 10 + 32 * 7 + 64 * 3


def test_traffic_record_follows_the_kernel_sources(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2605_14743_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in bench.SWEEP_SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_2605_14743_amd", "csrc", name), csrc / name)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_record() is None                    # no record
    rec = {"kernel_source_sha256": bench.kernel_source_digest(), "sweep_bytes_per_launch": 1.0e9, "source": "x"}
    path = tmp_path / "profiles" / "sweep_wave_ws1000_R10000_traffic.json"
    path.write_text(json.dumps(rec))
    assert bench.traffic_record()["sweep_bytes_per_launch"] == 1.0e9
    (csrc / bench.SWEEP_SOURCES[-1]).write_text("// changed\n")
    assert bench.traffic_record() is None                    # sources changed since the counters


def test_committed_traffic_record_is_well_formed():
    path = os.path.join(ROOT, "profiles", "sweep_wave_ws1000_R10000_traffic.json")
    rec = json.load(open(path))
    assert len(rec["kernel_source_sha256"]) == 64 and rec["sweep_bytes_per_launch"] > 0


def test_cpu_baseline_legs():
    wl = W.config_er20()
    one = bench.cpu_baseline(wl, 0.2)
    assert one["kind"] == "oracle" and one["cores"] == 1 and one["value"] > 0
    many = bench.cpu_all_cores("er20", 2, 0.2)
    assert many["kind"] == "oracle" and many["cores"] == 2 and many["value"] > 0
