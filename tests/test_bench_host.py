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


def test_counter_record_follows_the_kernel_and_planner_sources(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2605_14743_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in bench.KERNEL_SOURCES["sweep_wave"]:
        shutil.copy(os.path.join(ROOT, "paper_2605_14743_amd", "csrc", name), csrc / name)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_record("ws1000") is None                  # no record
    rec = {"kernel_source_sha256": bench.kernel_source_digest("sweep_wave"), "hbm_bytes_per_unit": 170.0,
           "valu_insts_per_unit": 17000.0, "lds_idx_active_per_unit": 8000.0}
    path = tmp_path / "profiles" / bench.COUNTER_RECORDS["ws1000"][1]
    path.write_text(json.dumps(rec))
    assert bench.counter_record("ws1000")["valu_insts_per_unit"] == 17000.0
    for name in ("wave_source.hpp", "amc_api.cpp", "query.cpp"):   # kernel and planner sources
        keep = (csrc / name).read_text()
        (csrc / name).write_text(keep + "// changed\n")
        assert bench.counter_record("ws1000") is None, name        # sources changed since the counters
        (csrc / name).write_text(keep)
        assert bench.counter_record("ws1000") is not None


def test_roofline_names_the_binding_resource():
    st = {"units": 10_000_000, "sum_DK": 10**10, "sum_AK": 10**10, "sum_nK": 10**10}
    rec = {"valu_insts_per_unit": 17000.0, "hbm_bytes_per_unit": 176.0, "lds_idx_active_per_unit": 8000.0,
           "lds_bank_conflict_per_unit": 3000.0, "source": "x"}
    r = bench.roofline(st, 400.0, rec)
    assert r["bound"] == "alu" and 0.0 < r["frac"] <= 1.0
    assert r["achieved"] == pytest.approx(17000.0 * 1e7 / 0.4 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.VALU_PEAK_GIPS)
    assert r["traffic"] == pytest.approx(176.0 * 1e7)
    assert r["hbm"]["frac"] < 1.0 and 0.0 < r["lds"]["frac"] < 1.0
    assert r["algorithmic"]["bytes_per_launch"] == bench.algorithmic_bytes(st)
    stale = bench.roofline(st, 400.0, None)
    assert stale["bound"] == "alu" and stale["frac"] is None and stale["traffic"] is None


def test_committed_counter_records_are_well_formed():
    found = 0
    for kernel, fname in bench.COUNTER_RECORDS.values():
        path = os.path.join(ROOT, "profiles", fname)
        if not os.path.exists(path):
            continue
        rec = json.load(open(path))
        assert len(rec["kernel_source_sha256"]) == 64 and rec["hbm_bytes_per_unit"] > 0
        assert rec["valu_insts_per_unit"] > 0
        found += 1
    if not found:
        pytest.skip("no counter record committed")


def test_cpu_baseline_all_cores():
    many = bench.cpu_baseline("er20", 2, 0.2)
    assert many["kind"] == "oracle" and many["cores"] == 2 and many["value"] > 0 and many["cpu_model"]
    assert 1 <= bench.cpu_cores() <= 16


def test_secondary_leg_failure_is_recorded():
    # a failing secondary leg leaves its error in the line instead of ending
    # the run before the headline is printed
    out = {}
    bench.secondary(out, "ok_leg", lambda: {"value": 1})

    def broken():
        raise RuntimeError("device says no")

    bench.secondary(out, "broken_leg", broken)
    assert out["ok_leg"] == {"value": 1}
    assert out["broken_leg"] == {"error": "RuntimeError: device says no"}
