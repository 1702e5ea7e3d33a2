"""Host logic of bench.py (no GPU): the roofline's traffic figure is reported
only while the kernel sources are those the counters were taken on, the
instruction-mix model reads the committed rate table, and a run asked for
more than one GPU stops with a message before touching a device."""

import json
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_traffic_reported_at_the_profiled_sources():
    rec = json.load(open(os.path.join(ROOT, "profiles", "slice_kernel_traffic.json")))
    assert bench.counter_traffic() == float(rec["bytes_per_launch"])
    # counters close to the algorithmic bytes: no re-reads
    assert 1.0 <= rec["bytes_per_launch"] / rec["algorithmic_bytes_per_launch"] < 1.05


def test_traffic_dropped_when_a_kernel_source_changes(tmp_path, monkeypatch):
    rec = json.load(open(os.path.join(ROOT, "profiles", "slice_kernel_traffic.json")))
    for rel in rec["kernel_sources"] + ["profiles/slice_kernel_traffic.json"]:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, rel), dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic() == float(rec["bytes_per_launch"])
    src = tmp_path / rec["kernel_sources"][0]
    src.write_text(src.read_text() + "\n// edited\n")
    assert bench.counter_traffic() is None


def test_mix_model_reads_the_rate_table():
    rate = bench.mix_attainable()
    # the FP32C block's instruction mix at the measured per-class rates:
    # a little under the kernel's measured ~1.50e12 replica-steps/s
    assert rate is not None and 1.2e12 < rate < 1.6e12
    assert bench.OPS_FP32C == 23.0


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU only" in res.stderr
    assert res.stdout == ""
