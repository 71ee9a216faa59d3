"""Host-side parts of the benchmark's contract: the one-GPU refusal and the
rule that a stage's measured HBM traffic is reported only while the kernel
source it was measured on is unchanged."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 1" in r.stderr
    assert r.stdout == ""


def test_traffic_is_reported_only_for_the_measured_source(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2605_06876_amd" / "csrc"
    csrc.mkdir(parents=True)
    shutil.copy(os.path.join(ROOT, "paper_2605_06876_amd", "csrc", "blend.hip"), csrc / "blend.hip")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("blend_bwd") is None   # no summary
    (tmp_path / "profiles").mkdir()
    summary = {"blend_bwd": {"source": "blend.hip", "source_sha256_16": bench.source_hash("blend_bwd"),
                             "bytes_per_launch": 123456789}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(summary))
    assert bench.measured_traffic("blend_bwd") == 123456789
    assert bench.measured_traffic("project") is None      # stage not in the summary
    with open(csrc / "blend.hip", "a") as f:
        f.write("\n// edited after the counters were taken\n")
    assert bench.measured_traffic("blend_bwd") is None


@pytest.mark.parametrize("stage", sorted(bench.KERNEL_SOURCES))
def test_every_stage_names_an_existing_source(stage):
    assert os.path.exists(os.path.join(ROOT, "paper_2605_06876_amd", "csrc", bench.KERNEL_SOURCES[stage]))
