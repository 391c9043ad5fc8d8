"""Host-side parts of the benchmark: the one-GPU guard and the rule that
the counted HBM traffic is reported only while the sources it was taken on
are unchanged."""
import json
import os
import shutil
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


FILES = ("csrc/step.hip", "csrc/internal.h", "csrc/api.hip", "build.py")


def _copy_sources(tmp_path):
    pkg = tmp_path / "paper_2101_09059_amd"
    (pkg / "csrc").mkdir(parents=True)
    for f in FILES:
        shutil.copy(os.path.join(ROOT, "paper_2101_09059_amd", f), pkg / f)
    (tmp_path / "profiles").mkdir()
    return pkg


def test_source_hash_follows_every_traffic_deciding_file(tmp_path, monkeypatch):
    pkg = _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.source_hash()
    assert h0 == bench.source_hash()
    for f in FILES:
        p = pkg / f
        text = p.read_text()
        p.write_text(text + "\n")
        assert bench.source_hash() != h0, f
        p.write_text(text)
        assert bench.source_hash() == h0


def test_traffic_is_reported_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    pkg = _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    key = "c2_cylinder:fused_step_f32apply_f64state"
    assert bench.measured_traffic("c2_cylinder", "fused_step_f32apply_f64state", 0) is None  # no file
    rec = {key: {"source_hash": bench.source_hash(), "bytes_per_launch": 123456789,
                 "bytes_per_launch_by_request_size": 120000000}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("c2_cylinder", "fused_step_f32apply_f64state", 0) == (123456789, 120000000)
    assert bench.measured_traffic("c4_batch", "fused_step_f32apply_f64state", 0) is None  # other workload
    p = pkg / "csrc" / "step.hip"
    p.write_text(p.read_text() + "// changed\n")
    assert bench.measured_traffic("c2_cylinder", "fused_step_f32apply_f64state", 0) is None


def test_committed_traffic_records_are_well_formed():
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert d
    for key, rec in d.items():
        workload, variant = key.split(":")
        assert workload and variant
        assert len(rec["source_hash"]) == 16
        assert rec["bytes_per_launch"] > 0
