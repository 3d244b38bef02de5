"""Host logic of bench.py (no GPU): the roofline bound and fraction, the
gating of committed traffic records by the kernel source's SHA-256, and the
refusal of more than one GPU."""
import hashlib
import importlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture()
def bench(monkeypatch):
    # importing bench sets GPU_MAX_HW_QUEUES for its own process; keep this
    # process's environment as it was
    saved = dict(os.environ)
    sys.path.insert(0, ROOT)
    try:
        mod = importlib.import_module("bench")
    finally:
        sys.path.remove(ROOT)
        os.environ.clear()
        os.environ.update(saved)
    return mod


def test_roofline_bound_and_fraction(bench):
    # 10 launches in 1 ms: 1e-4 s each
    r = bench.roofline(2, 10, 1.0, 1e9, 1e6)          # intensity 1000 flop/B: above the ridge
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(1.0)          # 1e8 flop / 1e-4 s
    assert r["frac"] == pytest.approx(1.0 / bench.PEAK_FP64_TFLOPS)
    assert bench.roofline(0, 10, 1.0, 1e9, 1e6)["bound"] == "mfma"
    h = bench.roofline(1, 10, 1.0, 1e6, 1e6)           # intensity 1: HBM side
    assert h["bound"] == "hbm" and h["unit"] == "GB/s"
    assert h["achieved"] == pytest.approx(1.0)          # 1e5 B / 1e-4 s = 1 GB/s
    assert h["frac"] == pytest.approx(1.0 / bench.PEAK_HBM_GBS)
    assert h["avg_launch_us"] == pytest.approx(100.0)


def test_traffic_records_follow_the_kernel_source(bench, tmp_path, monkeypatch):
    src = tmp_path / "paper_2006_09314_amd" / "csrc" / "kernels.hip"
    src.parent.mkdir(parents=True)
    src.write_text("// kernel source, first version\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"kernel": "eigensolver", "hbm_bytes_per_launch": 1234.5,
           "kernel_source_sha256": digest}
    (prof / "traffic.md").write_text("summary\n\ntraffic-record: " + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("eigensolver") == (1234.5, "traffic.md")
    assert bench.recorded_traffic("panel_mgs_kernel") == (None, "no counter record")
    src.write_text("// kernel source, changed\n")
    value, note = bench.recorded_traffic("eigensolver")
    assert value is None and "stale" in note


def test_committed_profiles_carry_records(bench):
    recs = []
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            recs += [json.loads(l[len("traffic-record: "):]) for l in f
                     if l.startswith("traffic-record: ")]
    kernels = {r["kernel"] for r in recs}
    assert set(bench.KERNEL_NAMES.values()) <= kernels
    for r in recs:
        assert r["hbm_bytes_per_launch"] > 0 and len(r["kernel_source_sha256"]) == 64


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
