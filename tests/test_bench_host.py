"""Host logic of bench.py: the measured HBM traffic is reported only for the
counter record that matches the run (batch, launch setting, kernel source),
and the one-GPU rule."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_committed_record_is_used_only_for_its_kernels():
    path = os.path.join(ROOT, "profiles", "stage_bulk_traffic.json")
    with open(path) as fh:
        rec = json.load(fh)
    with open(os.path.join(ROOT, "paper_1905_08717_amd", "csrc", "kernels.hip"), "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    lg = rec["launch"]["list_grid"]
    want = rec["hbm_bytes_per_launch"] if rec["kernels_hip_sha256"] == digest else None
    assert bench.stage_traffic(rec["batch"], lg) == want
    # another batch, another grid: no figure
    assert bench.stage_traffic(rec["batch"] // 2, lg) is None
    assert bench.stage_traffic(rec["batch"], lg + 1) is None
    # it holds both counters, scaled, and their sum
    assert rec["hbm_bytes_per_launch"] == rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def test_record_of_other_kernel_source_is_ignored(tmp_path, monkeypatch):
    # a copy of the repository layout with a changed kernel source
    prof = tmp_path / "profiles"
    csrc = tmp_path / "paper_1905_08717_amd" / "csrc"
    prof.mkdir(parents=True)
    csrc.mkdir(parents=True)
    (csrc / "kernels.hip").write_bytes(b"// other source\n")
    rec = {"batch": 512, "launch": {"list_grid": 1536}, "hbm_bytes_per_launch": 123,
           "kernels_hip_sha256": "0" * 64}
    (prof / "stage_bulk_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "__file__", str(tmp_path / "bench.py"))
    assert bench.stage_traffic(512, 1536) is None
    rec["kernels_hip_sha256"] = hashlib.sha256(b"// other source\n").hexdigest()
    (prof / "stage_bulk_traffic.json").write_text(json.dumps(rec))
    assert bench.stage_traffic(512, 1536) == 123


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert "one GPU only" in (out.stdout + out.stderr)


def test_cpu_oracle_leg_reports_a_rate():
    # the CPU-baseline leg (the oracle timed in a process of its own) runs on
    # the host alone
    env = dict(os.environ, OMP_NUM_THREADS="2")
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--mode", "cpu-oracle",
                          "--cpu-seconds", "0.2"], capture_output=True, text=True, timeout=300, env=env)
    rec = json.loads(out.stdout.strip().splitlines()[-1])
    assert rec["threads"] == 2 and rec["leaf_updates_per_s"] > 0 and rec["macro_steps"] >= 1
    assert bench.cpu_model()
