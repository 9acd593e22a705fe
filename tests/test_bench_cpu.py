"""Host-side parts of the benchmark (CPU): the one-GPU guard, the oracle
baseline leg on a small frame, and the rule that HBM traffic is reported only
while the profiled kernel sources are unchanged."""

import hashlib
import os
import shutil
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2411_00991_amd import synth  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_cpu_baseline_on_a_small_frame():
    fr = synth.frame_beads_segments(64, seed=0)
    rho = np.maximum(np.asarray(fr.image, np.float32) - 100.0, 1.0)[None] / 2.0
    ls = np.full_like(rho, -1.0)
    out = bench.cpu_baseline(fr, rho, ls, 3, 11, 1, 0, 1000, budget_s=0.2)
    assert out["kind"] == "oracle" and out["unit"] == "pixel-updates/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert "64x64" in out["sample"]


def _fake_tree(tmp_path):
    csrc = tmp_path / "paper_2411_00991_amd" / "csrc"
    csrc.mkdir(parents=True)
    h = hashlib.sha256()
    for name in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_2411_00991_amd", "csrc", name), csrc / name)
        h.update((csrc / name).read_bytes())
    (tmp_path / "profiles").mkdir()
    return csrc, h.hexdigest()


def test_traffic_only_while_sources_match(tmp_path, monkeypatch):
    csrc, sha = _fake_tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("k_x", "w_y") is None                 # no profile
    (tmp_path / "profiles" / "k_x_w_y.md").write_text(
        "# k_x\n\ntraffic_bytes_per_launch: 1.5e8\ntraffic_source_sha256: %s\n" % sha)
    assert bench.counter_traffic("k_x", "w_y") == 1.5e8
    with open(csrc / bench.KERNEL_SOURCES[0], "a") as fh:            # the kernel changed since
        fh.write("\n")
    assert bench.counter_traffic("k_x", "w_y") is None


def test_timed_sweeps_are_post_burn_in():
    """Every warm-up and timed sweep runs at a sweep index >= burn_in, so the
    timed region includes the Welford and batch moments."""
    import argparse
    for settle, warmup in ((60, 2), (60, 5), (0, 0), (10, 1)):
        args = argparse.Namespace(settle=settle, warmup=warmup)
        burn_in, timed_from = bench.sweep_plan(args)
        assert burn_in == settle
        assert timed_from >= burn_in and timed_from == settle + warmup
