"""The benchmark's command line on the host (no GPU work)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    """The path is measured on one GPU: --gpus N > 1 exits with a message."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_workloads_listed():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for name in ("deform3d", "shear3d", "tets"):
        assert name in r.stdout


def test_committed_profiles_are_read():
    """The benchmark reads the committed counter summaries of its default
    workload (128^3 deformation): both JSON lines parse and name the
    workload; taken on the current kernel sources, they give the register
    clip's HBM bytes and executed FP64 flops per (tet, cell) pair."""
    import json

    import pytest
    sys.path.insert(0, ROOT)
    import bench
    for prefix, tag in (("hbm_traffic", "traffic-json"), ("fp64_counters", "flops-json")):
        with open(os.path.join(ROOT, "profiles", f"{prefix}_deform3d_128.md")) as fh:
            line = next(ln for ln in fh if ln.startswith(tag + ":"))
        rec = json.loads(line.split(":", 1)[1])
        assert rec["workload"] == "deform3d" and rec["n"] == 128
        if rec["source_sha256_16"] != bench.kernel_source_hash():
            pytest.skip("the profiles were taken on other kernel sources")
    saved = list(bench.WORKLOAD)
    bench.WORKLOAD[:] = ["deform3d", 128]
    try:
        assert bench.recorded_traffic("clip") > 0
        per_pair, insts = bench.recorded_flops("clip", "clip_pairs")
        assert 100 < per_pair < 1000 and insts > 0
    finally:
        bench.WORKLOAD[:] = saved
