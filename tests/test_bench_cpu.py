"""bench.py contract checks that need no GPU: one GPU only, and the JSON line's
fixed fields for the metric the bench reports."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_the_documented_flags():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup", "--workload", "--precision", "--to-accuracy", "--graph-iters"):
        assert flag in r.stdout, flag


def test_cpu_leg_of_the_block_sparse_workloads():
    # the oracle leg that bench.py runs in a child process beside the GPU legs
    import json
    import tempfile
    out = os.path.join(tempfile.mkdtemp(), "leg.json")
    env = dict(os.environ, OPENBLAS_NUM_THREADS="1", OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--cpu-leg", "cubic8_sparse", out, "1"],
                       capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stderr
    with open(out) as f:
        leg = json.load(f)
    assert leg["kind"] == "oracle" and leg["unit"] == "CG iters/s" and leg["cores"] == 1
    assert leg["value"] > 0 and "block-sparse form" in leg["sample"]
