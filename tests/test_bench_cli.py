"""The benchmark's command line outside the GPU: one GPU only, and the step
counts it refuses (both exit before any device work)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_bad_step_counts_are_refused():
    for args in (("--steps", "0"), ("--warmup", "-1"), ("--relax-steps", "-5"), ("--timing-steps", "0"),
                 ("--warmup-seconds", "-1")):
        r = _run(*args)
        assert r.returncode == 2, args
        assert "bench.py needs" in r.stderr and r.stdout == "", args
