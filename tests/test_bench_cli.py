"""bench.py on the host: the one-GPU contract refuses other GPU counts before
touching a device, and every documented option parses."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "single MI355X" in r.stderr and r.stdout == ""


def test_help_lists_the_blocks():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for opt in ("--steps", "--warmup", "--no-512", "--no-steps", "--no-defect", "--no-table3",
                "--paper-run", "--explicit-only", "--table3-only", "--defect-only",
                "--profile-smoother", "--profile-solve", "--profile-solve-fp64", "--profile-step",
                "--chi-wall", "--min-coarse-nz"):
        assert opt in r.stdout, opt
