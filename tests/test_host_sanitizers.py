"""The host part of the library (hierarchy construction: level planning,
fine and Galerkin stencils, centre-block and coarsest inverses) built with
g++ under AddressSanitizer and UndefinedBehaviorSanitizer and run on grid
shapes the tests and workloads use: no memory or UB error, K symmetric on
every level, wall rows zero, centre inverses exact, the coarsest inverse
symmetric, uncoarsenable shapes refused, and the packed stencils the coarse
kernels read: the entries they leave out (cross-component couplings at a
zero offset along one of the components, zero in exact arithmetic) below
1e-14 of the largest on every level,
the kept ones in order, and a planted coupling refused."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_hierarchy_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "hierarchy_check"
    src = [os.path.join(ROOT, "tests", "host", "hierarchy_check.cpp"),
           os.path.join(ROOT, "paper_1904_03808_amd", "csrc", "hierarchy.cpp")]
    build = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                            "-fno-sanitize-recover=all", "-static-libasan", "-o", str(exe)] + src,
                           capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0 and run.stdout.strip().endswith("ok"), (run.stdout, run.stderr[-2000:])
