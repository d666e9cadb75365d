"""The serving scheduler's queue logic on the CPU, with a fake executor.

tests/serve_sched_check.cpp drives the header-only scheduler with random
arrivals, sizes, slice limits and device-side rejections, and checks that
admission keeps arrival order, the budget and the slot limit, that every
unit of every request is handed out exactly once, and that every request
finishes and is released exactly once.  Built with the host compiler under
AddressSanitizer and UndefinedBehaviorSanitizer.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1105_2769_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("sched") / "serve_sched_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", CSRC,
                    os.path.join(HERE, "serve_sched_check.cpp"), "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("seed", range(1, 21))
def test_scheduler_invariants(checker, seed):
    r = subprocess.run([checker, str(seed)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("OK")
