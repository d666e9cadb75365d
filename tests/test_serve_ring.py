"""The serving drain ring's protocol on the CPU.

tests/serve_ring_check.cpp models the persistent drain kernel with host
threads (tickets from a shared counter, bounded idle waits, a collective
exit) against the host bookkeeping of csrc/serve_ring.hpp (publication,
consumption of done flags, republication of abandoned items after a kernel
ends, relaunch), with requests in reused slots whose descriptors the workgroups
cache by slot word (slot and generation).  It checks that every unit of
every request runs exactly once and with its own request's descriptor, with
one slot (consecutive requests share it) and with five.  Built with the host
compiler under ThreadSanitizer, then under AddressSanitizer and
UndefinedBehaviorSanitizer.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1105_2769_amd", "csrc")


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_ring_protocol(tmp_path, san):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "serve_ring_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-pthread", f"-fsanitize={san}",
                    "-fno-sanitize-recover=all", "-I", CSRC,
                    os.path.join(HERE, "serve_ring_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("OK"), r.stdout
