"""The serving chunk layout on the CPU.

tests/serve_sizes_check.cpp checks, for the tile shapes the exhaustive sum
can be built with and N from 3 to 4096, that the (i, j) table the table
kernel writes (its extent, from the blocks its launch fills) fits the table
region reserved in a request's device chunk for either tile type, and that
the chunk's parts do not overlap: the condition whose violation (a binary32
table outgrowing a region sized for the binary64 one) once made the serving
tests fault.  Built with the host compiler under AddressSanitizer and
UndefinedBehaviorSanitizer.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1105_2769_amd", "csrc")


def test_table_fits_its_region(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "serve_sizes_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", CSRC,
                    os.path.join(HERE, "serve_sizes_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("OK")
