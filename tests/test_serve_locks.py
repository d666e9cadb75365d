"""Lock discipline of the server's host threads, checked by Clang's
thread-safety analysis at compile time.

The server's state shared between the callers' threads and its scheduler
thread is declared guarded by its mutex (csrc/lock_check.hpp annotations in
csrc/serve.hip), and the library is built with -Werror=thread-safety, so an
access without the mutex held does not compile.  These tests pin that the
check is on and effective: the build flags carry it, the server source
passes it, and the same source with one planted unlocked access - a read, a
write, a call of a function that needs the mutex - is rejected.  (A
ThreadSanitizer run of the live server is not possible on this ROCm stack:
the runtime must reserve its shared GPU address range where the sanitizer
keeps its shadow memory, and finds no device.)
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1105_2769_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

needs_hipcc = pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC),
                                 reason="no hipcc")


def flags():
    import sys

    sys.path.insert(0, os.path.join(HERE, ".."))
    from paper_1105_2769_amd import build_lib

    return build_lib.FLAGS


def check(src_text, tmp_path, name):
    """Host-pass syntax check of a serve.hip variant with the library's flags."""
    src = tmp_path / name
    src.write_text(src_text)
    r = subprocess.run([HIPCC, *flags(), "--cuda-host-only", "-fsyntax-only", "-I", CSRC,
                        str(src)], capture_output=True, text=True)
    return r.returncode, r.stderr


def serve_source():
    with open(os.path.join(CSRC, "serve.hip")) as f:
        return f.read()


def test_build_makes_lock_findings_errors():
    f = flags()
    assert "-Wthread-safety" in f and "-Werror=thread-safety" in f


@needs_hipcc
def test_server_source_passes(tmp_path):
    rc, err = check(serve_source(), tmp_path, "serve_ok.hip")
    assert rc == 0, err


ANCHOR = "    mb_status set_timeout(int32_t ms) {"
PLANTS = {
    "read": "    int64_t planted() { return next_id_; }\n",
    "write": "    void planted() { stats_.units += 1; }\n",
    "requires": "    void planted() { auto f = [&]() MB_REQUIRES(mu_) { return stop_; }; (void)f(); }\n",
}


@needs_hipcc
@pytest.mark.parametrize("kind", sorted(PLANTS))
def test_unlocked_access_is_rejected(kind, tmp_path):
    src = serve_source()
    assert src.count(ANCHOR) == 1
    rc, err = check(src.replace(ANCHOR, PLANTS[kind] + ANCHOR), tmp_path, f"serve_{kind}.hip")
    assert rc != 0
    assert "-Wthread-safety-analysis" in err and "requires holding mutex 'mu_'" in err, err
