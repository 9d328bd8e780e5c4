"""The host-side tests of libkl (argument checks, layouts, wisdom selection,
capture files, and the malformed-input corpus of the two readers) run again
against a build whose host code carries AddressSanitizer and
UndefinedBehaviorSanitizer.  Any out-of-bounds access, use after free,
signed overflow or other undefined behaviour in the host code those tests
reach ends the run with a sanitizer report, and this test fails."""
import os
import subprocess
import sys

import pytest

import host_sanitizer_build as hsb

HERE = os.path.dirname(os.path.abspath(__file__))
HOST_TESTS = ["test_lib_host.py", "test_capture_host.py", "test_host_readers_fuzz.py"]


@pytest.mark.skipif(not os.path.exists(hsb.CLANG), reason="needs the ROCm clang++")
def test_host_code_under_address_and_ub_sanitizers():
    lib = hsb.build()
    env = dict(os.environ)
    env["KL_LIBRARY"] = lib
    env["LD_PRELOAD"] = " ".join(x for x in (hsb.runtime(), env.get("LD_PRELOAD", "")) if x)
    # leaks of the Python interpreter and of torch are not this library's
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PYTHONDONTWRITEBYTECODE"] = "1"
    probe = ("from paper_2303_12374_amd import kl; import ctypes; "
             "assert kl.LIB_PATH == %r; ctypes.CDLL(None).__asan_init; print('sanitized build loaded')" % lib)
    r = subprocess.run([sys.executable, "-c", probe], capture_output=True, text=True, env=env, timeout=300,
                       cwd=os.path.dirname(HERE))
    assert r.returncode == 0 and "sanitized build loaded" in r.stdout, r.stdout + r.stderr
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + \
          [os.path.join(HERE, t) for t in HOST_TESTS]
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=900, cwd=HERE)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out, out[-6000:]
    assert "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert " passed" in out
