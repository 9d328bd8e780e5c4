"""The served form's host logic (arena, admission in arrival order under
the budget, the tick loop with one tick in flight, ticket calls from
several client threads, a device error, shutdown with work queued) runs
against a host test double of the GPU executor (server_host_test.cpp),
built with g++ under AddressSanitizer + UndefinedBehaviorSanitizer and,
separately, under ThreadSanitizer.  No GPU is used."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(ROOT, "_build", "server_host")
SRC = os.path.join(HERE, "server_host_test.cpp")
SAN = {"asan_ubsan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
       "tsan": ["-fsanitize=thread"]}


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("san", sorted(SAN))
def test_server_logic_under_sanitizers(san):
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, f"server_host_{san}")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Werror"] + SAN[san] + \
          ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2303_12374_amd", "csrc"),
           SRC, "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert "Sanitizer" not in out and "runtime error" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert out.rstrip().endswith("ALL OK"), out[-2000:]
