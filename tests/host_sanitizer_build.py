"""A test build of libkl whose host code carries AddressSanitizer and
UndefinedBehaviorSanitizer: the host sources (argument checks, layout,
wisdom reader and selection, capture reader and writer, tuner driver) are
compiled for the CPU only with both sanitizers; the device translation units
are the objects of the ordinary build, unchanged.  Used by
test_host_sanitizers.py; nothing here runs on a GPU."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_12374_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")
OUT = os.path.join(BUILD, "host_san")
LIB = os.path.join(OUT, "libkl_host_san.so")
CLANG = "/opt/rocm/llvm/bin/clang++"
HOST_SOURCES = ("api.cpp", "capture.cpp", "tune.cpp", "wisdom.cpp")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def runtime() -> str:
    """Path of the shared AddressSanitizer runtime the test process preloads."""
    r = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True,
                       check=True)
    return r.stdout.strip()


def _host_object(name: str) -> str:
    obj = os.path.join(OUT, name + ".o")
    cmd = [CLANG, "-x", "c++", "-std=c++17", "-O1", "-g", "-fPIC", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"), "-I", CSRC] + SAN + \
          ["-c", os.path.join(CSRC, name), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
    return obj


def build() -> str:
    """Compile the host sources with the sanitizers and link them with the
    device objects of the ordinary build (compiling any that are missing)."""
    import sys
    sys.path.insert(0, ROOT)
    from paper_2303_12374_amd import build as kb
    os.makedirs(OUT, exist_ok=True)
    dev_srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(8) as ex:
        host = list(ex.map(_host_object, HOST_SOURCES))
        dev = []
        for src in dev_srcs:
            obj = os.path.join(BUILD, os.path.basename(src) + ".o")
            if not os.path.exists(obj) or os.path.getmtime(obj) < os.path.getmtime(src):
                dev.append(ex.submit(kb._compile, src))
            else:
                dev.append(obj)
        dev = [d if isinstance(d, str) else d.result() for d in dev]
    cmd = [CLANG, "-shared", "-fPIC", "-shared-libsan"] + SAN + ["-o", LIB] + host + dev + \
          ["-L/opt/rocm/lib", "-lamdhip64", "-lpthread", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    return LIB
