"""CPU builds with AddressSanitizer and UndefinedBehaviorSanitizer.

    python -m paper_2604_07980_amd.sanitize [outdir]

* the oracle (oracle/ocsr_oracle.c) with oracle/sanitize_driver.c, built with gcc;
* the host side of libocsr: csrc/api.hip compiled by hipcc with the sanitizers on its
  host code only (the device code is built as usual), linked with the other objects of
  the library into a separate shared object, and tests/native/host_abi_driver.cpp built
  with the same compiler and sanitizer runtime.

Each driver runs to completion or aborts at the first report. Nothing here runs on a
GPU: the host driver exercises the calls that work without one.
"""
from __future__ import annotations

import os
import subprocess
import sys

from . import build as lib_build

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE = os.path.join(ROOT, "oracle")
CLANGXX = "/opt/rocm/llvm/bin/clang++"
# the sanitizers are applied to host code only (never to device code)
HOST_SAN = "-Xarch_host -fsanitize=address,undefined -Xarch_host -fno-sanitize-recover=all".split()


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def build_oracle(outdir: str) -> str:
    exe = os.path.join(outdir, "oracle_sanitized")
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fopenmp", "-I", ORACLE, os.path.join(ORACLE, "ocsr_oracle.c"),
          os.path.join(ORACLE, "sanitize_driver.c"), "-lm", "-o", exe])
    return exe


def build_host(outdir: str) -> str:
    """The library with a sanitized host side, and the host driver linked to it."""
    os.makedirs(outdir, exist_ok=True)
    objs = []
    for src in sorted(os.listdir(lib_build.CSRC)):
        if not src.endswith(".hip"):
            continue
        path = os.path.join(lib_build.CSRC, src)
        obj = os.path.join(outdir, src + ".o")
        extra = HOST_SAN if src == "api.hip" else []
        _run([lib_build.HIPCC, *lib_build.FLAGS, *extra, "-c", path, "-o", obj])
        objs.append(obj)
    so = os.path.join(outdir, "libocsr_sanitized.so")
    _run([lib_build.HIPCC, "-shared", f"--offload-arch={lib_build.ARCH}", "-fPIC",
          "-fsanitize=address,undefined", *objs, "-o", so])
    exe = os.path.join(outdir, "host_abi_driver")
    _run([CLANGXX, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-I", lib_build.INCLUDE, os.path.join(ROOT, "tests", "native", "host_abi_driver.cpp"),
          so, f"-Wl,-rpath,{outdir}", "-o", exe])
    return exe


def run(exe: str) -> str:
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    return _run([exe], env=env).stdout


if __name__ == "__main__":
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(ROOT, "_build", "sanitized")
    os.makedirs(out, exist_ok=True)
    print(run(build_oracle(out)), end="")
    print(run(build_host(out)), end="")
