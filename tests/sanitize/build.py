"""Sanitizer builds for the CPU tests (test infrastructure, not the product).

* the library's host code (csrc/runtime.cpp, tune.cpp, server.cpp) with
  host-only stand-ins for the kernel launchers (kernel_stubs.cpp), built by
  g++ -- no HIP device code is compiled -- with AddressSanitizer and
  UndefinedBehaviorSanitizer, or with ThreadSanitizer;
* the C oracle with AddressSanitizer and UndefinedBehaviorSanitizer.

Outputs go to tests/sanitize/_build/. The tests load them through the
MHC_LIB_PATH / ORACLE_LIB_PATH environment variables in a subprocess that
preloads the sanitizer runtime.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2005_06773_amd", "csrc")
OUT = os.path.join(HERE, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

SANITIZERS = {"asan": "address,undefined", "tsan": "thread"}


def runtime_library(kind: str) -> str:
    """The sanitizer's runtime library to preload into a Python process."""
    name = {"asan": "libasan.so", "tsan": "libtsan.so"}[kind]
    return subprocess.run(["gcc", f"-print-file-name={name}"], check=True, capture_output=True,
                          text=True).stdout.strip()


def build_host_library(kind: str) -> str:
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, f"libmhc_host_{kind}.so")
    srcs = [os.path.join(CSRC, f) for f in ("runtime.cpp", "tune.cpp", "server.cpp")]
    srcs.append(os.path.join(HERE, "kernel_stubs.cpp"))
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-fno-omit-frame-pointer",
           f"-fsanitize={SANITIZERS[kind]}", "-fno-sanitize-recover=all", "-Wno-unused-result",
           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, "-pthread", "-o", lib, *srcs, "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return lib


def build_oracle() -> str:
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, "liboracle_asan.so")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-omit-frame-pointer",
           "-ffp-contract=off", "-fno-fast-math", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", lib, os.path.join(ROOT, "oracle", "mhc_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return lib


if __name__ == "__main__":
    for k in SANITIZERS:
        print(build_host_library(k))
    print(build_oracle())
