"""Builds libqpe with AddressSanitizer and UndefinedBehaviorSanitizer on its
host code (the device code is compiled as usual, but nothing here launches
a kernel) and the plain-C driver tests/c_client/qpe_host_checks.c against
it, then runs the driver.

Used by a CPU test only; the GPU runs never build or load this copy.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

from paper_2507_17175_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(B.PKG, "_build_hostsan")
LIB = os.path.join(OUT, "libqpe_hostsan.so")
DRIVER_SRC = os.path.join(HERE, "c_client", "qpe_host_checks.c")
DRIVER = os.path.join(OUT, "qpe_host_checks")

SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)} failed:\n{msg}")
    return msg


def build() -> str:
    os.makedirs(OUT, exist_ok=True)
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(B.hipcc())))
    def compile_one(src):
        obj = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
        _run([B.hipcc(), "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={B.ARCH}", "-fvisibility=hidden",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", B.INCLUDE, "-I", B.CSRC] + SAN +
             ["-c", os.path.join(B.CSRC, src), "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(len(B.SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, B.SOURCES))
    _run([B.hipcc(), "-shared", "-fPIC", f"--offload-arch={B.ARCH}"] + SAN +
         ["-Xarch_host", "-shared-libasan", "-o", LIB] + objs)
    clang = os.path.join(rocm, "llvm", "bin", "clang")
    # the shared ASan runtime sits beside the compiler's own libraries
    rt = subprocess.run([clang, "-print-resource-dir"], capture_output=True, text=True).stdout.strip()
    rtdir = os.path.join(rt, "lib", "linux")
    _run([clang, "-O1", "-g", "-std=c11", "-Wall", "-Wextra", "-I", B.INCLUDE, "-I", os.path.join(rocm, "include"),
          "-D__HIP_PLATFORM_AMD__"] + SAN[1::2] + ["-shared-libasan", DRIVER_SRC, "-o", DRIVER, LIB,
          "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath," + OUT,
          "-Wl,-rpath," + os.path.join(rocm, "lib"), "-Wl,-rpath," + rtdir])
    return DRIVER


def run() -> subprocess.CompletedProcess:
    driver = build()
    env = dict(os.environ)
    # leaks of the HIP runtime's own start-up are not this code's
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return subprocess.run([driver], capture_output=True, text=True, env=env, timeout=600)
