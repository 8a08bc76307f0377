"""Build libqpe.so (the HIP kernels and the C ABI) for gfx950, in-tree.

    python -m paper_2507_17175_amd.build [-v]

Every translation unit under csrc/ is compiled with hipcc in parallel and
linked into paper_2507_17175_amd/libqpe.so. Packed FP32 instructions are
disabled for the device code (-packed-fp32-ops).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libqpe.so")

SOURCES = [
    "qpe_capi.hip",
    "k_elementwise.hip",
    "k_zgemm_f64.hip",
    "k_ctrl_mixed.hip",
    "k_ctrl_small.hip",
    "k_qft.hip",
    "k_estimate.hip",
    "k_rotate.hip",
]

ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (set HIPCC or install ROCm)")


def compile_flags():
    return [
        "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-fvisibility=hidden", "-Wall", "-Wextra",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE, "-I", CSRC,
    ]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + compile_flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns that it does not know the packed-fp32 feature
    noise = "is not a recognized feature for this target"
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{msg}")
    if verbose and msg.strip():
        print(msg)
    return obj


CLIENT_SRC = os.path.join(ROOT, "tests", "c_client", "qpe_client.c")
CLIENT = os.path.join(ROOT, "tests", "c_client", "qpe_client")


def build_c_client(verbose: bool = False) -> str:
    """The plain C caller of the ABI that the tests run (gcc, linked against
    libqpe.so and the HIP runtime, found through an rpath)."""
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))
    cmd = [shutil.which("gcc") or "cc", "-O2", "-std=c11", "-Wall", "-Wextra", "-I", INCLUDE,
           "-I", os.path.join(rocm, "include"), "-D__HIP_PLATFORM_AMD__", CLIENT_SRC, "-o", CLIENT,
           "-L", PKG, "-lqpe", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_2507_17175_amd", "-Wl,-rpath," + os.path.join(rocm, "lib"), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"building the C client failed:\n{r.stdout}{r.stderr}")
    return CLIENT


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libqpe.so failed:\n{r.stdout}{r.stderr}")
    os.replace(tmp, LIB)
    build_c_client(verbose)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("-v", "--verbose", action="store_true")
    ap.add_argument("-j", "--jobs", type=int, default=0)
    a = ap.parse_args(argv)
    path = build(a.verbose, a.jobs)
    print(path)


if __name__ == "__main__":
    sys.exit(main())
