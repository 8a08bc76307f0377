"""The C ABI from a plain C program (tests/c_client/qpe_client.c, built by
the package build next to libqpe.so): device memory, workspace and stream of
its own, the closed form of an exact-bit eigenphase (all probability on
m = k) in both forms, and the host-side error codes."""
import os
import subprocess

import pytest

from tests.libutil import ROOT, ensure_built

pytestmark = pytest.mark.gpu

CLIENT = os.path.join(ROOT, "tests", "c_client", "qpe_client")


def test_c_client():
    ensure_built()
    assert os.path.exists(CLIENT), "the C client is built with libqpe.so (paper_2507_17175_amd/build.py)"
    r = subprocess.run([CLIENT], capture_output=True, text=True, timeout=120)
    print(r.stdout, flush=True)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
