"""The C ABI on the host: the library loads, exports every declared symbol,
and its argument checks return the documented status codes without a device."""
import ctypes
import os
import re

import pytest

from tests.libutil import ensure_built

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    ensure_built()
    from paper_2507_17175_amd import qpe
    return qpe.load_library()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "qpe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qpe_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    from paper_2507_17175_amd import qpe
    assert sorted(qpe.EXPORTS) == names


def test_status_strings(L):
    assert L.qpe_status_string(0) == b"QPE_OK"
    for s in range(1, 9):
        assert L.qpe_status_string(s).startswith(b"QPE_ERR_")
    assert b"unknown" in L.qpe_status_string(99)
    assert L.qpe_version() == b"0.1.0"


def _problems(shapes, ptr=0x10000):
    from paper_2507_17175_amd.qpe import Problem
    arr = (Problem * len(shapes))()
    for i, (n, t) in enumerate(shapes):
        arr[i].n_meas, arr[i].n_mat = n, t
        arr[i].U = arr[i].psi = arr[i].prob = ptr
    return arr


def test_workspace_size(L):
    out = ctypes.c_size_t()
    assert L.qpe_workspace_size(_problems([(8, 2)]), 1, 1, 0, ctypes.byref(out)) == 0
    small = out.value
    assert small >= 2 * 256 * 4 * 8
    assert L.qpe_workspace_size(_problems([(16, 10)]), 1, 1, 0, ctypes.byref(out)) == 0
    # two c64 state buffers of 2^26 amplitudes dominate
    assert out.value >= 2 * (1 << 26) * 8
    mixed = out.value
    assert L.qpe_workspace_size(_problems([(16, 10)]), 1, 0, 0, ctypes.byref(out)) == 0
    assert out.value > mixed  # complex128 state
    # batch: every instance gets its own region, plus launch tables and
    # descriptors in front of them
    assert L.qpe_workspace_size(_problems([(8, 2), (16, 10)]), 2, 1, 0, ctypes.byref(out)) == 0
    assert out.value >= mixed + small
    assert out.value <= mixed + small + (1 << 20)


def test_workspace_second_plane_set(L):
    """A single prefix-doubling run with split-FP16 products (mixed form with
    the polar step, d >= 32) holds a second set of operator planes, six
    d x d 16-bit planes, after its other regions; no other run does."""
    out = ctypes.c_size_t()

    def need(n, t, form, flags):
        assert L.qpe_workspace_size(_problems([(n, t)]), 1, form, flags, ctypes.byref(out)) == 0
        return out.value

    dbl, no_polar, bf16 = 2, 1, 16
    for n, t in [(9, 5), (13, 8), (16, 10)]:
        d = 1 << t
        extra = -(-6 * d * d * 2 // 256) * 256
        assert need(n, t, 1, dbl) - need(n, t, 1, 0) == extra
        assert need(n, t, 0, dbl) == need(n, t, 0, 0)
        assert need(n, t, 1, dbl | no_polar) == need(n, t, 1, no_polar)
        assert need(n, t, 1, dbl | bf16) == need(n, t, 1, bf16)
    assert need(9, 4, 1, dbl) == need(9, 4, 1, 0)


@pytest.mark.parametrize("n,t,code", [(0, 2, 2), (31, 2, 2), (8, -1, 2), (8, 16, 2), (30, 10, 2), (20, 14, 0)])
def test_size_limits(L, n, t, code):
    out = ctypes.c_size_t()
    assert L.qpe_workspace_size(_problems([(n, t)]), 1, 1, 0, ctypes.byref(out)) == code


def test_bad_form_flags_count(L):
    out = ctypes.c_size_t()
    assert L.qpe_workspace_size(_problems([(8, 2)]), 1, 2, 0, ctypes.byref(out)) == 1
    assert L.qpe_workspace_size(_problems([(8, 2)]), 1, 1, 32, ctypes.byref(out)) == 1
    # forcing the target rotation on (4) and off (8) at once
    assert L.qpe_workspace_size(_problems([(8, 2)]), 1, 1, 4 | 8, ctypes.byref(out)) == 1
    assert L.qpe_workspace_size(_problems([(8, 2)]), 0, 1, 0, ctypes.byref(out)) == 1
    assert L.qpe_workspace_size(None, 1, 1, 0, ctypes.byref(out)) == 1


def test_check_run(L):
    out = ctypes.c_size_t()
    p = _problems([(8, 2)])
    assert L.qpe_workspace_size(p, 1, 1, 0, ctypes.byref(out)) == 0
    need = out.value
    ws = 0x100000  # 256-aligned fake device address: never dereferenced
    assert L.qpe_check_run(p, 1, 1, 0, ws, need, None) == 0
    assert L.qpe_check_run(p, 1, 1, 0, ws, need - 1, None) == 4
    assert L.qpe_check_run(p, 1, 1, 0, ws + 16, need, None) == 4
    assert L.qpe_check_run(p, 1, 1, 0, None, need, None) == 4
    assert L.qpe_check_run(p, 1, 1, 0, ws, need, ws + 4) == 3
    # the target rotation forced on (4) or off (8), with or without the
    # polar step (1); both at once is an argument error
    for f in (4, 4 | 1, 8, 8 | 1):
        assert L.qpe_check_run(p, 1, 1, f, ws, need, None) == 0
    assert L.qpe_check_run(p, 1, 1, 4 | 8, ws, need, None) == 1
    assert L.qpe_check_run(p, 1, 1, 32, ws, need, None) == 1
    assert L.qpe_check_run(p, 1, 1, 16, ws, need, None) == 0  # QPE_SPLIT_BF16
    two = _problems([(8, 2), (8, 2)])
    for f in (4, 4 | 1):
        # a forced rotation adds launches (table entries) to a batch
        assert L.qpe_workspace_size(two, 2, 1, f, ctypes.byref(out)) == 0
        assert L.qpe_check_run(two, 2, 1, f, ws, out.value, None) == 0
        assert L.qpe_check_run(two, 2, 1, f, ws, out.value - 1, None) == 4
    bad = _problems([(8, 2)])
    bad[0].U = 0x10008
    assert L.qpe_check_run(bad, 1, 1, 0, ws, need, None) == 3
    bad[0].U = 0x10000
    bad[0].prob = 0x10004
    assert L.qpe_check_run(bad, 1, 1, 0, ws, need, None) == 3
    bad[0].prob = None
    assert L.qpe_check_run(bad, 1, 1, 0, ws, need, None) == 1
    assert L.qpe_check_run(p, 1, 7, 0, ws, need, None) == 1


def test_null_context(L):
    p = _problems([(8, 2)])
    assert L.qpe_run(None, p, 1, 1, 0, 0x100000, 1 << 30, None) == 1
    al = (ctypes.c_double * 2)(1.0, 0.0)
    assert L.qpe_zgemm(None, b"N", b"N", 4, 4, 4, al, 0x1000, 4, 0x1000, 4, al, 0x1000, 4, 0x1000, 4) == 1
    assert L.qpe_powers(None, 2, 0x1000, 3, 0, 0x1000, 0x100000, 1 << 20, None) == 1
    assert L.qpe_ctx_set_timing_mask(None, 1) == 1
    assert L.qpe_ctx_destroy(None) == 0
    assert L.qpe_last_error(None) == b""


def test_estimate_host_checks(L):
    out = ctypes.c_size_t()
    assert L.qpe_estimate_workspace_size(0, ctypes.byref(out)) == 1
    assert L.qpe_estimate_workspace_size(3, ctypes.byref(out)) == 0
    one = ctypes.c_size_t()
    assert L.qpe_estimate_workspace_size(1, ctypes.byref(one)) == 0
    assert out.value == 3 * one.value and one.value % 256 == 0 and one.value > 0
    p = _problems([(8, 0)])
    assert L.qpe_estimate(None, p, 1, 0x1000, 0x100000, 1 << 20) == 1


def test_autotune_and_variant_host_checks(L):
    chosen = (ctypes.c_int * 6)()
    p = _problems([(8, 5)])
    assert L.qpe_autotune(None, p, 1, 0, 0x100000, 1 << 30, 2, chosen, None) == 1
    v = ctypes.c_int()
    assert L.qpe_ctx_get_variant(None, 0, 5, ctypes.byref(v)) == 1
    pb = _problems([(8, 5), (9, 7)])
    assert L.qpe_autotune_batch(None, pb, 2, 1, 0, 0x100000, 1 << 30, 2, chosen, None) == 1
    # the controlled product (nine tile variants), the power-chain GEMM
    # (seven), and the batched classes: controlled step (three variants),
    # power-chain tiles and schedule (two each)
    for cls, nv in ((0, 9), (1, 7), (3, 3), (4, 2), (5, 2)):
        c = ctypes.c_int()
        assert L.qpe_kernel_variants(cls, ctypes.byref(c)) == 0 and c.value == nv
    c = ctypes.c_int()
    assert L.qpe_kernel_variants(6, ctypes.byref(c)) == 1


def test_stage_workspace_sizes(L):
    out = ctypes.c_size_t()
    assert L.qpe_powers_workspace_size(10, ctypes.byref(out)) == 0
    assert out.value >= 2 * 1024 * 1024 * 16
    assert L.qpe_powers_workspace_size(16, ctypes.byref(out)) == 2
    assert L.qpe_controlled_step_workspace_size(12, 6, 1, ctypes.byref(out)) == 0
    assert out.value >= (1 << 18) * 8
    assert L.qpe_iqft_workspace_size(20, 8, 1, ctypes.byref(out)) == 0
    assert L.qpe_iqft_workspace_size(0, 8, 1, ctypes.byref(out)) == 2
    # the readout is summed inside the last DFT pass from n = 12 on (not at
    # n = 17, whose last pass has 5 bits): the workspace then also holds the
    # partial sums, one per row and column group of the last pass (32 columns
    # per group for complex64 at n = 16, 16 for complex128)
    sizes = {}
    for n, t, form in ((11, 10, 1), (16, 10, 1), (16, 10, 0), (17, 10, 1)):
        assert L.qpe_iqft_workspace_size(n, t, form, ctypes.byref(out)) == 0
        sizes[n, form] = out.value
    assert sizes[11, 1] < (1 << 11) * 8
    assert sizes[16, 1] >= (1 << 16) * (1024 // 32) * 8
    assert sizes[16, 0] >= (1 << 16) * (1024 // 16) * 8
    assert sizes[17, 1] < (1 << 17) * 8


@pytest.mark.skipif(os.environ.get("HIP_VISIBLE_DEVICES") is None and os.path.exists("/dev/kfd"),
                    reason="a GPU may be present")
def test_no_device(L):
    h = ctypes.c_void_p()
    assert L.qpe_ctx_create(ctypes.byref(h), 0, None) == 6
    assert L.qpe_ctx_create(None, 0, None) == 1


def test_python_binding_fails_loudly_without_library(tmp_path):
    from paper_2507_17175_amd import qpe
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        qpe._lib_saved = qpe._lib
        try:
            qpe._lib = None
            qpe.load_library(str(tmp_path / "missing.so"))
        finally:
            qpe._lib = qpe._lib_saved


@pytest.mark.slow
def test_host_code_under_sanitizers():
    """Every host-side entry point (argument, size, alignment and workspace
    checks, single and batched workspace planning up to 4500 uneven
    instances, stage-entry sizes, null contexts, status strings) driven from
    plain C against a build whose host code carries AddressSanitizer and
    UndefinedBehaviorSanitizer: no finding, every expectation holds."""
    import subprocess as sp

    from tests import host_sanitize as H
    r = H.run()
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "HOST CHECKS OK" in r.stdout
    assert "AddressSanitizer" not in out and "runtime error" not in out
    syms = sp.run(["nm", "-D", H.LIB], capture_output=True, text=True).stdout
    assert "__asan_" in syms and "__ubsan_handle" in syms  # the sanitizers are really in
