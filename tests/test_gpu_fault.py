"""The error path of the C ABI: a HIP call that fails in the middle of a run
(made to fail from the host with QPE_FAULT_INJECT, so that call is never
made and every kernel that runs exits normally) makes qpe_run return
QPE_ERR_HIP, with the failing call named in qpe_last_error, and leaves the
context usable: the next run on it gives the same probabilities, bit for
bit, as a run on an untouched context."""
import ctypes
import os
import sys

import numpy as np
import pytest
import torch

from tests.libutil import ensure_built
from workloads import make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qpe():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ensure_built()
    from paper_2507_17175_amd import qpe as q
    q.load_library()
    return q


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _faulty_context(qpe, at):
    os.environ["QPE_FAULT_INJECT"] = str(at)
    try:
        return qpe.Context(0)
    finally:
        del os.environ["QPE_FAULT_INJECT"]


def _run_raw(qpe, ctx, items, form, flags=0):
    L = qpe.load_library()
    arr = (qpe.Problem * len(items))()
    probs = []
    for i, (U, psi, n) in enumerate(items):
        P = torch.full((1 << n,), -1.0, dtype=torch.float64, device="cuda")
        probs.append(P)
        arr[i].n_meas, arr[i].n_mat = n, U.shape[0].bit_length() - 1
        arr[i].U, arr[i].psi, arr[i].prob = U.data_ptr(), psi.data_ptr(), P.data_ptr()
    need = ctypes.c_size_t()
    assert L.qpe_workspace_size(arr, len(items), qpe.FORMS[form], flags, ctypes.byref(need)) == 0
    ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    ctx.bind_current_stream()
    st = L.qpe_run(ctx.handle, arr, len(items), qpe.FORMS[form], flags, ws.data_ptr(), ws.numel(), None)
    torch.cuda.synchronize()
    return st, [P.cpu().numpy() for P in probs], (L.qpe_last_error(ctx.handle) or b"").decode()


@pytest.mark.parametrize("form", ["mixed", "fp64"])
@pytest.mark.parametrize("at", [1, 2, 7, 25, 34])  # the FP64 run makes 34 checked calls (34: the readout)
def test_injected_failure_single(qpe, form, at):
    p = make_problem(10, 7, np.random.default_rng(3000 + at))
    items = [(torch.from_numpy(p.U).cuda(), torch.from_numpy(p.psi).cuda(), p.n_meas)]
    want = qpe.run(items[0][0], items[0][1], p.n_meas, form).cpu().numpy()
    say("fault injected at checked HIP call", at, form)
    ctx = _faulty_context(qpe, at)
    st, _, err = _run_raw(qpe, ctx, items, form)
    assert st == 7 and "injected fault" in err, (st, err)
    st, out, err = _run_raw(qpe, ctx, items, form)
    assert st == 0, err
    assert np.array_equal(out[0], want)


# the prefix-doubling form of a single run puts its power chain on the
# context's second stream (about 90 checked calls here, event records and
# waits included); a failure at any of them must leave both streams usable
@pytest.mark.parametrize("at", [5, 20, 45, 70])
def test_injected_failure_doubling(qpe, at):
    from paper_2507_17175_amd.qpe import PREFIX_DOUBLING
    p = make_problem(10, 7, np.random.default_rng(3050 + at))
    items = [(torch.from_numpy(p.U).cuda(), torch.from_numpy(p.psi).cuda(), p.n_meas)]
    want = qpe.run(items[0][0], items[0][1], p.n_meas, "mixed").cpu().numpy()
    say("fault injected in a prefix-doubling run at", at)
    ctx = _faulty_context(qpe, at)
    st, _, err = _run_raw(qpe, ctx, items, "mixed", PREFIX_DOUBLING)
    assert st == 7 and "injected fault" in err, (st, err)
    st, out, err = _run_raw(qpe, ctx, items, "mixed", PREFIX_DOUBLING)
    assert st == 0, err
    assert np.array_equal(out[0], want)  # bit for bit the gate route's P


# the batched run makes about 130 checked calls here (launches, and the event
# record and wait of each hop between its two streams)
@pytest.mark.parametrize("at", [1, 4, 30, 60, 90])
def test_injected_failure_batch(qpe, at):
    rng = np.random.default_rng(3100 + at)
    probs = [make_problem(n, t, rng) for n, t in [(9, 5), (7, 3), (10, 7), (6, 0)]]
    items = [(torch.from_numpy(p.U).cuda(), torch.from_numpy(p.psi).cuda(), p.n_meas) for p in probs]
    want = [P.cpu().numpy() for P in qpe.run_batch(items, "mixed")]
    say("fault injected in a batch at", at)
    ctx = _faulty_context(qpe, at)
    st, _, err = _run_raw(qpe, ctx, items, "mixed")
    assert st == 7 and "injected fault" in err, (st, err)
    st, out, err = _run_raw(qpe, ctx, items, "mixed")
    assert st == 0, err
    for a, b in zip(out, want):
        assert np.array_equal(a, b)
