"""Per-kernel HIP-event timing of the C ABI: the timer-class mask restricts
which launches are bracketed (the benchmark times the controlled products
alone inside its timed region)."""
import numpy as np
import pytest
import torch

from tests.libutil import ensure_built
from workloads import make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qpe():
    ensure_built()
    from paper_2507_17175_amd import qpe as q
    return q


def test_timing_mask(qpe):
    p = make_problem(10, 7, np.random.default_rng(3))
    run = qpe.Runner([(torch.from_numpy(p.U).cuda(), torch.from_numpy(p.psi).cuda(), p.n_meas)], form="mixed")
    run()
    torch.cuda.synchronize()
    ctx = run.ctx
    ctx.enable_timing(1024)
    ctx.set_timing_mask(["ctrl_gemm"])
    ctx.reset_timing()
    run()
    tm = ctx.read_timing()
    assert tm["ctrl_gemm"][0] == p.n_meas and tm["ctrl_gemm"][1] > 0.0
    assert all(tm[c][0] == 0 for c in tm if c != "ctrl_gemm")
    ctx.set_timing_mask(None)
    ctx.reset_timing()
    run()
    tm = ctx.read_timing()
    assert tm["ctrl_gemm"][0] == p.n_meas
    assert tm["powers"][0] > 0 and tm["qft"][0] > 0 and tm["prob"][0] > 0 and tm["hlayer"][0] > 0
    # bits beyond the timer classes are rejected (QPE_ERR_ARG) and change nothing
    assert qpe.load_library().qpe_ctx_set_timing_mask(ctx.handle, 1 << len(qpe.TIMERS)) == 1
    ctx.reset_timing()
    run()
    assert ctx.read_timing()["powers"][0] > 0


def test_capture_records_no_timer_events(qpe):
    p = make_problem(9, 6, np.random.default_rng(5))
    run = qpe.Runner([(torch.from_numpy(p.U).cuda(), torch.from_numpy(p.psi).cuda(), p.n_meas)], form="mixed")
    ctx = run.ctx
    ctx.enable_timing(1024)
    ctx.set_timing_mask(None)
    ref = run()[0].cpu().numpy().copy()
    graph = qpe.CapturedRun(run)
    ctx.reset_timing()
    for _ in range(3):
        out = graph()[0].cpu().numpy()
        assert np.array_equal(out, ref)
    tm = ctx.read_timing()
    assert all(v[0] == 0 for v in tm.values()), tm  # the graph holds no event records
    run()  # eager timing works again, every class
    tm = ctx.read_timing()
    assert tm["ctrl_gemm"][0] == p.n_meas and tm["qft"][0] > 0
