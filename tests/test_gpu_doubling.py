"""GPU parity of the prefix-doubling form of the controlled stage.

Rows [2^k, 2^(k+1)) of the state equal rows [0, 2^k) times V_k^T because the
measurement register starts in |0...0>; every row receives the same ordered
sequence of products as in the gate route, so the two forms agree to
rounding (bit for bit in practice, which the tests report). Tolerances as in
test_gpu_parity.py.
"""
import sys

import numpy as np
import pytest
import torch

import oracle.qpe_oracle as O
from tests.libutil import ensure_built
from workloads import config_problems, haar_unitary, make_problem

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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.complex128).cuda()


def host(x):
    torch.cuda.synchronize()
    return x.cpu().numpy()


@pytest.mark.parametrize("form", ["mixed", "fp64"])
@pytest.mark.parametrize("n,t", [(1, 0), (2, 3), (5, 2), (8, 4), (9, 5), (10, 6), (11, 7), (9, 8), (6, 10), (13, 3)])
def test_doubling_vs_gate_and_oracle(qpe, form, n, t):
    say("doubling", form, "n", n, "t", t)
    rng = np.random.default_rng(1000 + 31 * n + t)
    d = 1 << t
    U = haar_unitary(d, rng)
    psi = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    psi /= np.linalg.norm(psi)
    Ud, pd = dev(U), dev(psi)
    gate = host(qpe.run(Ud, pd, n, form))
    dbl, rep = qpe.run(Ud, pd, n, form, flags=qpe.PREFIX_DOUBLING, report=True)
    dbl = host(dbl)
    same = bool(np.array_equal(gate, dbl))
    say("bitwise equal to gate route:", same, "max diff", float(np.abs(gate - dbl).max()))
    assert np.abs(gate - dbl).max() < 1e-14
    tol = 1e-6 if form == "mixed" else 1e-12
    assert np.abs(dbl - O.qpe_probs(U, psi, n)).max() < tol
    assert rep["flags"] == 0


@pytest.mark.parametrize("form", ["mixed", "fp64"])
def test_doubling_config2_full(qpe, form):
    p = config_problems("c2")[0]
    say("doubling c2 full size", form)
    P = host(qpe.run(dev(p.U), dev(p.psi), p.n_meas, form, flags=qpe.PREFIX_DOUBLING))
    err = float(np.abs(P - O.fejer(p.phis[0], p.n_meas)).max())
    say("max|dP| vs Fejer", err)
    assert err < (1e-6 if form == "mixed" else 1e-9)


@pytest.mark.parametrize("form", ["mixed", "fp64"])
def test_doubling_batch(qpe, form):
    probs = config_problems("c4", count=40)
    say("doubling batch of 40 c4 instances", form)
    items = [(dev(p.U), dev(p.psi), p.n_meas) for p in probs]
    batch = qpe.run_batch(items, form, flags=qpe.PREFIX_DOUBLING)
    for (U, psi, n), p, P in zip(items, probs, batch):
        P = host(P)
        single = host(qpe.run(U, psi, n, form, flags=qpe.PREFIX_DOUBLING))
        assert np.array_equal(P, single)
        assert np.abs(P - O.fejer(p.phis[0], n)).max() < (1e-6 if form == "mixed" else 1e-10)


# (2, 6): the corrected last power is V_1, whose stages rewrite V_0's buffer
# (split on the context stream); (11, 10) and (13, 6): an even last step, so
# the correction writes the first plane set while the odd step before it
# reads the second
@pytest.mark.parametrize("form,n,t", [("mixed", 12, 7), ("mixed", 11, 10), ("mixed", 13, 6), ("mixed", 2, 6),
                                      ("fp64", 10, 6), ("mixed", 9, 3)])
def test_single_doubling_two_streams(qpe, form, n, t):
    """A single run's prefix-doubling form with its power chain on the
    context's second stream (the default schedule) against the one-stream
    schedule and the gate route, bit for bit, eagerly and in every replay of
    its captured graph (the capture forks the second stream and joins it);
    also with the controlled-product timer recording (the chain stays on the
    second stream while only that timer class records)."""
    from paper_2507_17175_amd.qpe import PREFIX_DOUBLING
    p = make_problem(n, t, np.random.default_rng(8100 + n + t))
    say("single doubling, two streams", form, n, t)
    U, psi = dev(p.U), dev(p.psi)
    gate = host(qpe.run(U, psi, n, form))
    runner = qpe.Runner([(U, psi, n)], form=form, flags=PREFIX_DOUBLING)
    ctx = runner.ctx
    try:
        ctx.set_variant("batch_sched", 1)
        one = host(runner()[0]).copy()
        ctx.set_variant("batch_sched", 2)
        two = host(runner()[0]).copy()
        assert np.array_equal(one, gate) and np.array_equal(two, gate)
        ctx.enable_timing(4096)
        ctx.set_timing_mask(["ctrl_gemm"])
        timed = host(runner()[0]).copy()
        launches, ms = ctx.read_timing()["ctrl_gemm"]
        assert launches == n and ms > 0
        assert np.array_equal(timed, gate)
        ctx.set_timing_mask([])  # timing on, no class recording: two streams
        graph = qpe.CapturedRun(runner)
        for rep in range(3):
            runner.probs[0].fill_(-1.0)
            host(qpe.run(U, psi, n, form))
            out = graph()
            assert np.array_equal(host(out[0]), gate), rep
    finally:
        ctx.set_variant("batch_sched", 0)
        ctx.set_timing_mask([])  # the shared context records no more timer events
