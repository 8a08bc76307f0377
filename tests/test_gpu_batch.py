"""GPU parity of the batched path (many uneven QPE instances per run).

A batched run uses the same tile code as single runs, so its probabilities
must equal the single-instance results bit for bit; each instance is also
checked against the oracle (gate route for general inputs, the Fejer closed
form for eigenvector inputs) at the tolerances of test_gpu_parity.py.
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


SHAPES = [(1, 0), (2, 1), (3, 2), (5, 3), (7, 4), (9, 5), (8, 6), (10, 7), (9, 8), (12, 2), (6, 9), (4, 5),
          (11, 4), (8, 8)]


@pytest.mark.parametrize("form", ["mixed", "fp64"])
def test_batch_uneven_matches_single_and_oracle(qpe, form):
    say("batch uneven", form, SHAPES)
    rng = np.random.default_rng(900)
    probs = []
    for n, t in SHAPES:
        d = 1 << t
        U = haar_unitary(d, rng)
        psi = rng.standard_normal(d) + 1j * rng.standard_normal(d)
        psi /= np.linalg.norm(psi)
        probs.append((U, psi, n))
    dev_probs = [(dev(U), dev(psi), n) for U, psi, n in probs]
    batch, rep = qpe.run_batch(dev_probs, form, report=True)
    tol = 1e-6 if form == "mixed" else 1e-12
    for (U, psi, n), (Ud, pd, _), Pb, r in zip(probs, dev_probs, batch, rep):
        Pb = host(Pb)
        single = host(qpe.run(Ud, pd, n, form))
        assert np.array_equal(Pb, single), (n, U.shape[0])
        assert np.abs(Pb - O.qpe_probs(U, psi, n)).max() < tol, (n, U.shape[0])
        assert r["flags"] == 0 and abs(r["prob_sum"] - 1.0) < 1e-6


def test_config4_full_batch(qpe):
    problems = config_problems("c4")
    say("batch c4 full: 512 instances, t in 3..8, n in 8..16 (mixed)")
    out, rep = qpe.run_batch([(dev(p.U), dev(p.psi), p.n_meas) for p in problems], "mixed", report=True)
    worst = 0.0
    for p, P in zip(problems, out):
        worst = max(worst, float(np.abs(host(P) - O.fejer(p.phis[0], p.n_meas)).max()))
    say("c4 max|dP| vs Fejer", worst)
    assert worst < 1e-6
    assert np.all(rep["flags"] == 0)


@pytest.mark.parametrize("form,flags", [("mixed", 0), ("fp64", 0), ("mixed", 4)])
def test_graph_replay_matches_eager(qpe, form, flags):
    probs = config_problems("c4", count=24)
    say("graph capture of a 24-instance batch", form, flags)
    items = [(dev(p.U), dev(p.psi), p.n_meas) for p in probs]
    runner = qpe.Runner(items, form=form, flags=flags)
    eager = [host(P).copy() for P in runner()]
    graph = qpe.CapturedRun(runner)
    for rep in range(3):
        for P in runner.probs:
            P.fill_(-1.0)
        # eager work on the same stream between replays
        host(qpe.run(items[0][0], items[0][1], items[0][2], form))
        out = graph()
        for e, P in zip(eager, out):
            assert np.array_equal(host(P), e), rep


@pytest.mark.parametrize("form,flags", [("mixed", 0), ("fp64", 0), ("mixed", 2)])
def test_two_stream_schedule(qpe, form, flags):
    """The batch schedule with the power chain on a second stream: bitwise
    the one-stream result, eagerly and in every replay of its captured graph
    (the capture forks the second stream and joins it back)."""
    probs = config_problems("c4", count=24)
    say("two-stream schedule, 24-instance batch", form, flags)
    items = [(dev(p.U), dev(p.psi), p.n_meas) for p in probs]
    runner = qpe.Runner(items, form=form, flags=flags)
    ctx = runner.ctx
    try:
        ctx.set_variant("batch_sched", 1)
        one = [host(P).copy() for P in runner()]
        ctx.set_variant("batch_sched", 2)
        two = [host(P).copy() for P in runner()]
        for a, b in zip(one, two):
            assert np.array_equal(a, b)
        graph = qpe.CapturedRun(runner)
        for rep in range(3):
            for P in runner.probs:
                P.fill_(-1.0)
            host(qpe.run(items[0][0], items[0][1], items[0][2], form))
            out = graph()
            for e, P in zip(one, out):
                assert np.array_equal(host(P), e), rep
    finally:
        ctx.set_variant("batch_sched", 0)


@pytest.mark.parametrize("flags", [0, 2], ids=["gate_route", "prefix_doubling"])
def test_batch_wide_persistent(qpe, flags):
    """The d = 256 controlled step of a batch on persistent workgroups
    (batched controlled-step variant 3, with 512 or more tiles across three
    instances) against the one-tile-per-workgroup schedule (variant 2, the
    default) and against single runs, bit for bit, and against the Fejer
    closed form."""
    rng = np.random.default_rng(7700 + flags)
    probs = [make_problem(n, 8, rng) for n in (16, 16, 15)] + [make_problem(11, 6, rng)]
    say("persistent wide batch", flags)
    items = [(dev(p.U), dev(p.psi), p.n_meas) for p in probs]
    runner = qpe.Runner(items, form="mixed", flags=flags)
    ctx = runner.ctx
    out = {}
    try:
        for v in (2, 3):
            ctx.set_variant("batch_ctrl", v)
            out[v] = [host(P).copy() for P in runner()]
    finally:
        ctx.set_variant("batch_ctrl", 0)
    for a, b in zip(out[2], out[3]):
        assert np.array_equal(a, b)
    for (U, psi, n), p, P in zip(items, probs, out[3]):
        assert np.array_equal(host(qpe.run(U, psi, n, "mixed", flags=flags)), P)
        assert float(np.abs(P - O.fejer(float(p.phis[0]), n)).max()) <= 1e-6


def test_capture_first_run_of_a_fresh_context(qpe):
    """A batched run captured into a HIP graph as the very first call on a new
    context: the context already holds the second stream and its events, so
    the capture creates nothing; every replay equals an eager run."""
    probs = config_problems("c4", count=24)
    say("capture as the first call of a fresh context")
    items = [(dev(p.U), dev(p.psi), p.n_meas) for p in probs]
    runner = qpe.Runner(items, form="mixed")
    eager = [host(P).copy() for P in runner()]
    runner.ctx = qpe.Context(0)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        runner()
    torch.cuda.synchronize()
    for rep in range(3):
        for P in runner.probs:
            P.fill_(-1.0)
        graph.replay()
        for e, P in zip(eager, runner.probs):
            assert np.array_equal(host(P), e), rep


@pytest.mark.parametrize("flags", [0, 2, 4])
def test_graph_replay_single_instance(qpe, flags):
    # one instance (the single-run path: gate route, prefix doubling, and the
    # target rotation), captured: every replay must equal the eager run
    p = make_problem(11, 7, np.random.default_rng(77))
    say("graph capture of one mixed instance", flags)
    items = [(dev(p.U), dev(p.psi), p.n_meas)]
    runner = qpe.Runner(items, form="mixed", flags=flags)
    eager = host(runner()[0]).copy()
    graph = qpe.CapturedRun(runner)
    for rep in range(3):
        runner.probs[0].fill_(-1.0)
        host(qpe.run(items[0][0], items[0][1], items[0][2], "mixed"))
        out = graph()
        assert np.array_equal(host(out[0]), eager), rep
    ref = O.qpe_probs(p.U, p.psi, p.n_meas)
    assert float(np.abs(eager - ref).max()) < 1e-6


@pytest.mark.parametrize("form", ["mixed", "fp64"])
def test_batch_beyond_4096_instances(qpe, form):
    """More than 4096 members in a launch table: the instance lookup of the
    grouped kernels takes its third sampling round. 4500 tiny instances
    (n <= 3, d <= 4) against the oracle, a sample also against single runs."""
    rng = np.random.default_rng(4500)
    probs = [make_problem(1 + int(rng.integers(3)), int(rng.integers(3)), rng) for _ in range(4500)]
    say("batch of", len(probs), "tiny instances", form)
    items = [(dev(p.U), dev(p.psi), p.n_meas) for p in probs]
    out = qpe.run_batch(items, form)
    tol = 1e-6 if form == "mixed" else 1e-12
    worst = 0.0
    for p, P in zip(probs, out):
        worst = max(worst, float(np.abs(host(P) - O.qpe_probs(p.U, p.psi, p.n_meas)).max()))
    assert worst <= tol, worst
    for i in range(0, len(probs), 499):
        U, psi, n = items[i]
        assert np.array_equal(host(qpe.run(U, psi, n, form=form)), host(out[i])), i


@pytest.mark.parametrize("form", ["mixed", "fp64"])
def test_batch_mix_target_matches_single(qpe, form):
    """The target rotation in a batched run: every instance rotated in its
    own buffers, the same P as the single flagged run, bit for bit, and the
    oracle's P."""
    say("batch mix target", form)
    rng = np.random.default_rng(950)
    shapes = [(9, 5), (7, 3), (10, 7), (6, 0), (8, 6), (11, 2)]
    probs = []
    for n, t in shapes:
        d = 1 << t
        U = haar_unitary(d, rng)
        psi = rng.standard_normal(d) + 1j * rng.standard_normal(d)
        psi /= np.linalg.norm(psi)
        probs.append((U, psi, n))
    dev_probs = [(dev(U), dev(psi), n) for U, psi, n in probs]
    batch = qpe.run_batch(dev_probs, form, flags=qpe.MIX_TARGET)
    tol = 1e-6 if form == "mixed" else 1e-12
    for (U, psi, n), (Ud, pd, _), Pb in zip(probs, dev_probs, batch):
        Pb = host(Pb)
        single = host(qpe.run(Ud, pd, n, form, flags=qpe.MIX_TARGET))
        assert np.array_equal(Pb, single), (n, U.shape[0])
        assert np.abs(Pb - O.qpe_probs(U, psi, n)).max() < tol, (n, U.shape[0])


@pytest.mark.parametrize("form", ["mixed", "fp64"])
def test_batch_doubling_tiny_instances(qpe, form):
    """Prefix doubling in a batch whose instances include n_mat = 0 (a single
    amplitude in row 0) and n_mat = 1 beside larger ones: against the oracle
    and bit for bit against single runs."""
    shapes = [(5, 0), (3, 1), (9, 5), (1, 0), (6, 0), (8, 7), (2, 1), (7, 3)]
    say("batch doubling with tiny instances", form, shapes)
    rng = np.random.default_rng(960)
    probs = []
    for n, t in shapes:
        d = 1 << t
        U = haar_unitary(d, rng)
        psi = rng.standard_normal(d) + 1j * rng.standard_normal(d)
        psi /= np.linalg.norm(psi)
        probs.append((U, psi, n))
    items = [(dev(U), dev(psi), n) for U, psi, n in probs]
    batch = qpe.run_batch(items, form, flags=qpe.PREFIX_DOUBLING)
    tol = 1e-6 if form == "mixed" else 1e-12
    for (U, psi, n), (Ud, pd, _), Pb in zip(probs, items, batch):
        Pb = host(Pb)
        assert np.abs(Pb - O.qpe_probs(U, psi, n)).max() < tol, (n, U.shape[0])
        single = host(qpe.run(Ud, pd, n, form, flags=qpe.PREFIX_DOUBLING))
        assert np.array_equal(Pb, single), (n, U.shape[0])


@pytest.mark.parametrize("flags", [0, 8])
def test_batch_rotation_default_and_off_match_single(qpe, flags):
    """Mixed batches with the default rotation (n_mat >= 5 rotated) and with
    it turned off (QPE_NO_MIX_TARGET): bit for bit equal to single runs,
    reports equal too."""
    probs = config_problems("c4", count=16)
    say("mixed batch, rotation flags", flags)
    items = [(dev(p.U), dev(p.psi), p.n_meas) for p in probs]
    batch, rep = qpe.run_batch(items, "mixed", flags=flags, report=True)
    for (U, psi, n), p, Pb, r in zip(items, probs, batch, rep):
        single, rs = qpe.run(U, psi, n, "mixed", flags=flags, report=True)
        assert np.array_equal(host(Pb), host(single))
        assert r["input_peak"] == rs["input_peak"] and r["flags"] == rs["flags"] == 0
        assert np.abs(host(Pb) - O.fejer(p.phis[0], n)).max() < 1e-6
