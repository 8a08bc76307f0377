"""qpe_run_static, the entry point that allocates nothing (its workspace is
the library's static device array), against qpe_run with a caller
workspace: the same problems give the same probabilities and reports, bit
for bit (the same kernels in the same order), and the oracle's P within the
tolerances of the other parity tests (1e-6 mixed, 1e-12 FP64). Two calls in
a row, the second on a smaller problem, so the second runs on the first
one's leftover contents."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle.qpe_oracle as O
from tests.libutil import ensure_built
from workloads import haar_unitary, make_problem

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


def _general(n, t, seed):
    rng = np.random.default_rng(seed)
    d = 1 << t
    U = haar_unitary(d, rng)
    psi = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    psi /= np.linalg.norm(psi)
    return U, psi, n


@pytest.mark.parametrize("form", ["mixed", "fp64"])
def test_static_matches_run_two_calls(qpe, form):
    tol = 1e-6 if form == "mixed" else 1e-12
    # first call: the larger problem (a workspace of 35 MiB of the 64 MiB),
    # then a smaller one on top of its leftovers
    first = (13, 8, 1) if form == "mixed" else (12, 8, 1)
    for n, t, seed in [first, (9, 5, 2)]:
        U, psi, n = _general(n, t, 1500 + seed)
        need = qpe.workspace_bytes([(n, t)], form)
        say("static vs run", form, "n", n, "t", t, "workspace", need)
        assert need <= qpe.STATIC_WORKSPACE_BYTES
        Ud, pd = dev(U), dev(psi)
        Ps, rs = qpe.run_batch_static([(Ud, pd, n)], form, report=True)
        Pr, rr = qpe.run_batch([(Ud, pd, n)], form, report=True)
        Ps, Pr = host(Ps[0]), host(Pr[0])
        assert np.array_equal(Ps, Pr)
        assert rs.tobytes() == rr.tobytes()
        assert np.abs(Ps - O.qpe_probs(U, psi, n)).max() < tol


def test_static_doubling_two_plane_sets(qpe):
    """The prefix-doubling form in the static array (one stream there), whose
    split-FP16 operator planes alternate between two sets: the same P as
    qpe_run's two-stream schedule and as the gate route, bit for bit."""
    flags = qpe.PREFIX_DOUBLING
    for n, t, seed in [(13, 8, 3), (9, 5, 4)]:
        U, psi, n = _general(n, t, 1550 + seed)
        need = qpe.workspace_bytes([(n, t)], "mixed", flags)
        say("static doubling", "n", n, "t", t, "workspace", need)
        assert need <= qpe.STATIC_WORKSPACE_BYTES
        Ud, pd = dev(U), dev(psi)
        Ps = host(qpe.run_batch_static([(Ud, pd, n)], "mixed", flags=flags)[0])
        Pr = host(qpe.run_batch([(Ud, pd, n)], "mixed", flags=flags)[0])
        Pg = host(qpe.run_batch([(Ud, pd, n)], "mixed")[0])
        assert np.array_equal(Ps, Pr)
        assert np.array_equal(Ps, Pg)
        assert np.abs(Ps - O.qpe_probs(U, psi, n)).max() < 1e-6


def test_static_batch_then_single(qpe):
    """A batched call (uneven instances), then a single smaller instance."""
    probs = [make_problem(n, t, np.random.default_rng(1600 + i))
             for i, (n, t) in enumerate([(10, 6), (8, 3), (11, 5), (7, 7)])]
    items = [(dev(p.U), dev(p.psi), p.n_meas) for p in probs]
    say("static batch of", len(items))
    Ps = qpe.run_batch_static(items, "mixed")
    Pr = qpe.run_batch(items, "mixed")
    for p, a, b in zip(probs, Ps, Pr):
        a, b = host(a), host(b)
        assert np.array_equal(a, b)
        assert np.abs(a - O.fejer(p.phis[0], p.n_meas)).max() < 1e-6
    U, psi, n = _general(6, 2, 1700)
    say("static single after the batch")
    a = host(qpe.run_batch_static([(dev(U), dev(psi), n)], "mixed")[0])
    b = host(qpe.run_batch([(dev(U), dev(psi), n)], "mixed")[0])
    assert np.array_equal(a, b)
    assert np.abs(a - O.qpe_probs(U, psi, n)).max() < 1e-6


def test_static_rejects_oversized(qpe):
    """A problem whose workspace exceeds the array: QPE_ERR_WORKSPACE from
    the host checks, nothing enqueued; the library stays usable."""
    n, t = 16, 10
    assert qpe.workspace_bytes([(n, t)], "mixed") > qpe.STATIC_WORKSPACE_BYTES
    U, psi, _ = _general(6, t, 1800)
    say("static oversized", n, t)
    with pytest.raises(qpe.QpeError) as e:
        qpe.run_batch_static([(dev(U), dev(psi), n)], "mixed")
    assert e.value.status == 4 and "static workspace holds" in str(e.value)
    U, psi, n = _general(7, 4, 1801)
    a = host(qpe.run_batch_static([(dev(U), dev(psi), n)], "fp64")[0])
    assert np.abs(a - O.qpe_probs(U, psi, n)).max() < 1e-12
