"""The paper's analytic test problem (Sec. 3, eqs. 1-7) at the sizes of its
Table 2: (N_mat, N_meas) = (2, 18), (2, 19), (4, 14), (4, 15), (4, 16),
(5, 15), (5, 16), for the eigenvectors x_j with j in {0, 1, d/3, d-1}.

U = P Lambda P^-1 is not unitary, so every run uses QPE_NO_POLAR. The
eigenphase j / 2^N_mat is exact with 2^N_meas outcomes (N_meas >= N_mat), so
all the probability belongs on m = j 2^(N_meas - N_mat). Each run's WHOLE P
is compared with the oracle's gate route (O.qpe_probs, itself within 1e-11
of that unit vector at these sizes) and with the unit vector: 1e-6 mixed,
1e-10 FP64 on every outcome. x_0 = e_0 is the most concentrated input there
is; the default mixed path rotates it.
"""
import sys
from functools import lru_cache

import numpy as np
import pytest
import torch

import oracle.qpe_oracle as O
from tests.libutil import ensure_built
from workloads import analytic_problem

pytestmark = pytest.mark.gpu

TABLE2 = [(2, 18), (2, 19), (4, 14), (4, 15), (4, 16), (5, 15), (5, 16)]
TOL = {"mixed": 1e-6, "fp64": 1e-10}


def _js(t):
    d = 1 << t
    return sorted({0, 1, d // 3, d - 1})


CASES = [(t, n, j) for t, n in TABLE2 for j in _js(t)]


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


@lru_cache(maxsize=None)
def _oracle(t, n, j):
    p = analytic_problem(n, t, j)
    return O.qpe_probs(p.U, p.psi, n)


def _unit(t, n, j):
    u = np.zeros(1 << n)
    u[j << (n - t)] = 1.0
    return u


def _check(P, t, n, j, form):
    e_or = float(np.abs(P - _oracle(t, n, j)).max())
    e_ex = float(np.abs(P - _unit(t, n, j)).max())
    assert e_or < TOL[form], ("vs oracle", e_or)
    assert e_ex < TOL[form], ("vs unit vector", e_ex)
    return e_or, e_ex


@pytest.mark.parametrize("form", ["mixed", "fp64"])
@pytest.mark.parametrize("t,n,j", CASES)
def test_analytic_case_no_polar(qpe, form, t, n, j):
    say("analytic", form, "N_mat", t, "N_meas", n, "j", j)
    p = analytic_problem(n, t, j)
    P, rep = qpe.run(dev(p.U), dev(p.psi), n, form, flags=qpe.NO_POLAR, report=True)
    P = host(P)
    e_or, e_ex = _check(P, t, n, j, form)
    say("max|dP| vs oracle", e_or, "vs exact", e_ex, "input_peak", float(rep["input_peak"]))
    # psi is a unit vector; the run keeps its norm to the same tolerance
    assert abs(float(rep["prob_sum"]) - 1.0) < TOL[form] * 4
    assert abs(float(rep["prob_sum"]) - P.sum()) < 1e-12
    # x_0 = e_0 is reported as concentrated (it stays exact here: U is upper
    # triangular, so every state row has one non-zero component)
    assert rep["flags"] & ~np.uint32(qpe.REPORT_CONCENTRATED) == 0


@pytest.mark.parametrize("t,n,j", CASES)
def test_analytic_forced_rotation(qpe, t, n, j):
    """QPE_MIX_TARGET with QPE_NO_POLAR: the rotation is not a default for a
    non-unitary U, but forced on it keeps the Table 2 cases within 1e-6."""
    say("analytic, forced rotation, mixed", t, n, j)
    p = analytic_problem(n, t, j)
    P, rep = qpe.run(dev(p.U), dev(p.psi), n, "mixed", flags=qpe.NO_POLAR | qpe.MIX_TARGET, report=True)
    P = host(P)
    e_or, e_ex = _check(P, t, n, j, "mixed")
    say("max|dP| vs oracle", e_or, "input_peak", float(rep["input_peak"]))
    assert rep["flags"] == 0


@pytest.mark.parametrize("form", ["mixed", "fp64"])
def test_batch_no_polar_analytic(qpe, form):
    """All 26 Table 2 cases in one batched run: each P against the oracle
    and the unit vector, and bit for bit against its single run."""
    say("analytic batch", form, len(CASES), "instances")
    problems = [analytic_problem(n, t, j) for t, n, j in CASES]
    items = [(dev(p.U), dev(p.psi), p.n_meas) for p in problems]
    out = qpe.run_batch(items, form, flags=qpe.NO_POLAR)
    for (t, n, j), (U, psi, _), P in zip(CASES, items, out):
        P = host(P)
        _check(P, t, n, j, form)
        single = host(qpe.run(U, psi, n, form, flags=qpe.NO_POLAR))
        assert np.array_equal(P, single), (t, n, j)


@pytest.mark.parametrize("form", ["mixed", "fp64"])
def test_doubling_no_polar_analytic(qpe, form):
    """The prefix-doubling form on the Table 2 cases: against the oracle and
    the unit vector, and against the gate route to rounding."""
    for t, n, j in CASES:
        say("analytic doubling", form, t, n, j)
        p = analytic_problem(n, t, j)
        U, psi = dev(p.U), dev(p.psi)
        P = host(qpe.run(U, psi, n, form, flags=qpe.NO_POLAR | qpe.PREFIX_DOUBLING))
        _check(P, t, n, j, form)
        gate = host(qpe.run(U, psi, n, form, flags=qpe.NO_POLAR))
        assert np.abs(P - gate).max() < 1e-14


def test_scaling_sweep_analytic(qpe):
    """The section 4.1 sweep driver over N_total = 6..16 (analytic problem,
    N_mat = min(N_total / 2, 12), input x_j for j = d / 3): every row puts
    the probability on the exact outcome, and the memory the process held is
    at least the workspace the library asked for."""
    from paper_2507_17175_amd import study
    cases = []
    for nt in range(6, 17, 2):
        t = min(nt // 2, 12)
        n = nt - t
        j = (1 << t) // 3
        p = analytic_problem(n, t, j)
        cases.append({"U": dev(p.U), "psi": dev(p.psi), "n": n, "peak": j << (n - t)})
    say("scaling sweep", [(c["n"], c["U"].shape[0]) for c in cases])
    rows = study.scaling_sweep(cases, forms=("mixed", "fp64"), flags=qpe.NO_POLAR, reps=2)
    assert len(rows) == 2 * len(cases)
    for r in rows:
        say(r["n_total"], r["form"], r["ms_per_circuit"], "ms", "err", r["max_abs_err_vs_exact"])
        assert r["max_abs_err_vs_exact"] < TOL[r["form"]], r
        assert r["peak_device_bytes"] >= r["workspace_bytes"], r
        assert r["ms_per_circuit"] > 0.0
        assert r["fp64_statevector_bytes"] == 16 << r["n_total"]
