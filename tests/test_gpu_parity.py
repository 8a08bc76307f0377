"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (max absolute error over outcomes m, written per test):
  * mixed form: 1e-6 on P(m), the target stated for the method;
  * FP64 form: 1e-9 on P(m) against closed forms. The FP64 powers U^(2^k)
    drift by about 2^k eps sqrt(d) (2^19 * 1.1e-16 * 16 ~ 1e-9 at n = 20,
    t = 8) and each row of the state carries the drift of its top bit, so P
    moves by at most about twice that relative; 1e-12 where n <= 12.
Inputs are seeded; each case prints its name, seed and shape before running.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle.qpe_oracle as O
from tests.libutil import ensure_built
from workloads import analytic_problem, config_problems, haar_unitary, make_problem, unitary_from_phases

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


def dev(x, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def host(x):
    torch.cuda.synchronize()
    return x.cpu().numpy()


# ----------------------------------------------------------------- zgemm

@pytest.mark.parametrize("opA,opB", [("N", "N"), ("C", "N"), ("N", "T"), ("T", "C")])
@pytest.mark.parametrize("m,n,k", [(64, 64, 64), (100, 37, 53), (256, 256, 256), (1024, 1024, 1024)])
def test_zgemm(qpe, opA, opB, m, n, k):
    say("zgemm", opA, opB, m, n, k)
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    def mk(r, c):
        return rng.standard_normal((r, c)) + 1j * rng.standard_normal((r, c))
    A = mk(m, k) if opA == "N" else mk(k, m)
    B = mk(k, n) if opB == "N" else mk(n, k)
    Cin = mk(m, n)
    opf = {"N": lambda x: x, "T": lambda x: x.T, "C": lambda x: x.conj().T}
    alpha, beta = 0.5 - 0.25j, -1.0 + 0.5j
    want = alpha * (opf[opA](A) @ opf[opB](B)) + beta * Cin
    got = host(qpe.zgemm(opA, opB, dev(A), dev(B), alpha, beta, dev(Cin)))
    scale = math.sqrt(k) * 4
    assert np.abs(got - want).max() / scale < 1e-14


# ----------------------------------------------------------------- powers

# d = 1024 and 2048 take the stream-K Gram product (partial slots)
@pytest.mark.parametrize("t,count", [(2, 8), (5, 12), (8, 16), (10, 16), (11, 8)])
def test_powers_vs_spectral(qpe, t, count):
    say("powers", "t", t, "count", count)
    rng = np.random.default_rng(100 + t)
    q = haar_unitary(1 << t, rng)
    phis = rng.random(1 << t)
    U = unitary_from_phases(q, phis)
    V, defect = qpe.powers(dev(U), count, report=True)
    V = host(V)
    ref = O.powers_spectral(q, phis, count)
    for k in range(count):
        err = np.abs(V[k] - ref[k]).max()
        assert err < (2 ** k) * 4e-14 * math.sqrt(1 << t) + 1e-14, (k, err)
        assert np.abs(V[k].conj().T @ V[k] - np.eye(1 << t)).max() < 1e-13, k
    assert defect < 1e-10


def test_powers_no_polar_matches_plain_squaring(qpe):
    say("powers no-polar analytic t=3")
    p = analytic_problem(6, 3, 5)
    V = host(qpe.powers(dev(p.U), 6, flags=qpe.NO_POLAR))
    ref = O.powers_by_squaring(p.U, 6)
    for k in range(6):
        assert np.abs(V[k] - ref[k]).max() < 1e-11 * (2 ** k), k


# --------------------------------------------------------- controlled step

@pytest.mark.parametrize("form", ["fp64", "mixed"])
@pytest.mark.parametrize("n,t", [(6, 0), (7, 2), (8, 4), (8, 5), (9, 6), (8, 7), (10, 8), (7, 10)])
def test_controlled_step(qpe, form, n, t):
    say("controlled_step", form, "n", n, "t", t)
    rng = np.random.default_rng(200 + 13 * n + t)
    d, N = 1 << t, 1 << n
    V = haar_unitary(d, rng)
    S = (rng.standard_normal((N, d)) + 1j * rng.standard_normal((N, d))) / math.sqrt(N * d)
    dt = torch.complex64 if form == "mixed" else torch.complex128
    for k in sorted({0, 1, n // 2, n - 1}):
        S_dev = dev(S, dt)
        qpe.controlled_step(dev(V), S_dev, k, form)
        got = host(S_dev)
        want = S.astype(np.complex64 if form == "mixed" else np.complex128).astype(np.complex128)
        O.controlled_power_step(want, V, k)
        rel = np.abs(got - want).max() / np.abs(want).max()
        tol = 2e-6 if form == "mixed" else 1e-14
        assert rel < tol, (k, rel)


# --------------------------------------------------------------- inverse QFT

@pytest.mark.parametrize("form", ["fp64", "mixed"])
# From n = 12 (not 17) the readout is summed inside the last DFT pass over
# column groups of min(d, E) columns (E = 16-64 elements per workgroup):
# (12, 4), (13, 5), (16, 2) have one group per row, (15, 5) exactly E columns,
# (12, 7), (15, 6), (14, 8) several partials per row, (16, 0) and (13, 1)
# one or two columns (no lane exchange, one exchange).
@pytest.mark.parametrize("n,t", [(1, 0), (3, 2), (4, 1), (5, 3), (8, 0), (9, 2), (12, 4), (13, 5), (16, 2), (17, 1),
                                 (15, 5), (12, 7), (15, 6), (14, 8), (16, 0), (13, 1)])
def test_iqft_probs(qpe, form, n, t):
    say("iqft_probs", form, "n", n, "t", t)
    rng = np.random.default_rng(300 + 17 * n + t)
    N, d = 1 << n, 1 << t
    S = (rng.standard_normal((N, d)) + 1j * rng.standard_normal((N, d))) / math.sqrt(N * d)
    dt = torch.complex64 if form == "mixed" else torch.complex128
    S_in = S.astype(np.complex64).astype(np.complex128) if form == "mixed" else S
    got = host(qpe.iqft_probs(dev(S_in, dt), form))
    want = O.marginal_probs(O.inverse_qft(S_in))
    err = np.abs(got - want).max()
    tol = 1e-7 * max(1.0, want.max() * 10) if form == "mixed" else 1e-14
    assert err < tol, err


@pytest.mark.parametrize("n,t,k0", [(16, 6, 357), (16, 6, 65535), (18, 4, 12345), (20, 2, 699050)])
def test_iqft_tone_keeps_norm(qpe, n, t, k0):
    """Mixed form on a pure tone: the inverse DFT of exp(2 pi i j k0 / N)
    is the basis vector k0 (Sec. 2, the inverse QFT), so all of the input's
    norm must land on outcome k0. The rotations inside the register DFTs are
    done in FP64; with FP32 roots of unity the norm drifted by about 1e-7 at
    n = 16, the same way on every element."""
    say("iqft tone", "n", n, "t", t, "k0", k0)
    rng = np.random.default_rng(310 + n + t)
    N, d = 1 << n, 1 << t
    psi = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    psi /= np.linalg.norm(psi)
    tone = np.exp(2j * np.pi * (np.arange(N) * k0 % N) / N) / math.sqrt(N)
    S = (tone[:, None] * psi[None, :]).astype(np.complex64)
    norm_in = float((np.abs(S.astype(np.complex128)) ** 2).sum())
    P = host(qpe.iqft_probs(dev(S, torch.complex64), "mixed"))
    assert abs(P.sum() - norm_in) < 6e-8, P.sum() - norm_in
    assert abs(P[k0] - norm_in) < 6e-8, P[k0] - norm_in


# ----------------------------------------------------------------- full runs

@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_config1_exact_bit(qpe, form):
    p = config_problems("c1")[0]
    say("run c1 (n=8,t=2, exact bit)", form)
    P, rep = qpe.run(dev(p.U), dev(p.psi), p.n_meas, form, report=True)
    P = host(P)
    want = O.qpe_probs(p.U, p.psi, p.n_meas)
    k = int(round(p.phis[0] * 256))
    tol = 1e-6 if form == "mixed" else 1e-12
    assert np.abs(P - want).max() < tol
    assert abs(P[k] - 1.0) < tol
    assert rep["flags"] == 0 and abs(rep["prob_sum"] - 1) < 1e-6


@pytest.mark.parametrize("form", ["fp64", "mixed"])
@pytest.mark.parametrize("n,t,seed", [(1, 0, 1), (2, 1, 2), (5, 3, 3), (7, 4, 4), (9, 5, 5), (8, 6, 6),
                                      (10, 7, 7), (9, 8, 8), (6, 9, 9), (12, 5, 10), (11, 2, 11)])
def test_run_random_state(qpe, form, n, t, seed):
    """General input (not an eigenvector) against the oracle's gate route."""
    say("run random psi", form, "n", n, "t", t, "seed", seed)
    rng = np.random.default_rng(400 + seed)
    d = 1 << t
    U = haar_unitary(d, rng)
    psi = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    psi /= np.linalg.norm(psi)
    P = host(qpe.run(dev(U), dev(psi), n, form))
    want = O.qpe_probs(U, psi, n)
    tol = 1e-6 if form == "mixed" else 1e-12
    assert np.abs(P - want).max() < tol


@pytest.mark.parametrize("form", ["fp64", "mixed"])
@pytest.mark.parametrize("n,t", [(12, 6), (14, 5), (10, 9)])
def test_run_eigenvector_fejer(qpe, form, n, t):
    say("run eigenvector vs Fejer", form, "n", n, "t", t)
    p = make_problem(n, t, np.random.default_rng(500 + n + t))
    P = host(qpe.run(dev(p.U), dev(p.psi), n, form))
    want = O.fejer(p.phis[0], n)
    tol = 1e-6 if form == "mixed" else 1e-11
    assert np.abs(P - want).max() < tol


@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_config2_full_size(qpe, form):
    p = config_problems("c2")[0]
    say("run c2 full size (n=16,t=10)", form)
    P, rep = qpe.run(dev(p.U), dev(p.psi), p.n_meas, form, report=True)
    P = host(P)
    want = O.fejer(p.phis[0], p.n_meas)
    err = np.abs(P - want).max()
    say("c2", form, "max|dP| vs Fejer", err, "defect", rep["unitarity_defect"])
    assert err < (1e-6 if form == "mixed" else 1e-9)
    assert rep["flags"] == 0
    assert abs(float(rep["prob_sum"]) - P.sum()) < 1e-12


@pytest.mark.parametrize("form", ["mixed", "fp64"])
def test_config3_full_size(qpe, form):
    p = config_problems("c3")[0]
    say("run c3 full size (n=20,t=8, clustered superposition)", form)
    P, rep = qpe.run(dev(p.U), dev(p.psi), p.n_meas, form, report=True)
    P = host(P)
    want = O.superposition_probs(p.phis[:3], [1 / 3] * 3, p.n_meas)
    err = np.abs(P - want).max()
    say("c3", form, "max|dP| vs closed form", err)
    assert err < (1e-6 if form == "mixed" else 1e-9)
    assert rep["flags"] == 0
    assert abs(float(rep["prob_sum"]) - P.sum()) < 1e-12


@pytest.mark.parametrize("n", [13, 14, 15])
def test_report_sums(qpe, n):
    """The per-run report on both sides of the two-stage probability sum
    (2^14 outcomes and up): prob_sum against the host sum of the same P, and
    ||psi||^2 for an input that is not normalised."""
    say("report sums n", n)
    rng = np.random.default_rng(900 + n)
    U = haar_unitary(4, rng)
    psi = (rng.standard_normal(4) + 1j * rng.standard_normal(4)) * 0.8
    P, rep = qpe.run(dev(U), dev(psi), n, "mixed", report=True)
    P = host(P)
    norm2 = float(np.vdot(psi, psi).real)
    assert rep["flags"] == 0
    assert abs(float(rep["prob_sum"]) - P.sum()) < 1e-13 * n
    assert abs(float(rep["psi_norm2"]) - norm2) < 1e-13
    assert abs(P.sum() - norm2) < 1e-5


def test_deterministic(qpe):
    p = config_problems("c2")[0]
    say("determinism c2 mixed x2")
    U, psi = dev(p.U), dev(p.psi)
    a = host(qpe.run(U, psi, p.n_meas, "mixed"))
    b = host(qpe.run(U, psi, p.n_meas, "mixed"))
    assert np.array_equal(a, b)


def test_batch_matches_single(qpe):
    probs = config_problems("c4", count=6)
    say("batch of 6 c4 instances", [(p.n_meas, p.n_mat) for p in probs])
    batch = qpe.run_batch([(dev(p.U), dev(p.psi), p.n_meas) for p in probs], "mixed")
    for p, P in zip(probs, batch):
        single = host(qpe.run(dev(p.U), dev(p.psi), p.n_meas, "mixed"))
        Pb = host(P)
        assert np.array_equal(Pb, single)
        assert np.abs(Pb - O.fejer(p.phis[0], p.n_meas)).max() < 1e-6


@pytest.mark.parametrize("form", ["fp64", "mixed"])
@pytest.mark.parametrize("n,t,seed", [(9, 5, 1), (7, 3, 2), (10, 7, 3), (6, 0, 4), (8, 10, 5)])
def test_mix_target_keeps_P(qpe, form, n, t, seed):
    """The target rotation (QPE_MIX_TARGET: U <- M U M^T, psi <- M psi with
    M orthogonal) leaves P, a marginal over the target register, unchanged:
    against the oracle's gate route for a general input."""
    say("mix target", form, "n", n, "t", t)
    rng = np.random.default_rng(1200 + seed)
    d = 1 << t
    U = haar_unitary(d, rng)
    psi = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    psi /= np.linalg.norm(psi)
    P = host(qpe.run(dev(U), dev(psi), n, form, flags=qpe.MIX_TARGET))
    want = O.qpe_probs(U, psi, n)
    assert np.abs(P - want).max() < (1e-6 if form == "mixed" else 1e-12)


def test_mix_target_state_output(qpe):
    """A rotated run's final statevector is rotated back: equal to the
    unrotated run's state (FP64 form, forced rotation) element by element."""
    from workloads import make_problem
    p = make_problem(9, 6, np.random.default_rng(1250))
    U, psi = dev(p.U), dev(p.psi)
    _, A0 = qpe.run_state(U, psi, p.n_meas, "fp64")
    _, A1 = qpe.run_state(U, psi, p.n_meas, "fp64", flags=qpe.MIX_TARGET)
    assert float(np.abs(host(A1) - host(A0)).max()) < 1e-13
