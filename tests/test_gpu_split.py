"""The two split-product schemes of the mixed form on the GPU.

Default: split-FP16 x3 (state scaled by a power of two sigma from ||psi||,
operator by 2^14, two FP16 pieces each, three products). QPE_SPLIT_BF16:
split-BF16 x6. Without the polar step the BF16 scheme always runs.
Tolerances as in test_gpu_parity.py (1e-6 on P for the mixed form; P
scales with ||psi||^2, so unnormalised inputs compare P / ||psi||^2).
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


@pytest.mark.parametrize("scale", [1e-12, 1e-3, 1.0, 37.0, 1e6])
@pytest.mark.parametrize("n,t", [(10, 7), (13, 5), (24, 5)])
def test_fp16_any_input_norm(qpe, scale, n, t):
    """sigma follows ||psi||: tiny and large inputs neither overflow FP16 nor
    lose precision; P / ||psi||^2 matches the normalised oracle run."""
    rng = np.random.default_rng(2000 + n + t)
    d = 1 << t
    U = haar_unitary(d, rng)
    psi = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    psi /= np.linalg.norm(psi)
    say("fp16 scale", scale, "n", n, "t", t)
    P, rep = qpe.run(dev(U), dev(psi * scale), n, "mixed", report=True)
    P = host(P) / scale ** 2
    want = O.qpe_probs(U, psi, n) if n <= 13 else None
    if want is not None:
        assert np.abs(P - want).max() < 1e-6
    assert abs(P.sum() - 1.0) < 1e-6
    assert rep["flags"] == 0


@pytest.mark.parametrize("form_flags", [0, 16], ids=["split_fp16", "split_bf16"])
def test_config2_both_schemes(qpe, form_flags):
    p = config_problems("c2")[0]
    say("c2 full size, flags", form_flags)
    P, rep = qpe.run(dev(p.U), dev(p.psi), p.n_meas, "mixed", flags=form_flags, report=True)
    err = float(np.abs(host(P) - O.fejer(p.phis[0], p.n_meas)).max())
    say("max|dP| vs Fejer", err)
    assert err < 1e-6 and rep["flags"] == 0


@pytest.mark.parametrize("n,t,seed", [(9, 5, 1), (8, 6, 2), (10, 7, 3), (7, 9, 4)])
def test_bf16_flag_matches_oracle_and_differs_from_fp16(qpe, n, t, seed):
    rng = np.random.default_rng(2100 + seed)
    d = 1 << t
    U = haar_unitary(d, rng)
    psi = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    psi /= np.linalg.norm(psi)
    want = O.qpe_probs(U, psi, n)
    a = host(qpe.run(dev(U), dev(psi), n, "mixed"))
    b = host(qpe.run(dev(U), dev(psi), n, "mixed", flags=qpe.SPLIT_BF16))
    say("schemes", n, t, "fp16", float(np.abs(a - want).max()), "bf16", float(np.abs(b - want).max()))
    assert np.abs(a - want).max() < 1e-6 and np.abs(b - want).max() < 1e-6
    assert not np.array_equal(a, b)  # two different roundings


def test_no_polar_runs_bf16(qpe):
    """Without the polar step the mixed form uses the BF16 scheme: the
    results equal the explicit QPE_SPLIT_BF16 run bit for bit."""
    p = make_problem(10, 6, np.random.default_rng(2200))
    U, psi = dev(p.U), dev(p.psi)
    a = host(qpe.run(U, psi, 10, "mixed", flags=qpe.NO_POLAR))
    b = host(qpe.run(U, psi, 10, "mixed", flags=qpe.NO_POLAR | qpe.SPLIT_BF16))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("flags", [0, 16, 2 | 16])
def test_batch_schemes_match_single(qpe, flags):
    probs = config_problems("c4", count=12)
    say("batch of 12 c4 instances, flags", flags)
    items = [(dev(p.U), dev(p.psi), p.n_meas) for p in probs]
    batch = qpe.run_batch(items, "mixed", flags=flags)
    for (U, psi, n), p, Pb in zip(items, probs, batch):
        Pb = host(Pb)
        assert np.array_equal(Pb, host(qpe.run(U, psi, n, "mixed", flags=flags)))
        assert np.abs(Pb - O.fejer(p.phis[0], n)).max() < 1e-6
