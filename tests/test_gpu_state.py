"""Final statevector output (qpe_run_state) against the oracle's statevector
after the inverse QFT, element by element."""
import numpy as np
import pytest
import torch

import oracle.qpe_oracle as O
from tests.libutil import ensure_built
from workloads import config_problems, make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qpe():
    ensure_built()
    from paper_2507_17175_amd import qpe as q
    return q


def _oracle_state(p):
    S = O.hadamard_layer(p.psi, p.n_meas)
    for k, V in enumerate(O.powers_by_squaring(p.U, p.n_meas)):
        O.controlled_power_step(S, V, k)
    return O.inverse_qft(S)


CASES = [(8, 2, 1), (9, 3, 2), (10, 5, 3), (11, 6, 4), (17, 1, 5), (12, 7, 6)]


@pytest.mark.parametrize("form,tol", [("fp64", 1e-11), ("mixed", 2e-6)])
@pytest.mark.parametrize("n,t,seed", CASES)
def test_state_matches_oracle(qpe, form, tol, n, t, seed):
    p = make_problem(n, t, np.random.default_rng(seed))
    prob, A = qpe.run_state(torch.from_numpy(p.U).cuda(), torch.from_numpy(p.psi).cuda(), n, form=form)
    Ao = _oracle_state(p)
    Ag = A.cpu().numpy().astype(np.complex128)
    err = float(np.abs(Ag - Ao).max())
    assert err <= tol, err
    # the readout is the marginal of this state
    assert float(np.abs(prob.cpu().numpy() - (np.abs(Ag) ** 2).sum(axis=1)).max()) <= 10 * tol


def test_state_prefix_doubling_and_c1(qpe):
    from paper_2507_17175_amd.qpe import PREFIX_DOUBLING
    p = config_problems("c1")[0]
    U, psi = torch.from_numpy(p.U).cuda(), torch.from_numpy(p.psi).cuda()
    _, A_gate = qpe.run_state(U, psi, p.n_meas, form="mixed")
    _, A_dbl = qpe.run_state(U, psi, p.n_meas, form="mixed", flags=PREFIX_DOUBLING)
    assert torch.equal(A_gate, A_dbl)
    # exact-bit phase: all weight in row k, which is psi up to a phase
    k = int(round(p.phis[0] * 256))
    row = A_gate[k].cpu().numpy().astype(np.complex128)
    assert abs(np.vdot(p.psi, row)) == pytest.approx(1.0, abs=1e-6)
