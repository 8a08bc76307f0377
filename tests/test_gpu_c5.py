"""The VRAM-scale workload (N_meas = 18, N_mat = 14: 2^32 amplitudes, a
16384 x 16384 Haar unitary) in the prefix-doubling form, against the Fejer
closed form over all 2^18 outcomes. Slow (about half a minute)."""
import sys

import numpy as np
import pytest
import torch

import oracle.qpe_oracle as O
from tests.libutil import ensure_built
from workloads import config5_device

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_c5_doubling_matches_fejer():
    ensure_built()
    from paper_2507_17175_amd import qpe
    say("c5: generating the 16384 x 16384 Haar input on the device")
    U, psi, phi0, n, t = config5_device()
    torch.cuda.synchronize()
    say("c5: running the prefix-doubling form")
    P, rep = qpe.run(U, psi, n, form="mixed", flags=qpe.PREFIX_DOUBLING, report=True)
    P = P.cpu().numpy()
    say("c5: done")
    F = O.fejer(phi0, n)
    err = float(np.abs(P - F).max())
    say("c5 max|dP| vs Fejer", err)
    assert err <= 1e-6
    assert int(rep["flags"]) == 0
    assert abs(float(rep["prob_sum"]) - 1.0) < 1e-5
    assert float(rep["unitarity_defect"]) < 1e-10
