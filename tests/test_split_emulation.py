"""CPU emulation of the split-FP16 x3 scheme of the mixed form's controlled
products against the closed forms, beside the split-BF16 x6 scheme (the
model in tests/split_emulation.py), at the operator sizes of the n = 16,
t = 10 and n = 20, t = 8 workloads with fewer measurement qubits, and on an
eigenvector close to e_0 with and without the target rotation.

Measured here (max |dP|): split-FP16 x3 4e-8 to 8e-8 on Haar eigenvectors
and 5e-9 to 4e-8 on rotated concentrated ones; split-BF16 x6 3e-8 to 7e-8;
both schemes lose up to 3.6e-6 on the unrotated concentrated input (the
reason the target register is rotated by default). The full-size n = 16,
t = 10 workload emulates to 6.0e-8 (rotated) with split-FP16 x3.
"""
import numpy as np
import pytest

import oracle.qpe_oracle as O
from tests import split_emulation as E
from workloads import haar_unitary

pytestmark = pytest.mark.slow


@pytest.mark.parametrize("scheme", ["fp16x3", "bf16x6"])
@pytest.mark.parametrize("n,t", [(11, 10), (12, 8), (13, 5)])
def test_haar_eigenvector(scheme, n, t):
    rng = np.random.default_rng(40 + n + t)
    Q = haar_unitary(1 << t, rng)
    phis = rng.random(1 << t)
    P = E.mixed_probs(Q, phis, Q[:, 0], n, scheme)
    assert np.abs(P - O.fejer(phis[0], n)).max() < 2.5e-7


def _householder(t, n):
    d = 1 << t
    i = np.arange(d)
    v = 1.0 + 0.37 * i - 0.011 * i * i
    Q = np.eye(d) - 2.0 * np.outer(v, v) / (v @ v)
    phis = np.mod(0.1234567 + 0.7071067811865476 * i, 1.0)
    k = 357 % (1 << n)
    phis[0] = k / float(1 << n)
    return Q, phis, k


@pytest.mark.parametrize("scheme", ["fp16x3", "bf16x6"])
def test_concentrated_eigenvector_rotated(scheme):
    n, t = 14, 8
    Q, phis, k = _householder(t, n)
    want = np.zeros(1 << n)
    want[k] = 1.0
    rng = np.random.default_rng(5)
    rotated = E.mixed_probs(Q, phis, Q[:, 0], n, scheme, rot=E.rotation(1 << t, rng))
    plain = E.mixed_probs(Q, phis, Q[:, 0], n, scheme)
    e_rot, e_plain = np.abs(rotated - want).max(), np.abs(plain - want).max()
    assert e_rot < 2.5e-7
    # the unrotated run of the same input loses far more
    assert e_plain > 5 * e_rot


def test_state_scale_bounds():
    """sigma ||psi|| 2^(-n/2) lies in [2^13, 2^14) for any norm and n, so
    the scaled state stays inside FP16's range (below 65520)."""
    rng = np.random.default_rng(9)
    for n in (1, 8, 20, 30):
        for scale in (1e-30, 1e-3, 1.0, 7.5, 1e20):
            psi = (rng.standard_normal(16) + 1j * rng.standard_normal(16)) * scale
            r = np.linalg.norm(psi) * 2.0 ** (-n / 2.0)
            v = E.state_scale(psi, n) * r
            assert 2.0 ** 13 <= v < 2.0 ** 14, (n, scale, v)
