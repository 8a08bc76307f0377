"""The CPU oracle against the paper and closed-form mathematics."""
import numpy as np
import pytest

import oracle.qpe_oracle as O
from tests.oracle_pins import PINS


@pytest.mark.parametrize("name", sorted(PINS))
def test_pin(name):
    fn, tol = PINS[name]
    dev = fn()
    assert dev <= tol, f"pin {name}: deviation {dev:.3e} > {tol:.1e}"


def test_estimators():
    # Max-norm and weighted-average estimators (section 4.2).
    n = 10
    P = O.fejer(0.3, n)
    assert O.phase_error(O.estimate_argmax(P), 0.3) <= 0.5 / (1 << n)
    assert O.phase_error(O.estimate_weighted(P), 0.3, circular=False) < 1e-2
    # exact-bit: both estimators are exact
    P = O.fejer(5 / 32, 5)
    assert O.estimate_argmax(P) == 5 / 32
    assert abs(O.estimate_weighted(P) - 5 / 32) < 1e-15
    # circular distance wraps at 1
    assert abs(O.phase_error(0.99, 0.01) - 0.02) < 1e-15
    assert abs(O.phase_error(0.99, 0.01, circular=False) - 0.98) < 1e-15


def test_argmax_tie_smallest():
    P = np.array([0.1, 0.4, 0.4, 0.1])
    assert O.estimate_argmax(P) == 0.25


def test_error_halves_per_qubit_trend():
    # Section 4.2: the argmax error roughly halves per extra measurement
    # qubit. Averaged over 64 phases, the mean error at n+1 is between
    # 0.3x and 0.7x of that at n (closed form, eigenvector input).
    rng = np.random.default_rng(5)
    phis = rng.random(64)
    errs = []
    for n in range(6, 12):
        errs.append(np.mean([O.phase_error(O.estimate_argmax(O.fejer(p, n)), p) for p in phis]))
    ratios = np.array(errs[1:]) / np.array(errs[:-1])
    assert np.all(ratios > 0.3) and np.all(ratios < 0.7), ratios
