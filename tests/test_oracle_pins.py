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


def _circular_closed_form(phi, n):
    # For eigenvector input, sum_m P(m) exp(2 pi i m / N) with
    # P(m) = |N^-1 sum_j exp(2 pi i j (phi - m/N))|^2 expands to
    # N^-2 sum_{j,j'} exp(2 pi i (j - j') phi) sum_m exp(2 pi i m (1 - j + j') / N);
    # the inner sum is N when j - j' = 1 (N - 1 pairs) or j - j' = 1 - N
    # (one pair), and 0 otherwise.
    N = 1 << n
    z = ((N - 1) * np.exp(2j * np.pi * phi) + np.exp(2j * np.pi * (1 - N) * phi)) / N
    a = np.angle(z) / (2 * np.pi)
    return a + 1.0 if a < 0 else a


@pytest.mark.parametrize("n", [1, 3, 8, 12])
def test_circular_estimator_closed_form(n):
    rng = np.random.default_rng(100 + n)
    for phi in list(rng.random(6)) + [0.0, 0.999, 3 / 8]:
        est = O.estimate_circular(O.fejer(phi, n))
        ref = _circular_closed_form(phi, n)
        assert O.phase_error(est, ref) < 1e-11, (phi, est, ref)


def test_circular_estimator_exact_bit_and_wrap():
    # exact-bit phase: the estimate is the phase itself
    P = O.fejer(5 / 32, 5)
    assert abs(O.estimate_circular(P) - 5 / 32) < 1e-15
    # weight split over m = 0 and m = N - 1: the circular mean sits at the
    # wrap (1 - 1/(2N)), the plain weighted average in the middle
    N = 16
    P = np.zeros(N)
    P[0] = P[N - 1] = 0.5
    assert abs(O.estimate_circular(P) - (1 - 0.5 / N)) < 1e-14
    assert abs(O.estimate_weighted(P) - (N - 1) / (2 * N)) < 1e-15


def test_fejer_at_against_geometric_sum():
    # the pointwise closed form against |N^-1 sum_j exp(2 pi i j (phi - m/N))|^2
    for n, phi in [(3, 0.3), (10, 0.7123), (16, 5 / 64), (20, 0.999)]:
        N = 1 << n
        m = np.array([0, 1, int(phi * N), int(phi * N) + 1, N - 1, N // 3])
        j = np.arange(N, dtype=np.float64)
        direct = np.array([abs(np.exp(2j * np.pi * j * (phi - mm / N)).sum() / N) ** 2 for mm in m])
        assert np.abs(O.fejer_at(phi, n, m) - direct).max() < 1e-12
    # and it is the full table's entries
    assert np.array_equal(O.fejer_at(0.3, 9, np.arange(512)), O.fejer(0.3, 9))
