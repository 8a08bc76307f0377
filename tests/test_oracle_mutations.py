"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins
catch every one of them: a pin set that a dropped term, a wrong sign, a wrong
index or a transposed operand slips through would not pin anything."""
import math

import numpy as np
import pytest
import scipy.fft

import oracle.qpe_oracle as O
from tests.oracle_pins import PINS


def _ctrl_untransposed(S, V, k):
    j = np.arange(S.shape[0])
    rows = j[((j >> k) & 1) == 1]
    S[rows] = S[rows] @ V          # V instead of V^T


def _ctrl_conj(S, V, k):
    j = np.arange(S.shape[0])
    rows = j[((j >> k) & 1) == 1]
    S[rows] = S[rows] @ V.conj().T  # V^H instead of V^T


def _ctrl_bit_clear(S, V, k):
    j = np.arange(S.shape[0])
    rows = j[((j >> k) & 1) == 0]   # wrong control value
    S[rows] = S[rows] @ V.T


def _ctrl_reversed_order(S, V, k):
    n = S.shape[0].bit_length() - 1
    kk = n - 1 - k                  # register read in the opposite bit order
    j = np.arange(S.shape[0])
    rows = j[((j >> kk) & 1) == 1]
    S[rows] = S[rows] @ V.T


def _iqft_wrong_sign(S):
    return scipy.fft.ifft(S, axis=0, norm="ortho")


def _iqft_no_norm(S):
    return scipy.fft.fft(S, axis=0)


def _powers_linear(U, n):
    V = [np.array(U, dtype=np.complex128)]
    for _ in range(1, n):
        V.append(V[-1] @ U)          # U^(k+1) instead of U^(2^k)
    return V


def _hadamard_unscaled(psi, n):
    N = 1 << n
    S = np.zeros((N, psi.shape[0]), dtype=np.complex128)
    S[0] = psi
    j = np.arange(N)
    for k in range(n):
        lo = j[((j >> k) & 1) == 0]
        hi = lo | (1 << k)
        a, b = S[lo].copy(), S[hi].copy()
        S[lo], S[hi] = a + b, a - b  # dropped 1/sqrt(2)
    return S


def _hadamard_sign(psi, n):
    N = 1 << n
    S = np.zeros((N, psi.shape[0]), dtype=np.complex128)
    S[0] = psi
    j = np.arange(N)
    s = 1.0 / math.sqrt(2.0)
    for k in range(n):
        lo = j[((j >> k) & 1) == 0]
        hi = lo | (1 << k)
        a, b = S[lo].copy(), S[hi].copy()
        S[lo], S[hi] = (a + b) * s, (b - a) * s  # wrong sign on one branch
    return S


def _probs_abs(A):
    return np.abs(A).sum(axis=1)     # |A| instead of |A|^2


def _probs_real_only(A):
    return (A.real ** 2).sum(axis=1)  # dropped imaginary part


def _fejer_off_by_one(phi, n):
    N = 1 << n
    m = np.arange(N, dtype=np.float64) + 1.0   # index shifted
    x = float(N) * float(phi) - m
    num = np.sin(np.pi * x) ** 2
    den = (float(N) ** 2) * np.sin(np.pi * x / N) ** 2
    out = np.ones(N)
    nz = np.mod(x, float(N)) != 0
    out[nz] = num[nz] / den[nz]
    return out


MUTATIONS = {
    "ctrl_untransposed": ("controlled_power_step", _ctrl_untransposed),
    "ctrl_conj": ("controlled_power_step", _ctrl_conj),
    "ctrl_bit_clear": ("controlled_power_step", _ctrl_bit_clear),
    "ctrl_reversed_order": ("controlled_power_step", _ctrl_reversed_order),
    "iqft_wrong_sign": ("inverse_qft", _iqft_wrong_sign),
    "iqft_no_norm": ("inverse_qft", _iqft_no_norm),
    "powers_linear": ("powers_by_squaring", _powers_linear),
    "hadamard_unscaled": ("hadamard_layer", _hadamard_unscaled),
    "hadamard_sign": ("hadamard_layer", _hadamard_sign),
    "probs_abs": ("marginal_probs", _probs_abs),
    "probs_real_only": ("marginal_probs", _probs_real_only),
    "fejer_off_by_one": ("fejer", _fejer_off_by_one),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(O, attr, fn)
    caught = []
    for pin, (pfn, tol) in PINS.items():
        try:
            dev = pfn()
        except Exception:  # a crash also counts as caught
            caught.append(pin)
            continue
        if not (dev <= tol):
            caught.append(pin)
    assert caught, f"mutation {name} slipped through every pin"
