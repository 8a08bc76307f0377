"""Pins that tie the CPU oracle to facts other than itself.

Each pin returns the maximum absolute deviation between what the oracle
computes and a value fixed by the paper or by mathematics. The pins are plain
functions so that ``test_oracle_pins.py`` can assert them and
``test_oracle_mutations.py`` can show that a planted mistake in the oracle
breaks at least one of them.
"""
from __future__ import annotations

import math
import os

import numpy as np

import oracle.qpe_oracle as O
from workloads import analytic_problem, config_problems, haar_unitary, make_problem, unitary_from_phases

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def pin_exact_bit() -> float:
    """Exactly representable phase k/2^n with eigenvector input gives
    P(k) = 1 and 0 elsewhere (section 3: such phases are estimated with zero
    error). Uses the n=8, t=2 workload whose phase is k/256."""
    p = config_problems("c1")[0]
    P = O.qpe_probs(p.U, p.psi, p.n_meas)
    k = int(round(p.phis[0] * p.N))
    want = np.zeros(p.N)
    want[k] = 1.0
    return float(np.abs(P - want).max())


def pin_exact_bit_many() -> float:
    """Exact-bit phases at several sizes, with phases whose bit patterns are
    not palindromes (a reversed register order would move the peak)."""
    worst = 0.0
    rng = np.random.default_rng(11)
    for n, t, k in [(5, 2, 0b00110), (6, 3, 0b101100), (7, 1, 0b0000011), (9, 2, 0b100000110)]:
        q = haar_unitary(1 << t, rng)
        phis = np.concatenate([[k / float(1 << n)], rng.random((1 << t) - 1)])
        U = unitary_from_phases(q, phis)
        P = O.qpe_probs(U, q[:, 0], n)
        want = np.zeros(1 << n)
        want[k] = 1.0
        worst = max(worst, float(np.abs(P - want).max()))
    return worst


def pin_fejer() -> float:
    """General phase, eigenvector input: the gate route against the Fejer
    closed form sin^2(pi x)/(N^2 sin^2(pi x/N)) (derived from the definition
    by summing the geometric series)."""
    worst = 0.0
    rng = np.random.default_rng(12)
    for n, t in [(5, 2), (8, 3), (10, 4), (11, 5)]:
        p = make_problem(n, t, rng)
        P = O.qpe_probs(p.U, p.psi, n)
        worst = max(worst, float(np.abs(P - O.fejer(p.phis[0], n)).max()))
    return worst


def pin_fejer_direct_sum() -> float:
    """The closed form against the geometric sum it stands for, evaluated
    term by term in Python: |2^-n sum_j exp(2 pi i j (phi - m/N))|^2."""
    worst = 0.0
    for n, phi in [(3, 0.3), (4, 0.8125), (5, 0.013), (6, 0.9999)]:
        N = 1 << n
        F = O.fejer(phi, n)
        for m in range(N):
            s = sum(complex(math.cos(2 * math.pi * j * (phi - m / N)),
                            math.sin(2 * math.pi * j * (phi - m / N))) for j in range(N)) / N
            worst = max(worst, abs(F[m] - abs(s) ** 2))
    return worst


def pin_one_qubit() -> float:
    """n = 1: P = (cos^2(pi phi), sin^2(pi phi)) (textbook one-bit QPE)."""
    worst = 0.0
    rng = np.random.default_rng(13)
    for t in (0, 1, 3):
        p = make_problem(1, t, rng)
        phi = p.phis[0]
        want = np.array([math.cos(math.pi * phi) ** 2, math.sin(math.pi * phi) ** 2])
        worst = max(worst, float(np.abs(O.qpe_probs(p.U, p.psi, 1) - want).max()))
    return worst


def pin_identity() -> float:
    """U = I: every row keeps psi, so all weight lands on m = 0."""
    rng = np.random.default_rng(14)
    psi = rng.standard_normal(8) + 1j * rng.standard_normal(8)
    P = O.qpe_probs(np.eye(8, dtype=np.complex128), psi, 6)
    want = np.zeros(64)
    want[0] = float(np.vdot(psi, psi).real)
    return float(np.abs(P - want).max())


def pin_scalar_unitary() -> float:
    """U = exp(2 pi i phi) I (and the 1x1 case t = 0): any psi is an
    eigenvector, so P = ||psi||^2 * Fejer(phi)."""
    worst = 0.0
    rng = np.random.default_rng(15)
    for t, n, phi in [(2, 7, 0.37), (0, 9, 0.71)]:
        d = 1 << t
        psi = rng.standard_normal(d) + 1j * rng.standard_normal(d)
        U = np.exp(2j * np.pi * phi) * np.eye(d, dtype=np.complex128)
        P = O.qpe_probs(U, psi, n)
        worst = max(worst, float(np.abs(P - np.vdot(psi, psi).real * O.fejer(phi, n)).max()))
    return worst


def pin_norm() -> float:
    """Unitary circuit: sum_m P(m) = ||psi||^2 for any psi (not an eigenvector),
    and the Fejer distribution sums to 1 (Parseval)."""
    rng = np.random.default_rng(16)
    q = haar_unitary(16, rng)
    psi = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    P = O.qpe_probs(q, psi, 9)
    a = abs(P.sum() - np.vdot(psi, psi).real)
    b = abs(O.fejer(0.123456, 10).sum() - 1.0)
    return float(max(a, b))


def pin_dense_circuit() -> float:
    """Gate route against the dense full-circuit matrix (n + t <= 10), for a
    random non-eigenvector input, a Haar U and a non-unitary U."""
    worst = 0.0
    rng = np.random.default_rng(17)
    cases = []
    q = haar_unitary(4, rng)
    cases.append((q, 5))
    cases.append((haar_unitary(8, rng) @ np.diag(np.exp(2j * np.pi * rng.random(8))), 4))
    cases.append((analytic_problem(4, 2, 1).U, 3))
    for U, n in cases:
        d = U.shape[0]
        psi = rng.standard_normal(d) + 1j * rng.standard_normal(d)
        a = O.qpe_probs(U, psi, n)
        b = O.qpe_probs_dense_circuit(U, psi, n)
        worst = max(worst, float(np.abs(a - b).max()))
    return worst


def pin_krylov() -> float:
    """Gate route against K[j] = U^j psi built by repeated matrix-vector
    products (no squaring, no controlled rows)."""
    worst = 0.0
    rng = np.random.default_rng(18)
    for n, t in [(6, 3), (9, 2)]:
        U = haar_unitary(1 << t, rng)
        psi = rng.standard_normal(1 << t) + 1j * rng.standard_normal(1 << t)
        worst = max(worst, float(np.abs(O.qpe_probs(U, psi, n) - O.qpe_probs_krylov(U, psi, n)).max()))
    return worst


def pin_explicit_dft() -> float:
    """The inverse QFT against the DFT matrix written entry by entry:
    A[m] = N^-1/2 sum_j exp(-2 pi i j m / N) S[j]."""
    rng = np.random.default_rng(19)
    N, d = 32, 3
    S = rng.standard_normal((N, d)) + 1j * rng.standard_normal((N, d))
    F = np.array([[complex(math.cos(-2 * math.pi * j * m / N), math.sin(-2 * math.pi * j * m / N))
                   for j in range(N)] for m in range(N)]) / math.sqrt(N)
    return float(np.abs(O.inverse_qft(S) - F @ S).max())


def pin_hadamard_layer() -> float:
    """H on |0...0> gives the uniform superposition: every row is psi/sqrt(N)."""
    rng = np.random.default_rng(20)
    psi = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    S = O.hadamard_layer(psi, 7)
    return float(np.abs(S - psi[None, :] / math.sqrt(128.0)).max())


def pin_superposition() -> float:
    """Three clustered phases with an equal superposition of their
    eigenvectors: P = (1/3) sum_i Fejer(phi_i) (no cross terms for a unitary
    U with orthonormal eigenvectors)."""
    rng = np.random.default_rng(21)
    d = 32
    q = haar_unitary(d, rng)
    phi_a = rng.random()
    phis = np.concatenate([[phi_a, (phi_a + 2 ** -9 * rng.random()) % 1, (phi_a + 2 ** -9 * rng.random()) % 1],
                           rng.random(d - 3)])
    U = unitary_from_phases(q, phis)
    psi = (q[:, 0] + q[:, 1] + q[:, 2]) / math.sqrt(3.0)
    n = 11
    P = O.qpe_probs(U, psi, n)
    return float(np.abs(P - O.superposition_probs(phis[:3], [1 / 3] * 3, n)).max())


def pin_not_mirrored() -> float:
    """The peak sits at m ~ phi N, not at N - phi N: returns the distance
    of the argmax from round(phi N)."""
    rng = np.random.default_rng(22)
    p = make_problem(8, 2, rng, target_phase=0.3)
    P = O.qpe_probs(p.U, p.psi, 8)
    return float(abs(int(np.argmax(P)) - int(round(0.3 * 256))))


def pin_powers() -> float:
    """Repeated squaring against exact spectral powers exp(2 pi i frac(2^k phi)):
    relative deviation at k = 13 (error grows about 2^k eps)."""
    rng = np.random.default_rng(23)
    q = haar_unitary(16, rng)
    phis = rng.random(16)
    U = unitary_from_phases(q, phis)
    a = O.powers_by_squaring(U, 14)
    b = O.powers_spectral(q, phis, 14)
    return float(max(np.abs(x - y).max() for x, y in zip(a, b)))


def load_analytic_golden():
    rows = []
    with open(os.path.join(GOLDEN, "analytic_case.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            t, n, j, m, p = line.split()
            rows.append((int(t), int(n), int(j), int(m), float(p)))
    return rows


def pin_analytic_golden() -> float:
    """The paper's analytic test problem (section 3, eqs. 1-7): phases
    j/2^N_mat on an N_meas >= N_mat register are recovered with zero error,
    so the stored peak outcome has probability 1."""
    worst = 0.0
    for t, n, j, m, p in load_analytic_golden():
        prob = analytic_problem(n, t, j)
        P = O.qpe_probs(prob.U, prob.psi, n)
        want = np.zeros(1 << n)
        want[m] = p
        worst = max(worst, float(np.abs(P - want).max()))
    return worst


# pin name -> (function, tolerance)
PINS = {
    "exact_bit": (pin_exact_bit, 1e-12),
    "exact_bit_many": (pin_exact_bit_many, 1e-12),
    "fejer": (pin_fejer, 1e-12),
    "fejer_direct_sum": (pin_fejer_direct_sum, 1e-12),
    "one_qubit": (pin_one_qubit, 1e-14),
    "identity": (pin_identity, 1e-13),
    "scalar_unitary": (pin_scalar_unitary, 1e-12),
    "norm": (pin_norm, 1e-12),
    "dense_circuit": (pin_dense_circuit, 1e-12),
    "krylov": (pin_krylov, 1e-12),
    "explicit_dft": (pin_explicit_dft, 1e-13),
    "hadamard_layer": (pin_hadamard_layer, 1e-15),
    "superposition": (pin_superposition, 1e-12),
    "not_mirrored": (pin_not_mirrored, 0.5),
    "powers": (pin_powers, 1e-11),
    "analytic_golden": (pin_analytic_golden, 1e-10),
}
