"""CPU complex128 oracle for the QPE measurement probabilities.

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import, call or run
this module; only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark use it. It shares no code with the HIP library: no kernels,
tables, constants or helpers. It is deliberately plain and slow.

What it computes (the QPE circuit of the paper, section 2, Fig. 1):

  measurement register |0...0> (n qubits), target register |psi> (d = 2^t),
  H on every measurement qubit, then for k = 0..n-1 the measurement qubit
  that carries bit k of the register integer j controls U^(2^k), then the
  inverse QFT on the measurement register, then the measurement.

With the state held as S[j][r] (j the measurement-register integer, r the
target index), the result is, for m in [0, 2^n):

  A[m, :] = 2^-n * sum_j exp(-2 pi i j m / 2^n) * U^j psi
  P(m)    = sum_r |A[m, r]|^2

Readings of the paper (which is silent on them):
  * bit k of j is the qubit that controls U^(2^k) (the top wire of Fig. 1
    controls U^(2^0)); m uses the same bit weights, so the inverse QFT is the
    unitary inverse DFT of the register integer (output swaps included) and
    the peak lies at m ~ phi 2^n;
  * the QFT maps |j> to 2^-n/2 sum_m exp(+2 pi i j m/2^n)|m>, so its inverse
    uses exp(-...): numpy's forward FFT with norm="ortho";
  * "the norm of the final statevector" (section 3) is read as the marginal
    probability over the target register;
  * psi is not renormalised, so sum_m P(m) = ||psi||^2.

Pins (tests/test_oracle_*.py): exact-bit phase gives P = 1 (section 3); the
Fejer closed form for eigenvector input; n = 1 gives (cos^2, sin^2); U = I;
scalar U; norm preservation; a dense brute-force circuit unitary; the Krylov
route; the superposition closed form; the paper's analytic test problem.
"""
from __future__ import annotations

import math
import os
from typing import List, Optional, Sequence

import numpy as np
import scipy.fft

__all__ = [
    "hadamard_layer",
    "controlled_power_step",
    "powers_by_squaring",
    "powers_spectral",
    "inverse_qft",
    "marginal_probs",
    "qpe_probs",
    "qpe_probs_krylov",
    "qpe_probs_dense_circuit",
    "fejer",
    "fejer_at",
    "superposition_probs",
    "estimate_argmax",
    "estimate_weighted",
    "estimate_circular",
    "phase_error",
]


def _workers() -> int:
    return max(1, os.cpu_count() or 1)


# -- O1/O2: initial state and Hadamard layer (Fig. 1, H gates) --------------

def hadamard_layer(psi: np.ndarray, n: int) -> np.ndarray:
    """|0...0> (x) psi followed by H on each of the n measurement qubits.

    Applied gate by gate: for bit k, every pair of rows (j, j | 2^k) with bit
    k of j clear is mapped to ((a + b)/sqrt 2, (a - b)/sqrt 2).
    """
    N = 1 << n
    d = psi.shape[0]
    S = np.zeros((N, d), dtype=np.complex128)
    S[0] = psi
    j = np.arange(N)
    s = 1.0 / math.sqrt(2.0)
    for k in range(n):
        lo = j[((j >> k) & 1) == 0]
        hi = lo | (1 << k)
        a = S[lo].copy()
        b = S[hi].copy()
        S[lo] = (a + b) * s
        S[hi] = (a - b) * s
    return S


# -- O3: controlled-U^(2^k) (Fig. 1) -----------------------------------------

def controlled_power_step(S: np.ndarray, V: np.ndarray, k: int) -> None:
    """Apply V = U^(2^k) to the target register of every row whose bit k is set.

    In row form the target vector s becomes V s, i.e. S[j, :] <- S[j, :] V^T.
    """
    N = S.shape[0]
    j = np.arange(N)
    rows = j[((j >> k) & 1) == 1]
    S[rows] = S[rows] @ V.T


def powers_by_squaring(U: np.ndarray, n: int) -> List[np.ndarray]:
    """V_0 = U, V_{k+1} = V_k V_k (plain complex128, no re-unitarisation)."""
    V = [np.array(U, dtype=np.complex128)]
    for _ in range(1, n):
        V.append(V[-1] @ V[-1])
    return V


def powers_spectral(Q: np.ndarray, phis: np.ndarray, n: int) -> List[np.ndarray]:
    """V_k = Q diag(exp(2 pi i frac(2^k phi))) Q^H for a unitary Q.

    2^k phi and its fractional part are exact in binary floating point, so
    these powers carry no error that grows with k.
    """
    out = []
    phis = np.asarray(phis, dtype=np.float64)
    for k in range(n):
        f = np.mod(phis * float(1 << k), 1.0)
        lam = np.exp(2j * np.pi * f)
        out.append((Q * lam[None, :]) @ Q.conj().T)
    return out


# -- O4/O5: inverse QFT and readout ----------------------------------------

def inverse_qft(S: np.ndarray) -> np.ndarray:
    """Unitary inverse QFT on the measurement register (axis 0):
    A[m] = 2^-n/2 sum_j exp(-2 pi i j m / 2^n) S[j]."""
    return scipy.fft.fft(S, axis=0, norm="ortho", workers=_workers())


def marginal_probs(A: np.ndarray) -> np.ndarray:
    """P(m) = sum_r |A[m, r]|^2 in float64."""
    return (A.real ** 2 + A.imag ** 2).sum(axis=1)


def qpe_probs(U: np.ndarray, psi: np.ndarray, n: int,
              powers: Optional[Sequence[np.ndarray]] = None) -> np.ndarray:
    """Gate route: H layer, controlled powers, inverse QFT, readout.

    ``powers`` (V_k for k < n) defaults to plain repeated squaring of U.
    """
    U = np.asarray(U, dtype=np.complex128)
    psi = np.asarray(psi, dtype=np.complex128)
    V = list(powers) if powers is not None else powers_by_squaring(U, n)
    S = hadamard_layer(psi, n)
    for k in range(n):
        controlled_power_step(S, V[k], k)
    A = inverse_qft(S)
    return marginal_probs(A)


def qpe_probs_krylov(U: np.ndarray, psi: np.ndarray, n: int) -> np.ndarray:
    """Second route: K[j] = 2^-n/2 U^j psi by repeated matrix-vector products,
    then the inverse QFT and the readout."""
    N = 1 << n
    U = np.asarray(U, dtype=np.complex128)
    K = np.empty((N, U.shape[0]), dtype=np.complex128)
    K[0] = np.asarray(psi, dtype=np.complex128) / math.sqrt(N)
    for j in range(1, N):
        K[j] = U @ K[j - 1]
    return marginal_probs(inverse_qft(K))


def qpe_probs_dense_circuit(U: np.ndarray, psi: np.ndarray, n: int) -> np.ndarray:
    """Third route, for n + t <= 10: the full circuit as one dense matrix.

    Flat index = j * d + r (the measurement register is the high part).
    Circuit = (F (x) I_d) * prod_k CU_k * (H^(x)n (x) I_d), applied to
    e_0 (x) psi, with F[m, j] = exp(-2 pi i j m / N)/sqrt(N) and CU_k the
    block-diagonal matrix holding U^(2^k) in the blocks whose j has bit k set.
    """
    U = np.asarray(U, dtype=np.complex128)
    d = U.shape[0]
    N = 1 << n
    h = np.array([[1.0, 1.0], [1.0, -1.0]]) / math.sqrt(2.0)
    Hn = np.array([[1.0]])
    for _ in range(n):
        Hn = np.kron(Hn, h)
    eye_d = np.eye(d, dtype=np.complex128)
    circuit = np.kron(Hn, eye_d).astype(np.complex128)
    for k in range(n):
        Vk = np.linalg.matrix_power(U, 1 << k)
        CU = np.zeros((N * d, N * d), dtype=np.complex128)
        for jj in range(N):
            blk = Vk if (jj >> k) & 1 else eye_d
            CU[jj * d:(jj + 1) * d, jj * d:(jj + 1) * d] = blk
        circuit = CU @ circuit
    m = np.arange(N)[:, None]
    jv = np.arange(N)[None, :]
    F = np.exp(-2j * np.pi * m * jv / N) / math.sqrt(N)
    circuit = np.kron(F, eye_d) @ circuit
    init = np.zeros(N * d, dtype=np.complex128)
    init[:d] = psi
    final = (circuit @ init).reshape(N, d)
    return marginal_probs(final)


# -- closed forms --------------------------------------------------------------

def fejer(phi: float, n: int) -> np.ndarray:
    """Eigenvector input with eigenphase phi: the probability of outcome m is
    P(m) = sin^2(pi x) / (N^2 sin^2(pi x / N)),  x = N phi - m,
    which is 1 when x is a multiple of N (closed form of the geometric sum
    |2^-n sum_j exp(2 pi i j (phi - m/N))|^2)."""
    N = 1 << n
    m = np.arange(N, dtype=np.float64)
    x = float(N) * float(phi) - m
    num = np.sin(np.pi * x) ** 2
    den = (float(N) ** 2) * np.sin(np.pi * x / N) ** 2
    out = np.empty(N, dtype=np.float64)
    xm = np.mod(x, float(N))
    exact = (xm == 0.0)
    out[exact] = 1.0
    ne = ~exact
    out[ne] = num[ne] / den[ne]
    return out


def fejer_at(phi: float, n: int, m: np.ndarray) -> np.ndarray:
    """The closed form of fejer(phi, n) at the outcomes m only (for
    registers too large to tabulate): P(m) = sin^2(pi x) / (N^2 sin^2(pi x /
    N)), x = N phi - m, and 1 where x is a multiple of N."""
    N = 1 << n
    m = np.asarray(m, dtype=np.float64)
    x = float(N) * float(phi) - m
    out = np.ones(m.shape, dtype=np.float64)
    ne = np.mod(x, float(N)) != 0.0
    out[ne] = np.sin(np.pi * x[ne]) ** 2 / ((float(N) ** 2) * np.sin(np.pi * x[ne] / N) ** 2)
    return out


def superposition_probs(phis: Sequence[float], weights: Sequence[float], n: int) -> np.ndarray:
    """psi = sum_i c_i u_i with orthonormal eigenvectors u_i of a unitary U:
    the outcomes do not interfere, so P = sum_i |c_i|^2 F_n(phi_i)."""
    out = np.zeros(1 << n, dtype=np.float64)
    for phi, w in zip(phis, weights):
        out += float(w) * fejer(phi, n)
    return out


# -- estimators (section 4.2) -------------------------------------------------

def estimate_argmax(P: np.ndarray) -> float:
    """Max-norm estimator: the outcome with the largest probability, divided
    by 2^n (ties go to the smallest m)."""
    return float(np.argmax(P)) / float(P.shape[0])


def estimate_weighted(P: np.ndarray) -> float:
    """Weighted-average estimator: sum_m P(m) * (m / 2^n), with P normalised
    to unit sum."""
    N = P.shape[0]
    m = np.arange(N, dtype=np.float64) / float(N)
    return float((P * m).sum() / P.sum())


def estimate_circular(P: np.ndarray) -> float:
    """Circular mean of the outcome phases m / 2^n weighted by P: the angle
    of sum_m P(m) exp(2 pi i m / 2^n), divided by 2 pi, in [0, 1). Unlike
    the plain weighted average it has no bias at the 0/1 wrap of phases."""
    N = P.shape[0]
    ang = 2.0 * np.pi * np.arange(N, dtype=np.float64) / float(N)
    z = complex((P * np.cos(ang)).sum(), (P * np.sin(ang)).sum())
    a = math.atan2(z.imag, z.real) / (2.0 * math.pi)
    return a + 1.0 if a < 0.0 else a


def phase_error(est: float, ref: float, circular: bool = True) -> float:
    """|est - ref|, or its distance on the unit circle of phases."""
    e = abs(float(est) - float(ref))
    if circular:
        e = min(e, 1.0 - e)
    return e
