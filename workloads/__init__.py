"""Seeded synthetic QPE problem generators.

This module is shared by the CPU oracle, the tests and the benchmark. It only
draws random inputs (a unitary U, an input state psi and the eigenphases used
to build them); it holds none of the phase-estimation arithmetic itself.

Construction (the paper's random-unitary test problem, section 3, with a
seeded Haar generator standing in for the unavailable third-party matrix):

* ``haar_unitary(d, rng)``: draw a d x d real Gaussian A, then another d x d
  real Gaussian B (in that order), form Z = (A + iB)/sqrt(2), take Z = QR and
  fix the phases Q <- Q diag(R_ii/|R_ii|) (Mezzadri 2007), which makes Q
  Haar-distributed.
* ``U = Q diag(exp(2 pi i phi)) Q^H`` so that the columns of Q are the
  eigenvectors and ``phi`` the eigenphases in [0, 1).

Draw order per problem: the Haar matrix first, then the target-phase
parameters, then the remaining phases.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

__all__ = [
    "Problem",
    "haar_unitary",
    "unitary_from_phases",
    "make_problem",
    "config_problems",
    "CONFIG_NAMES",
    "analytic_problem",
    "eigenbasis_problems",
    "config5_device",
]


@dataclasses.dataclass
class Problem:
    """One QPE instance: U (d x d complex128), psi (d complex128), n_meas."""

    n_meas: int
    n_mat: int
    U: np.ndarray
    psi: np.ndarray
    # Eigenphases of U in the order of the columns of Q (may be None for
    # problems that are not built from a spectral decomposition).
    phis: Optional[np.ndarray] = None
    # Coefficients of psi in the eigenbasis (only the non-zero ones), and the
    # indices of the eigenvectors they multiply.
    coeff_idx: Optional[np.ndarray] = None
    coeffs: Optional[np.ndarray] = None
    Q: Optional[np.ndarray] = None
    label: str = ""

    @property
    def d(self) -> int:
        return 1 << self.n_mat

    @property
    def N(self) -> int:
        return 1 << self.n_meas


def haar_unitary(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random d x d unitary (complex128) via phase-fixed QR."""
    a = rng.standard_normal((d, d))
    b = rng.standard_normal((d, d))
    z = (a + 1j * b) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    diag = np.diagonal(r)
    q = q * (diag / np.abs(diag))[None, :]
    return np.ascontiguousarray(q, dtype=np.complex128)


def unitary_from_phases(q: np.ndarray, phis: np.ndarray) -> np.ndarray:
    """U = Q diag(exp(2 pi i phi)) Q^H in complex128."""
    lam = np.exp(2j * np.pi * np.asarray(phis, dtype=np.float64))
    return np.ascontiguousarray((q * lam[None, :]) @ q.conj().T, dtype=np.complex128)


def make_problem(n_meas: int, n_mat: int, rng: np.random.Generator,
                 target_phase: Optional[float] = None, label: str = "") -> Problem:
    """Haar U with one target eigenphase and its eigenvector as input."""
    d = 1 << n_mat
    q = haar_unitary(d, rng)
    phi0 = rng.random() if target_phase is None else float(target_phase)
    others = rng.random(d - 1)
    phis = np.concatenate([[phi0], others])
    U = unitary_from_phases(q, phis)
    psi = np.ascontiguousarray(q[:, 0].copy())
    return Problem(n_meas, n_mat, U, psi, phis=phis, coeff_idx=np.array([0]),
                   coeffs=np.array([1.0 + 0j]), Q=q, label=label)


def _config1(seed: int = 1) -> Problem:
    # N_meas = 8, N_mat = 2, phi_0 = k/256 exactly (bit-exact phase).
    rng = np.random.default_rng(seed)
    q = haar_unitary(4, rng)
    k = int(rng.integers(0, 256))
    phis = np.concatenate([[k / 256.0], rng.random(3)])
    U = unitary_from_phases(q, phis)
    return Problem(8, 2, U, np.ascontiguousarray(q[:, 0].copy()), phis=phis,
                   coeff_idx=np.array([0]), coeffs=np.array([1.0 + 0j]), Q=q,
                   label="qpe-n8-t2-exactbit")


def _config2(seed: int = 2) -> Problem:
    # N_meas = 16, N_mat = 10, phi_0 uniform (Fejer-spread distribution).
    rng = np.random.default_rng(seed)
    p = make_problem(16, 10, rng, label="qpe-n16-t10")
    return p


def _config3(seed: int = 3) -> Problem:
    # N_meas = 20, N_mat = 8: three eigenphases within 2^-18 of each other,
    # input the equal superposition of their eigenvectors.
    rng = np.random.default_rng(seed)
    d = 256
    q = haar_unitary(d, rng)
    phi_a = rng.random()
    u_b, u_c = rng.random(), rng.random()
    phi_b = (phi_a + 2.0 ** -18 * u_b) % 1.0
    phi_c = (phi_a + 2.0 ** -18 * u_c) % 1.0
    others = rng.random(d - 3)
    phis = np.concatenate([[phi_a, phi_b, phi_c], others])
    U = unitary_from_phases(q, phis)
    psi = np.ascontiguousarray((q[:, 0] + q[:, 1] + q[:, 2]) / np.sqrt(3.0))
    c = np.full(3, 1.0 / np.sqrt(3.0), dtype=np.complex128)
    return Problem(20, 8, U, psi, phis=phis, coeff_idx=np.array([0, 1, 2]),
                   coeffs=c, Q=q, label="qpe-n20-t8-cluster3")


def _config4(seed: int = 4, count: int = 512) -> List[Problem]:
    # 512 independent instances, N_mat in {3..8}, N_meas in {8..16}.
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for i, child in enumerate(children):
        rng = np.random.default_rng(child)
        t = int(rng.integers(3, 9))
        n = int(rng.integers(8, 17))
        out.append(make_problem(n, t, rng, label=f"batch-{i}-n{n}-t{t}"))
    return out


def analytic_problem(n_meas: int, n_mat: int, j: int) -> Problem:
    """The paper's analytically tractable case (section 3, eqs. 1-7).

    Eigenphases phi_j = j / 2^N_mat, eigenvectors x_j with entries 1 for
    indices k <= j and 0 otherwise, normalised (the printed 1/sqrt(j) is read
    as 1/sqrt(j+1) for 0-based j), U = P Lambda P^{-1}. U is not unitary.
    The input is the eigenvector x_j.
    """
    d = 1 << n_mat
    P = np.zeros((d, d), dtype=np.complex128)
    for col in range(d):
        P[: col + 1, col] = 1.0 / np.sqrt(col + 1.0)
    phis = np.arange(d, dtype=np.float64) / d
    lam = np.exp(2j * np.pi * phis)
    U = (P * lam[None, :]) @ np.linalg.inv(P)
    psi = np.ascontiguousarray(P[:, j].copy())
    return Problem(n_meas, n_mat, np.ascontiguousarray(U), psi, phis=phis,
                   coeff_idx=np.array([j]), coeffs=np.array([1.0 + 0j]), Q=P,
                   label=f"analytic-n{n_meas}-t{n_mat}-j{j}")


def eigenbasis_problems(n_meas: int, n_mat: int = 4, seed: int = 12) -> List[Problem]:
    """One Haar unitary with uniform eigenphases and each of its d eigenvectors
    as the input of its own instance (the paper's precision evaluation,
    section 4.2, runs every eigenvector of a 16 x 16 random unitary). Every
    instance shares U; instance i has psi = Q[:, i] and phase phis[i]."""
    d = 1 << n_mat
    rng = np.random.default_rng(seed)
    q = haar_unitary(d, rng)
    phis = rng.random(d)
    U = unitary_from_phases(q, phis)
    return [Problem(n_meas, n_mat, U, np.ascontiguousarray(q[:, i].copy()), phis=phis,
                    coeff_idx=np.array([i]), coeffs=np.array([1.0 + 0j]), Q=q,
                    label=f"eigenbasis-n{n_meas}-t{n_mat}-i{i}") for i in range(d)]


def config5_device(seed: int = 5, device: str = "cuda"):
    """The VRAM-scale workload: N_meas = 18, N_mat = 14 (2^32 amplitudes), a
    16384 x 16384 Haar unitary with a uniform target eigenphase and its
    eigenvector as input. The Gaussians are drawn on the host in the usual
    order (A, then B, then the phases); the QR factorisation and U = Q
    diag(exp(2 pi i phi)) Q^H run on the device with torch, because on the
    host they take many minutes. Returns (U, psi, phi_0, n_meas, n_mat) with
    U and psi complex128 device tensors."""
    import torch

    n, t = 18, 14
    d = 1 << t
    rng = np.random.default_rng(seed)
    a = torch.from_numpy(rng.standard_normal((d, d))).to(device)
    b = torch.from_numpy(rng.standard_normal((d, d))).to(device)
    z = torch.complex(a, b) / np.sqrt(2.0)
    del a, b
    q, r = torch.linalg.qr(z)
    del z
    diag = torch.diagonal(r)
    q = q * (diag / diag.abs())[None, :]
    del r
    phi0 = float(rng.random())
    phis = np.concatenate([[phi0], rng.random(d - 1)])
    lam = torch.exp(2j * np.pi * torch.from_numpy(phis).to(device))
    U = ((q * lam[None, :]) @ q.conj().T).contiguous()
    psi = q[:, 0].contiguous().clone()
    del q
    return U, psi, phi0, n, t


CONFIG_NAMES = ("c1", "c2", "c3", "c4")


def config_problems(name: str, seed: Optional[int] = None, count: Optional[int] = None) -> List[Problem]:
    """Problems of one named workload.

    c1: n=8,  t=2,  exact-bit phase (1 problem)
    c2: n=16, t=10, uniform phase (1 problem)
    c3: n=20, t=8,  three clustered phases, superposed input (1 problem)
    c4: 512 uneven instances, t in 3..8, n in 8..16
    """
    if name == "c1":
        return [_config1(1 if seed is None else seed)]
    if name == "c2":
        return [_config2(2 if seed is None else seed)]
    if name == "c3":
        return [_config3(3 if seed is None else seed)]
    if name == "c4":
        return _config4(4 if seed is None else seed, 512 if count is None else count)
    raise KeyError(name)
