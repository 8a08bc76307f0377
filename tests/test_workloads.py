"""Seeded input generators: unitarity, eigenpairs, determinism, config shapes."""
import numpy as np

from workloads import analytic_problem, config_problems, haar_unitary, make_problem


def test_haar_unitary_is_unitary():
    q = haar_unitary(64, np.random.default_rng(0))
    assert np.abs(q.conj().T @ q - np.eye(64)).max() < 1e-13


def test_haar_phase_fix_positive_r():
    # After the phase fix Q^H Z has a positive real diagonal (Mezzadri 2007).
    rng = np.random.default_rng(1)
    a = rng.standard_normal((8, 8)); b = rng.standard_normal((8, 8))
    z = (a + 1j * b) / np.sqrt(2)
    q = haar_unitary(8, np.random.default_rng(1))
    r = q.conj().T @ z
    assert np.abs(np.tril(r, -1)).max() < 1e-12
    assert np.all(np.diag(r).real > 0) and np.abs(np.diag(r).imag).max() < 1e-12


def test_eigenpair():
    p = make_problem(6, 4, np.random.default_rng(2))
    lam = np.exp(2j * np.pi * p.phis[0])
    assert np.abs(p.U @ p.psi - lam * p.psi).max() < 1e-13
    assert abs(np.linalg.norm(p.psi) - 1) < 1e-14


def test_deterministic():
    a = config_problems("c1")[0]
    b = config_problems("c1")[0]
    assert np.array_equal(a.U, b.U) and np.array_equal(a.psi, b.psi)
    assert a.n_meas == 8 and a.n_mat == 2
    k = a.phis[0] * 256
    assert k == int(k)


def test_config2_shape():
    p = config_problems("c2")[0]
    assert (p.n_meas, p.n_mat) == (16, 10) and p.U.shape == (1024, 1024)
    assert np.abs(p.U @ p.psi - np.exp(2j * np.pi * p.phis[0]) * p.psi).max() < 1e-12


def test_config3_cluster():
    p = config_problems("c3")[0]
    assert (p.n_meas, p.n_mat) == (20, 8)
    ph = p.phis[:3]
    dist = [min(abs(x - ph[0]), 1 - abs(x - ph[0])) for x in ph[1:]]
    assert max(dist) <= 2.0 ** -18
    assert abs(np.linalg.norm(p.psi) - 1) < 1e-14


def test_config4_sizes():
    probs = config_problems("c4", count=64)
    for p in probs:
        assert 3 <= p.n_mat <= 8 and 8 <= p.n_meas <= 16
    full = config_problems("c4", count=8)
    assert [p.n_mat for p in full] == [p.n_mat for p in probs[:8]]


def test_analytic_eigenpair():
    p = analytic_problem(4, 3, 5)
    lam = np.exp(2j * np.pi * 5 / 8)
    assert np.abs(p.U @ p.psi - lam * p.psi).max() < 1e-12
