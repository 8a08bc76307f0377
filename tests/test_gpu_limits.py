"""The largest registers the library accepts: N_meas = 30 (2^30 outcomes,
t = 0) and N_mat = 15 (a dense 32768 x 32768 operator, n = 2). The outputs
are checked against the Fejer closed form on sampled outcomes (all of them
for the small register). Slow (each about 10-20 s)."""
import sys

import numpy as np
import pytest
import torch

import oracle.qpe_oracle as O
from tests.libutil import ensure_built

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def qpe():
    ensure_built()
    from paper_2507_17175_amd import qpe as q
    return q


@pytest.mark.parametrize("form", ["mixed", "fp64"])
def test_max_n_meas(qpe, form):
    n = 30
    N = 1 << n
    # phi = 1/4: U = i is exact in binary and so are its powers, so the
    # distribution is exactly a unit peak at N / 4
    say("n=30 t=0 exact phase", form)
    U = torch.tensor([[1j]], dtype=torch.complex128, device="cuda")
    psi = torch.tensor([1.0 + 0j], dtype=torch.complex128, device="cuda")
    P, rep = qpe.run(U, psi, n, form=form, report=True)
    e = qpe.estimate([P])[0]
    assert e["argmax_index"] == N // 4
    assert abs(float(P[N // 4]) - 1.0) < (1e-6 if form == "mixed" else 1e-12)
    assert abs(float(rep["prob_sum"]) - 1.0) < 1e-5
    del P
    # a general phase: sampled outcomes against the closed form. Repeated
    # squaring carries the rounding of U's phase (~1e-16 turns) times 2^k
    # into V_k; at k = 29 that is ~6e-8 turns, which moves P by up to ~1e-6
    # near the peak, so both forms get that bound here.
    phi = 0.3141592653589793
    say("n=30 t=0 general phase", form)
    U = torch.tensor([[np.exp(2j * np.pi * phi)]], dtype=torch.complex128, device="cuda")
    P = qpe.run(U, psi, n, form=form)
    k = int(np.floor(phi * N + 0.5))
    rng = np.random.default_rng(30)
    m = np.unique(np.concatenate([rng.integers(0, N, 4096), (np.arange(-64, 64) + k) % N]))
    got = P[torch.from_numpy(m).cuda()].cpu().numpy()
    err = float(np.abs(got - O.fejer_at(phi, n, m)).max())
    say("n=30", form, "max|dP| on", m.size, "sampled outcomes", err)
    assert err < 2e-6


@pytest.mark.parametrize("form", ["mixed", "fp64"])
def test_max_n_mat(qpe, form):
    # a dense circulant unitary U[j, k] = c[(j - k) mod d], c = ifft(exp(2 pi
    # i phi)): its eigenvectors are the Fourier modes, eigenvalue exp(2 pi i
    # phi_m) for mode m, so the input mode m0 gives the Fejer distribution
    t, n = 15, 2
    d = 1 << t
    say("t=15 n=2 circulant", form)
    rng = np.random.default_rng(15)
    phis = rng.random(d)
    c = np.fft.ifft(np.exp(2j * np.pi * phis))
    e = torch.from_numpy(np.concatenate([c[::-1], c[::-1]]).copy()).cuda()
    U = torch.empty((d, d), dtype=torch.complex128, device="cuda")
    for j in range(d):
        U[j] = e[d - 1 - j: 2 * d - 1 - j]
    m0 = 12345
    psi = torch.from_numpy(np.exp(2j * np.pi * np.arange(d) * m0 / d) / np.sqrt(d)).cuda()
    torch.cuda.synchronize()
    P, rep = qpe.run(U, psi, n, form=form, report=True)
    P = P.cpu().numpy()
    err = float(np.abs(P - O.fejer(phis[m0], n)).max())
    say("t=15", form, "max|dP|", err, "defect", float(rep["unitarity_defect"]))
    assert err < (1e-6 if form == "mixed" else 1e-10)
    assert int(rep["flags"]) == 0
