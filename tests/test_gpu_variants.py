"""Every tile variant of every kernel class against the default variant and
the oracle, including grids whose last row tile is ragged or whose row count
is below one tile."""
import numpy as np
import pytest
import torch

import oracle.qpe_oracle as O
from tests.libutil import ensure_built
from workloads import make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qpe():
    ensure_built()
    from paper_2507_17175_amd import qpe as q
    return q


def _run_all_variants(qpe, cls, form, n, t, seed, flags=0):
    p = make_problem(n, t, np.random.default_rng(seed))
    U, psi = torch.from_numpy(p.U).cuda(), torch.from_numpy(p.psi).cuda()
    ctx = qpe.context(0)
    out = {}
    try:
        for v in range(qpe.kernel_variants(cls) + 1):
            ctx.set_variant(cls, v)
            out[v] = qpe.run(U, psi, n, form=form, flags=flags).cpu().numpy()
    finally:
        ctx.set_variant(cls, 0)
    return p, out


@pytest.mark.parametrize("scheme", [0, 16], ids=["split_fp16", "split_bf16"])
@pytest.mark.parametrize("n,t", [(10, 5), (10, 6), (9, 7), (8, 8), (5, 7), (3, 8), (12, 7)])
def test_ctrl_mixed_variants(qpe, n, t, scheme):
    p, out = _run_all_variants(qpe, "ctrl_mixed", "mixed", n, t, 100 + n + t, flags=scheme)
    ref = O.qpe_probs(p.U, p.psi, n)
    for v, P in out.items():
        assert np.array_equal(P, out[0]), f"variant {v} differs from the default"
        assert float(np.abs(P - ref).max()) <= 1e-6, v


@pytest.mark.parametrize("scheme", [0, 16], ids=["split_fp16", "split_bf16"])
@pytest.mark.parametrize("n,t", [(9, 7), (6, 8), (13, 7)])
def test_ctrl_mixed_variants_prefix_doubling(qpe, n, t, scheme):
    from paper_2507_17175_amd.qpe import PREFIX_DOUBLING
    p, out = _run_all_variants(qpe, "ctrl_mixed", "mixed", n, t, 200 + n + t, flags=PREFIX_DOUBLING | scheme)
    ref = O.qpe_probs(p.U, p.psi, n)
    for v, P in out.items():
        assert np.array_equal(P, out[0]), v
        assert float(np.abs(P - ref).max()) <= 1e-6, v


@pytest.mark.parametrize("n,t", [(8, 5), (9, 7), (11, 9)])
def test_ctrl_f64_variants(qpe, n, t):
    p, out = _run_all_variants(qpe, "ctrl_f64", "fp64", n, t, 300 + n + t)
    ref = O.qpe_probs(p.U, p.psi, n)
    for v, P in out.items():
        # every tile shape sums each output over K in the same order
        assert np.array_equal(P, out[0]), v
        assert float(np.abs(P - ref).max()) <= 1e-11, v


@pytest.mark.parametrize("form", ["fp64", "mixed"])
@pytest.mark.parametrize("n,t", [(9, 7), (8, 10)])
def test_zgemm_variants_bitwise(qpe, form, n, t):
    """Every tile variant of the power-chain GEMM sums each output over K in
    the same order, through the same MFMA operand layout (the K slab only
    groups the steps between barriers, and a Hermitian product mirrors the
    same way at every tile size): the same P bit for bit, at d = 128 and at
    d = 1024 (where the Gram product takes the stream-K plan)."""
    p, out = _run_all_variants(qpe, "zgemm", form, n, t, 450 + t)
    for v, P in out.items():
        assert np.array_equal(P, out[0]), f"variant {v} differs from the default"
    ref = O.qpe_probs(p.U, p.psi, n)
    assert float(np.abs(out[0] - ref).max()) <= (1e-11 if form == "fp64" else 1e-6)


@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_zgemm_variants(qpe, form):
    n, t = 9, 7
    p, out = _run_all_variants(qpe, "zgemm", form, n, t, 400)
    ref = O.qpe_probs(p.U, p.psi, n)
    for v, P in out.items():
        assert float(np.abs(P - out[0]).max()) <= (1e-12 if form == "fp64" else 1e-7), v
        assert float(np.abs(P - ref).max()) <= (1e-11 if form == "fp64" else 1e-6), v


@pytest.mark.parametrize("flags", [0, 2], ids=["gate_route", "prefix_doubling"])
@pytest.mark.parametrize("n,t", [(14, 10), (15, 10), (16, 9), (17, 8)])
def test_wide_tile_variants_bitwise(qpe, n, t, flags):
    """The 128 x 256 tile schedules (variant 8, and variant 9, its persistent
    form and the default from 512 tiles: one workgroup per CU taking 1, 2 or
    more tiles in turn) at sizes with at least 256 such tiles: bit for bit
    the default run, and within 1e-6 of the Fejer closed form of the
    eigenvector input."""
    p = make_problem(n, t, np.random.default_rng(500 + n + t))
    U, psi = torch.from_numpy(p.U).cuda(), torch.from_numpy(p.psi).cuda()
    ctx = qpe.context(0)
    out = {}
    try:
        for v in (0, 8, 9):
            ctx.set_variant("ctrl_mixed", v)
            out[v] = qpe.run(U, psi, n, form="mixed", flags=flags).cpu().numpy()
    finally:
        ctx.set_variant("ctrl_mixed", 0)
    for v in (8, 9):
        assert np.array_equal(out[v], out[0]), v
    F = O.fejer(float(p.phis[0]), n)
    assert float(np.abs(out[0] - F).max()) <= 1e-6
