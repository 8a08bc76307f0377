"""The autotuner: every variant it tries computes the same probabilities, and
the choice it keeps is a valid variant that the context then uses."""
import numpy as np
import pytest
import torch

from tests.libutil import ensure_built
from workloads import make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qpe():
    ensure_built()
    from paper_2507_17175_amd import qpe as q
    return q


@pytest.mark.parametrize("form,n,t", [("mixed", 12, 7), ("mixed", 11, 5), ("fp64", 10, 6), ("mixed", 9, 3)])
def test_autotune_keeps_results(qpe, form, n, t):
    p = make_problem(n, t, np.random.default_rng(40 + t))
    U, psi = torch.from_numpy(p.U).cuda(), torch.from_numpy(p.psi).cuda()
    ctx = qpe.context(0)
    for name in qpe.KERNEL_CLASSES:
        ctx.set_variant(name, 0)
    before = qpe.run(U, psi, n, form=form).cpu().numpy()
    res = ctx.autotune(U, psi, n, form=form, reps=1)
    assert res["n_mat"] == t
    for name, v in res["chosen"].items():
        assert 0 <= v <= qpe.kernel_variants(name)
        assert ctx.get_variant(name, t) == v
        assert len(res["ms_per_circuit"][name]) == qpe.kernel_variants(name) + 1
        assert all(m > 0 for m in res["ms_per_circuit"][name])
    if t >= 5:
        assert ("ctrl_mixed" if form == "mixed" else "ctrl_f64") in res["chosen"]
    else:
        assert "ctrl_mixed" not in res["chosen"] and "ctrl_f64" not in res["chosen"]
    after = qpe.run(U, psi, n, form=form).cpu().numpy()
    assert float(np.abs(after - before).max()) <= 1e-12
    table = ctx.tuning_table()
    for name, v in res["chosen"].items():
        assert table.get(name, {}).get(t, 0) == v
    for name in qpe.KERNEL_CLASSES:
        ctx.set_variant(name, 0)


def _batch_items(seed):
    # uneven sizes on both sides of the d >= 64 tile switch and of the d >= 128
    # controlled-step class, and one d = 1024 instance (stream-K Gram product)
    shapes = [(9, 3), (10, 6), (8, 7), (11, 8), (7, 5), (12, 6), (9, 8), (6, 10)]
    rng = np.random.default_rng(seed)
    probs = [make_problem(n, t, rng) for n, t in shapes]
    return probs, [(torch.from_numpy(p.U).cuda(), torch.from_numpy(p.psi).cuda(), p.n_meas) for p in probs]


@pytest.mark.parametrize("form", ["mixed", "fp64"])
def test_batch_variants_bitwise(qpe, form):
    probs, items = _batch_items(61)
    run = qpe.Runner(items, form=form)
    ctx = run.ctx
    ref = None
    try:
        for vc in (0, 1, 2, 3):
            for vg in (0, 1, 2):
                for vs in (1, 2):
                    ctx.set_variant("batch_ctrl", vc)
                    ctx.set_variant("batch_gemm", vg)
                    ctx.set_variant("batch_sched", vs)
                    out = [P.cpu().numpy().copy() for P in run()]
                    if ref is None:
                        ref = out
                    for i, (a, b) in enumerate(zip(out, ref)):
                        assert np.array_equal(a, b), (form, vc, vg, vs, i)
    finally:
        for name in ("batch_ctrl", "batch_gemm", "batch_sched"):
            ctx.set_variant(name, 0)
    # and the batch equals the single runs, bit for bit
    for (U, psi, n), P in zip(items, ref):
        assert np.array_equal(qpe.run(U, psi, n, form=form).cpu().numpy(), P)


def test_autotune_batch(qpe):
    probs, items = _batch_items(62)
    run = qpe.Runner(items, form="mixed")
    before = [P.cpu().numpy().copy() for P in run()]
    ctx = run.ctx
    try:
        res = run.autotune(reps=1)
        assert set(res["chosen"]) == {"batch_ctrl", "batch_gemm", "batch_sched"}
        for name, v in res["chosen"].items():
            assert 0 <= v <= qpe.kernel_variants(name)
            assert ctx.get_variant(name, 0) == v and ctx.get_variant(name, 9) == v
            assert len(res["ms_per_batch"][name]) == qpe.kernel_variants(name) + 1
            assert all(m > 0 for m in res["ms_per_batch"][name])
        after = [P.cpu().numpy() for P in run()]
        for a, b in zip(after, before):
            assert np.array_equal(a, b)
    finally:
        for name in ("batch_ctrl", "batch_gemm", "batch_sched"):
            ctx.set_variant(name, 0)
