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
