"""The schedule autotuner and the kernel clocks on single problems.

The autotuner runs real steps (they advance k) with every schedule it tries,
both layouts included; the run must stay on the oracle's trajectory through
and after the tuning (float64, 1e-10 on F), for the LASSO, another loss and
blocks."""

import numpy as np
import pytest

import oracle
from oracle import group
from workloads import make_config, planted_lasso, random_csc, random_csc_ragged

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    import torch
    assert torch.cuda.is_available()
    import paper_1212_0873_amd as pc
    pc.load()
    return pc


def test_autotune_keeps_the_lasso_trajectory(pc):
    inst = make_config("small_2000x1000", dtype="f64")
    ref = oracle.Solver(inst.A, inst.b, inst.lam, tau=40, seed=2)
    with pc.Problem(inst.A, inst.b, inst.lam, 40, seed=2) as p:
        p.set_option("refresh_every", 0)
        choice = p.autotune(2)
        k = p.info()["k"]
        assert k > 0 and k % 2 == 0
        assert choice["lanes_per_column"] in (1, 2, 4, 8, 16)
        ref.step(k)
        p.step(50)
        ref.step(50)
        F, _ = p.objective()
        assert F == pytest.approx(ref.objective(), rel=1e-10)
        np.testing.assert_allclose(p.get_x(), ref.x, rtol=0, atol=1e-9)


def test_autotune_on_a_model_and_on_blocks(pc):
    rng = np.random.default_rng(3)
    A = random_csc_ragged(500, 400, 2, 20, rng)
    y = np.where(rng.standard_normal(500) > 0, 1.0, -1.0)
    ref = oracle.ModelSolver(A, y, tau=30, seed=1, loss="logistic", l1=0.02, l2=0.5)
    with pc.Problem(A, y, 0.02, 30, seed=1, model=dict(loss="logistic", l2=0.5)) as p:
        p.autotune(1)
        inf = p.info()
        assert inf["chunks_per_lane"] == 1
        ref.step(inf["k"])
        p.step(40)
        ref.step(40)
        F, _ = p.objective()
        assert F == pytest.approx(ref.objective(), rel=1e-10)

    B = random_csc(300, 240, 5, rng)
    inst = planted_lasso(B, 20, 0.01, 0.2, rng)
    bp = np.arange(0, 241, 4, dtype=np.int64)
    gref = group.GroupSolver(inst.A, inst.b, inst.lam, bp, tau=6, seed=4)
    with pc.Problem(inst.A, inst.b, inst.lam, 6, seed=4, blocks=bp) as p:
        p.autotune(1)
        gref.step(p.info()["k"])
        p.step(30)
        gref.step(30)
        F, _ = p.objective()
        assert F == pytest.approx(gref.objective(), rel=1e-10)


def test_kernel_clocks(pc):
    inst = make_config("small_2000x1000", dtype="f32")
    with pc.Problem(inst.A, inst.b, inst.lam, 100, seed=0) as p:
        p.set_option("kernel_timing", 1)
        p.step(25)                          # refresh every 10 steps
        p.step_async(1)
        for kind, want in (("gather", 25), ("scatter", 25), ("refresh", 3), ("async", None)):
            n, ms = p.kernel_time(kind)
            assert ms > 0.0
            if want is not None:
                assert n == want, kind
            else:
                assert n >= 1
        p.set_option("kernel_timing", 0)
        assert p.kernel_time("gather") == (0, 0.0)
        from paper_1212_0873_amd import PCDMError
        with pytest.raises(PCDMError):
            p.kernel_time("nonsense")
