"""Warm-started regularisation path on one (A, b): every solution on the path
against the oracle's solve at the same lambda (each side to its own certified
duality gap), the closed form at lambda >= ||A^T b||_inf (x = 0), and the
saving of warm starts over cold solves."""

import numpy as np
import pytest

import oracle
from workloads import make_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    import torch
    assert torch.cuda.is_available()
    import paper_1212_0873_amd as pc
    pc.load()
    return pc


def _oracle_F(inst, lam, tau=8):
    s = oracle.Solver(inst.A, inst.b, lam, tau=tau, seed=0)
    for _ in range(500):
        s.step(10 * s.steps_per_epoch())
        gap, F, _ = s.gap()
        if gap <= 1e-13 * F:
            return F
    raise AssertionError("oracle did not converge")


def test_path_matches_oracle_at_every_lambda(pc):
    inst = make_config("small_2000x1000", dtype="f64")
    lam_max = float(np.max(np.abs(oracle.gradient(inst.A, -inst.b))))
    lams = lam_max * np.geomspace(1.0, 0.01, 8)
    with pc.Problem(inst.A, inst.b, lams[0], 16, seed=0) as p:
        path = p.solve_path(lams, rel_gap=1e-10)
        warm = sum(st["epochs"] for st in path)
    # lambda_max: zero is optimal (|a_i^T b| <= lambda for all i) and certified at once
    assert path[0]["epochs"] == 0 and np.all(path[0]["x"] == 0)
    for st in path:
        assert st["converged"]
        Fo = _oracle_F(inst, st["lambda"])
        assert st["F"] == pytest.approx(Fo, rel=2e-10), st["lambda"]
    cold = 0
    for lam in lams[1:]:
        with pc.Problem(inst.A, inst.b, lam, 16, seed=0) as p:
            cold += p.solve(rel_gap=1e-10, check_every=1)["epochs"]
    print(f"path epochs warm {warm} vs cold {cold}", flush=True)
    assert warm < cold


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_auto_gap_schedule_certifies_and_keeps_the_trajectory(pc, dtype):
    """solve(check_every="auto") stops at a point whose gap, recomputed by the
    oracle from the returned x, meets the target; the gap evaluations do not
    touch the iterate, so the same number of steps without any evaluation
    reaches the same F."""
    inst = make_config("small_2000x1000", dtype=dtype)
    target = 1e-9 if dtype == "f64" else 1e-6
    with pc.Problem(inst.A, inst.b, inst.lam, 8, seed=0) as p:
        st = p.solve(rel_gap=target)
        x = p.get_x()
    assert st["converged"] and st["checks"] >= 1 and st["seconds"] > 0
    gap, F, D = oracle.dual_gap(inst.A, inst.b, x, inst.lam)
    assert gap / abs(D) <= target * 1.01, (gap / abs(D), st)
    assert st["F"] == pytest.approx(F, rel=1e-10)  # both float64 at the same x
    spe = -(-inst.A.n // 8)
    with pc.Problem(inst.A, inst.b, inst.lam, 8, seed=0) as q:
        q.step(st["epochs"] * spe)
        Fq, _ = q.objective()
    assert Fq == pytest.approx(st["F"], rel=1e-12 if dtype == "f64" else 1e-6)
    print(f"  {dtype}: {st['epochs']} epochs, {st['checks']} gap evaluations", flush=True)
