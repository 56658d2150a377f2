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
