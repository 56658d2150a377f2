"""Batched solver vs the oracle run on each problem alone (float64 kernels:
1e-10 relative on F, 1e-9 on x), with graph replays between direct launches."""

import numpy as np
import pytest

import oracle
from workloads import planted_lasso, random_csc, random_csc_ragged

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    import torch
    assert torch.cuda.is_available()
    import paper_1212_0873_amd as pc
    pc.load()
    return pc


def _problems(dtype="f64", seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for j, (n, ragged) in enumerate([(300, False), (1000, True), (2500, False), (777, True), (64, False),
                                     (5000, False)]):
        m = max(n // 3, 30)
        A = (random_csc_ragged(m, n, 2, 14, rng) if ragged else random_csc(m, n, 10, rng, normalize=False))
        A = A.astype(dtype)
        inst = planted_lasso(A, max(1, n // 50), 0.01, 0.5 * (0.1 ** (j / 5)), rng)
        out.append((inst.A, inst.b, inst.lam, min(n, [1, 16, 256, 100, 64, 700][j])))
    return out


@pytest.mark.parametrize("graph_steps", [0, 8])
def test_batch_matches_oracle_per_problem(pc, graph_steps):
    probs = _problems("f64")
    refs = [oracle.Solver(A, b, lam, tau=tau, seed=7 + j) for j, (A, b, lam, tau) in enumerate(probs)]
    with pc.Batch(probs, seed=7) as B:
        B.set_option("graph_steps", graph_steps)
        for j, r in enumerate(refs):
            inf = B.info(j)
            assert inf["omega"] == r.omega and inf["beta"] == pytest.approx(r.beta, rel=1e-15)
        for rnd in range(4):
            B.step(20)  # with graph_steps = 8: two replays and four direct steps
            for r in refs:
                r.step(20)
            F, gap = B.objective()
            for j, r in enumerate(refs):
                assert F[j] == pytest.approx(r.objective(), rel=1e-10), (rnd, j)
        for j, r in enumerate(refs):
            np.testing.assert_allclose(B.get_x(j), r.x, atol=1e-9)


def test_batch_float32_matches_oracle(pc):
    probs = _problems("f32", seed=1)
    refs = [oracle.Solver(A, b, lam, tau=tau, seed=3 + j) for j, (A, b, lam, tau) in enumerate(probs)]
    with pc.Batch(probs, seed=3) as B:
        for _ in range(5):
            B.step(40)
            for r in refs:
                r.step(40)
            F, _ = B.objective()
            for j, r in enumerate(refs):
                assert F[j] == pytest.approx(r.objective(), rel=1e-5)


def test_retired_problem_holds_still(pc):
    probs = _problems("f64", seed=2)
    with pc.Batch(probs, seed=0) as B:
        B.step(10)
        x_before = B.get_x(2)
        flags = [True] * len(probs)
        flags[2] = False
        B.set_active(flags)
        B.step(10)
        np.testing.assert_array_equal(B.get_x(2), x_before)
        assert B.info(2)["k"] == 10 and B.info(0)["k"] == 20
        # resuming continues the same trajectory as an uninterrupted oracle run
        flags[2] = True
        B.set_active(flags)
        B.step(15)
        A, b, lam, tau = probs[2]
        ref = oracle.Solver(A, b, lam, tau=tau, seed=2)
        ref.step(25)
        np.testing.assert_allclose(B.get_x(2), ref.x, atol=1e-9)


def test_batch_solve_and_autotune(pc):
    probs = _problems("f32", seed=4)
    with pc.Batch(probs, seed=1) as B:
        choice = B.autotune(2)
        assert choice["lanes_per_column"] in (1, 2, 4, 8, 16)
        st = B.solve(rel_gap=1e-6, check_every_steps=32, max_steps=200000)
        assert st["converged"], st
        for j, (A, b, lam, tau) in enumerate(probs):
            gap, D = _scipy_gap(A, b, B.get_x(j), lam)  # property: the certificate holds
            assert gap <= 2e-6 * abs(D)


def _scipy_gap(A, b, x, lam):
    """LASSO duality gap at x computed with scipy (test-side property check)."""
    import scipy.sparse as sp
    M = sp.csc_matrix((A.values_f64(), A.row_idx, A.col_ptr), shape=(A.m, A.n))
    r = M @ x - b
    g = np.max(np.abs(M.T @ r))
    s = min(1.0, lam / g) if g > 0 else 1.0
    F = 0.5 * r @ r + lam * np.abs(x).sum()
    D = -0.5 * s * s * (r @ r) - s * (b @ r)
    return F - D, D
