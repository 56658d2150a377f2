"""Pins of the oracle's adjoint (dL/db, dL/dlambda through the LASSO solution)."""

import numpy as np
import pytest

import oracle
from workloads import csc_to_dense, orthonormal_block_hadamard, planted_lasso, random_csc


def test_adjoint_orthonormal_closed_form():
    """A^T A = I: x = soft(A^T b, lam), so on the support dx_i/db = a_i and
    dx_i/dlam = -sign(x_i); dL/db = sum_{i in S} g_i a_i, dL/dlam = -sum s_i g_i."""
    rng = np.random.default_rng(1)
    A = orthonormal_block_hadamard(4, 8, rng)
    M = csc_to_dense(A)
    b = rng.standard_normal(32)
    lam = 0.3
    x = np.sign(M.T @ b) * np.maximum(np.abs(M.T @ b) - lam, 0)
    g = rng.standard_normal(32)
    dldb, dldlam = oracle.lasso_adjoint(A, x, g)
    S = x != 0
    np.testing.assert_allclose(dldb, M[:, S] @ g[S], atol=1e-12)
    assert dldlam == pytest.approx(-np.sum(np.sign(x[S]) * g[S]), abs=1e-12)


def _solve(A, b, lam, seed=0):
    s = oracle.Solver(A, b, lam, tau=1, seed=seed)
    for _ in range(400):
        s.step(20 * s.steps_per_epoch())
        gap, F, _ = s.gap()
        if gap <= 1e-15 * F:
            break
    return s.x.copy()


def test_adjoint_matches_central_differences_of_the_solution_map():
    """Central differences (h = 1e-6) of L(x(b, lam)) = c^T x with x from the
    oracle's converged PCDM solve; the support is stable under +-h."""
    rng = np.random.default_rng(2)
    A = random_csc(30, 20, 6, rng)
    inst = planted_lasso(A, 5, 0.05, 0.15, rng)
    x = _solve(A, inst.b, inst.lam)
    c = rng.standard_normal(20)
    dldb, dldlam = oracle.lasso_adjoint(A, x, c)
    h = 1e-6
    for _ in range(4):
        d = rng.standard_normal(30)
        d /= np.linalg.norm(d)
        xp = _solve(A, inst.b + h * d, inst.lam)
        xm = _solve(A, inst.b - h * d, inst.lam)
        assert np.array_equal(xp != 0, x != 0) and np.array_equal(xm != 0, x != 0)
        fd = (c @ xp - c @ xm) / (2 * h)
        assert fd == pytest.approx(dldb @ d, rel=1e-6, abs=1e-9)
    xp = _solve(A, inst.b, inst.lam + h)
    xm = _solve(A, inst.b, inst.lam - h)
    fd = (c @ xp - c @ xm) / (2 * h)
    assert fd == pytest.approx(dldlam, rel=1e-6, abs=1e-9)


def test_adjoint_empty_support():
    rng = np.random.default_rng(3)
    A = random_csc(10, 8, 3, rng)
    dldb, dldlam = oracle.lasso_adjoint(A, np.zeros(8), rng.standard_normal(8))
    assert np.all(dldb == 0) and dldlam == 0.0
