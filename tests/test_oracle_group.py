"""Pins for the oracle's block (group LASSO) PCDM1 (section "Block structure,
notation and assumptions"; group-lasso example of block separable Omega;
eq. h(x); Table ESO, tau-nice row over blocks).

Independent references: blocks of one coordinate reduce to the LASSO oracle;
orthonormal columns give the closed form x_i = max(0, 1 - lam/||A_i^T b||)
A_i^T b; the block Lipschitz constants against a singular value
decomposition and hand-computable cases; the block soft threshold against
its optimality conditions; KKT and a zero duality gap at convergence; the ESO
over blocks by exact enumeration of all tau-subsets of blocks."""

import itertools

import numpy as np
import pytest

import oracle
from oracle import group
from workloads import CSC, csc_to_dense, orthonormal_block_hadamard, planted_lasso, random_csc


def _blocks(n, sizes):
    bp = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    assert bp[-1] == n
    return bp


def test_single_coordinate_blocks_are_the_lasso():
    rng = np.random.default_rng(1)
    A = random_csc(50, 40, 4, rng)
    inst = planted_lasso(A, 5, 0.01, 0.1, rng)
    g = group.GroupSolver(inst.A, inst.b, inst.lam, np.arange(41), tau=6, seed=3)
    l = oracle.Solver(inst.A, inst.b, inst.lam, tau=6, seed=3)
    assert g.omega == l.omega and g.beta == l.beta
    np.testing.assert_allclose(g.L, l.L, rtol=1e-13)
    g.step(60)
    l.step(60)
    np.testing.assert_allclose(g.x, l.x, rtol=0, atol=1e-13)


def test_orthonormal_columns_closed_form():
    A = orthonormal_block_hadamard(32, 4)          # A^T A = I
    M = csc_to_dense(A)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(A.m) * 3
    sizes = []
    left = A.n
    while left:
        s = min(left, int(rng.integers(1, 6)))
        sizes.append(s)
        left -= s
    bp = _blocks(A.n, sizes)
    lam = 1.2
    s = group.GroupSolver(A, b, lam, bp, tau=3, seed=1)
    np.testing.assert_allclose(s.L, 1.0, rtol=1e-12)
    s.step(400 * s.steps_per_epoch())
    atb = M.T @ b
    want = np.concatenate([group.block_soft(atb[bp[i]:bp[i + 1]], lam) for i in range(len(bp) - 1)])
    np.testing.assert_allclose(s.x, want, atol=1e-12)
    assert 0 < np.count_nonzero(want) < A.n


def test_block_lipschitz_cases():
    rng = np.random.default_rng(3)
    # disjoint supports: lambda_max = max ||a_c||^2
    rows = np.array([0, 1, 2, 3, 4, 5], dtype=np.int32)
    vals = np.array([1.0, 2.0, 3.0, -1.0, 0.5, 2.0])
    A = CSC(m=6, n=3, col_ptr=np.array([0, 2, 4, 6], dtype=np.int64), row_idx=rows, values=vals)
    assert group.block_lipschitz(A, np.array([0, 3]))[0] == pytest.approx(max(5.0, 10.0, 4.25))
    # two equal columns: lambda_max = 2 ||a||^2
    A2 = CSC(m=3, n=2, col_ptr=np.array([0, 2, 4], dtype=np.int64), row_idx=np.array([0, 2, 0, 2], np.int32),
             values=np.array([1.0, 2.0, 1.0, 2.0]))
    assert group.block_lipschitz(A2, np.array([0, 2]))[0] == pytest.approx(10.0)
    # random blocks against the largest singular value (a different factorisation)
    B = random_csc(30, 20, 6, rng)
    bp = _blocks(20, [4, 6, 1, 9])
    L = group.block_lipschitz(B, bp)
    M = csc_to_dense(B)
    for i in range(4):
        smax = np.linalg.svd(M[:, bp[i]:bp[i + 1]], compute_uv=False)[0]
        assert L[i] == pytest.approx(smax * smax, rel=1e-12)


def test_block_omega_hand_built():
    # columns: c0 rows {0, 1}, c1 {1}, c2 {1, 2}, c3 {2}
    A = CSC(m=3, n=4, col_ptr=np.array([0, 2, 3, 5, 6], dtype=np.int64),
            row_idx=np.array([0, 1, 1, 1, 2, 2], dtype=np.int32), values=np.ones(6))
    # blocks {c0, c1}, {c2}, {c3}: row 1 is hit by blocks 0 (twice) and 1, row 2 by 1 and 2
    assert group.block_omega(A, np.array([0, 2, 3, 4])) == 2
    # single columns: row 1 is hit by c0, c1, c2
    assert group.block_omega(A, np.array([0, 1, 2, 3, 4])) == 3
    assert group.block_omega(A, np.array([0, 4])) == 1


def test_block_soft_threshold_optimality():
    rng = np.random.default_rng(4)
    for _ in range(200):
        u = rng.standard_normal(rng.integers(1, 7)) * rng.uniform(0.1, 3)
        t = rng.uniform(0, 3)
        v = group.block_soft(u, t)
        if np.linalg.norm(u) <= t:
            assert np.all(v == 0)
        else:
            # v - u + t v/||v|| = 0
            np.testing.assert_allclose(v - u + t * v / np.linalg.norm(v), 0, atol=1e-12)


def test_kkt_and_gap_at_convergence():
    rng = np.random.default_rng(5)
    A = random_csc(80, 60, 5, rng)
    inst = planted_lasso(A, 10, 0.01, 0.15, rng)
    bp = _blocks(60, [3] * 20)
    s = group.GroupSolver(inst.A, inst.b, inst.lam, bp, tau=5, seed=2)
    s.step(3000 * s.steps_per_epoch())
    M = csc_to_dense(inst.A)
    g = M.T @ (M @ s.x - inst.b)
    for i in range(20):
        xi = s.x[bp[i]:bp[i + 1]]
        gi = g[bp[i]:bp[i + 1]]
        if np.all(xi == 0):
            assert np.linalg.norm(gi) <= inst.lam * (1 + 1e-9)
        else:
            np.testing.assert_allclose(gi, -inst.lam * xi / np.linalg.norm(xi), atol=1e-9)
    gap, F, D = s.gap()
    assert 0 <= gap <= 1e-10 * F


@pytest.mark.parametrize("tau", [1, 2, 3, 4])
def test_block_eso_by_enumeration(tau):
    """E[f(x + h_[S])] <= f(x) + (tau/nb)(<grad f, h> + beta/2 sum_i L_i ||h^(i)||^2)
    over all tau-subsets of blocks, beta from the block omega."""
    rng = np.random.default_rng(10 + tau)
    A = random_csc(9, 12, 3, rng)
    bp = _blocks(12, [2, 3, 1, 2, 4])
    nb = 5
    M = csc_to_dense(A)
    b = rng.standard_normal(9)
    L = group.block_lipschitz(A, bp)
    om = group.block_omega(A, bp)
    beta = oracle.beta_nice(om, tau, nb)
    f = lambda z: 0.5 * float((M @ z - b) @ (M @ z - b))
    for _ in range(10):
        x = rng.standard_normal(12)
        h = rng.standard_normal(12)
        grad = M.T @ (M @ x - b)
        vals = []
        for S in itertools.combinations(range(nb), tau):
            hs = np.zeros(12)
            for i in S:
                hs[bp[i]:bp[i + 1]] = h[bp[i]:bp[i + 1]]
            vals.append(f(x + hs))
        wnorm = sum(L[i] * float(h[bp[i]:bp[i + 1]] @ h[bp[i]:bp[i + 1]]) for i in range(nb))
        rhs = f(x) + tau / nb * (grad @ h + 0.5 * beta * wnorm)
        assert np.mean(vals) <= rhs + 1e-10 * max(1.0, abs(rhs))
