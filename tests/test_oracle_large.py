"""Pins of the oracle's pieces for instances too large for the host:
the threaded column-slice statistics (omega, ||A^T b||_inf) and the solver
whose step receives S_k's columns from the caller."""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from workloads import planted_lasso, random_csc, random_csc_ragged


def _slices(A, cuts):
    for c0, c1 in zip(cuts[:-1], cuts[1:]):
        p0, p1 = A.col_ptr[c0], A.col_ptr[c1]
        yield A.col_ptr[c0:c1 + 1], A.row_idx[p0:p1], A.values[p0:p1]


def test_column_stats_match_bincount_and_scipy():
    rng = np.random.default_rng(0)
    A = random_csc_ragged(700, 900, 1, 25, rng).astype("f32")
    # explicit zeros on the fullest row: a count that included stored zeros
    # would differ there
    raw = np.bincount(A.row_idx, minlength=A.m)
    h = int(np.argmax(raw))
    vals = A.values.copy()
    vals[A.row_idx == h] = 0.0
    A.values = vals
    b = rng.standard_normal(A.m)
    st = oracle.ColumnStats(A.m, b)
    for cp, ri, v in _slices(A, [0, 1, 333, 334, 900]):
        st.add(cp, ri, v)
    nz = A.values != 0
    counts = np.bincount(A.row_idx[nz], minlength=A.m)
    assert st.omega == counts.max()
    assert np.array_equal(st.counts, counts)
    assert st.counts[h] == 0 and raw[h] > 0  # the planted zeros matter
    M = sp.csc_matrix((A.values.astype(np.float64), A.row_idx, A.col_ptr), shape=(A.m, A.n))
    assert st.atb_inf == pytest.approx(np.abs(M.T @ b).max(), rel=1e-14)
    assert st.omega == oracle.omega(A)


def test_column_stats_rejects_rows_out_of_range():
    st = oracle.ColumnStats(10, np.ones(10))
    with pytest.raises(ValueError):
        st.add(np.array([0, 2]), np.array([3, 10], dtype=np.int32), np.ones(2, dtype=np.float32))


def _columns(A, S):
    cp = np.concatenate([[0], np.cumsum(A.col_ptr[S + 1] - A.col_ptr[S])])
    ri = np.concatenate([A.row_idx[A.col_ptr[i]:A.col_ptr[i + 1]] for i in S])
    v = np.concatenate([A.values_f64()[A.col_ptr[i]:A.col_ptr[i + 1]] for i in S])
    return cp, ri, v


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_column_set_solver_follows_the_whole_matrix_solver(dtype):
    """Steps on the columns of S_k alone reproduce the solver that holds all
    of A, bit for bit (same sums in the same order), with the large-instance
    solver never seeing the columns outside the sets."""
    rng = np.random.default_rng(1)
    A = random_csc(400, 600, 12, rng).astype(dtype)
    inst = planted_lasso(A, 20, 0.01, 0.1, rng)
    tau = 50
    ref = oracle.Solver(inst.A, inst.b, inst.lam, tau=tau, seed=4)
    big = oracle.ColumnSetSolver(A.m, A.n, inst.b, inst.lam, ref.beta)
    for k in range(30):
        S = np.sort(oracle.sample_nice(4, k, tau, A.n))
        c_big = big.step_with_columns(S, *_columns(inst.A, S))
        c_ref = ref.step(1)
        assert c_big == c_ref
    np.testing.assert_array_equal(big.x, ref.x)
    np.testing.assert_array_equal(big.r, ref.r)
    assert big.objective() == ref.objective(fresh=False)


def test_column_set_solver_tau1_is_exact_coordinate_minimisation():
    """tau = 1, beta = 1: each step minimises F exactly along its coordinate,
    so the touched coordinate satisfies its own optimality condition."""
    rng = np.random.default_rng(2)
    A = random_csc(200, 150, 8, rng)
    inst = planted_lasso(A, 10, 0.01, 0.1, rng)
    big = oracle.ColumnSetSolver(A.m, A.n, inst.b, inst.lam, 1.0)
    for k in range(200):
        i = int(rng.integers(A.n))
        S = np.array([i])
        big.step_with_columns(S, *_columns(inst.A, S))
        g = big.gradient(S, *_columns(inst.A, S))[0]
        if big.x[i] == 0.0:
            assert abs(g) <= inst.lam * (1 + 1e-12)
        else:
            assert g == pytest.approx(-inst.lam * np.sign(big.x[i]), abs=1e-12)
    M = sp.csc_matrix((A.values_f64(), A.row_idx, A.col_ptr), shape=(A.m, A.n))
    np.testing.assert_allclose(big.r, M @ big.x - inst.b, atol=1e-12)


def test_column_set_solver_rejects_unsorted_sets():
    big = oracle.ColumnSetSolver(5, 5, np.ones(5), 0.1, 1.0)
    with pytest.raises(ValueError):
        big.step_with_columns(np.array([3, 1]), np.array([0, 1, 2]), np.array([0, 1], dtype=np.int32),
                              np.ones(2))
