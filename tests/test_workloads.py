"""The seeded input generators (CPU): determinism and the structure each
recipe promises (distinct rows per column, balanced row degrees, unit
columns, planted solution, lambda relative to ||A^T b||_inf, the uneven
batch), and the counter-based host generator of the large instance."""

import numpy as np
import pytest

from workloads import biggen, make_config, planted_lasso, random_csc
from workloads.configs import batched_path


def _arrays(A):
    return A.col_ptr, A.row_idx, A.values


def test_make_config_is_deterministic():
    a = make_config("small_2000x1000", dtype="f32")
    b = make_config("small_2000x1000", dtype="f32")
    for u, v in zip(_arrays(a.A), _arrays(b.A)):
        assert np.array_equal(u, v)
    assert np.array_equal(a.b, b.b) and a.lam == b.lam
    c = make_config("small_2000x1000", seed=1, dtype="f32")
    assert not np.array_equal(a.A.row_idx, c.A.row_idx)


@pytest.mark.parametrize("balanced", [False, True])
def test_random_csc_structure(balanced):
    rng = np.random.default_rng(0)
    m, n, d = 3000, 4000, 12
    A = random_csc(m, n, d, rng, balanced=balanced)
    assert np.array_equal(A.col_ptr, np.arange(n + 1) * d)
    rows = A.row_idx.reshape(n, d)
    assert rows.min() >= 0 and rows.max() < m
    assert np.all(np.diff(rows, axis=1) > 0)  # distinct and sorted within each column
    norms = np.sqrt((A.values.reshape(n, d) ** 2).sum(1))
    np.testing.assert_allclose(norms, 1.0, rtol=1e-13)
    deg = np.bincount(A.row_idx, minlength=m)
    if balanced:
        # slots dealt round-robin by a permutation: floor/ceil of n d / m, up to
        # the rare redraw of a row repeated inside a column
        # (here about 2% of columns hold a repeated row, so a few % of rows move)
        lo, hi = (n * d) // m, -(-(n * d) // m)
        assert np.mean((deg >= lo) & (deg <= hi)) > 0.9
        assert deg.min() >= lo - 4 and deg.max() <= hi + 4
    else:
        assert deg.max() > -(-(n * d) // m) + 3  # uniform rows spread wider


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_storage_rounding(dtype):
    rng = np.random.default_rng(1)
    A64 = random_csc(500, 300, 5, rng)
    A = A64.astype(dtype)
    v = A.values_f64()
    assert np.array_equal(A.row_idx, A64.row_idx)
    rel = np.max(np.abs(v - A64.values) / np.abs(A64.values))
    assert rel <= (2.0 ** -24 if dtype == "f32" else 2.0 ** -8)
    assert np.array_equal(A.astype(dtype).values, A.values)  # rounding twice changes nothing


def test_planted_lasso():
    import scipy.sparse as sp
    rng = np.random.default_rng(2)
    A = random_csc(800, 1200, 7, rng)
    inst = planted_lasso(A, 40, 0.05, 0.1, rng)
    nz = np.nonzero(inst.xstar)[0]
    assert nz.size == 40
    assert np.all((np.abs(inst.xstar[nz]) >= 1.0) & (np.abs(inst.xstar[nz]) <= 2.0))
    S = sp.csc_matrix((A.values_f64(), A.row_idx, A.col_ptr), shape=(A.m, A.n))
    noise = inst.b - S @ inst.xstar
    assert abs(np.std(noise) - 0.05) < 0.01
    assert inst.lam == pytest.approx(0.1 * np.max(np.abs(S.T @ inst.b)), rel=1e-12)


def test_batched_path_recipe():
    insts = batched_path(count=8, seed=3, nmin=1e3, nmax=3e4)
    for j, it in enumerate(insts):
        n = it.A.n
        assert 1e3 <= n <= 3e4 and it.A.m == max(n // 5, 10)
        assert np.all(np.diff(it.A.col_ptr) == 10)
        assert np.count_nonzero(it.xstar) == max(1, n // 100)
        assert it.tau == min(n, 4096)
    again = batched_path(count=8, seed=3, nmin=1e3, nmax=3e4)
    assert all(np.array_equal(a.b, b.b) for a, b in zip(insts, again))


def test_host_generator_columns_and_instance():
    m, n, d, K = 997, 1500, 9, 30
    A, b, xstar = biggen.host_instance(m, n, d, K, 0.01, seed=5, dtype="f64")
    rows = A.row_idx.reshape(n, d)
    assert rows.min() >= 0 and rows.max() < m
    assert np.all(np.diff(rows, axis=1) > 0)
    np.testing.assert_allclose(np.sqrt((A.values.reshape(n, d) ** 2).sum(1)), 1.0, rtol=1e-12)
    deg = np.bincount(A.row_idx, minlength=m)
    assert deg.max() - deg.min() <= 4  # balanced slots up to redraws
    nz = np.nonzero(xstar)[0]
    assert nz.size == K and np.all((np.abs(xstar[nz]) >= 1) & (np.abs(xstar[nz]) < 2))
    for i in (0, 17, n - 1):
        r, v = biggen.host_column(5, m, n, d, i, dtype="f64")
        assert np.array_equal(r, rows[i]) and np.array_equal(v, A.values.reshape(n, d)[i])
    sel = np.array([0, 5, m - 1])
    np.testing.assert_allclose(biggen.host_b_at(5, m, n, d, K, 0.01, sel, dtype="f64"), b[sel], rtol=0, atol=1e-15)
    A2, b2, x2 = biggen.host_instance(m, n, d, K, 0.01, seed=5, dtype="f64")
    assert np.array_equal(A2.row_idx, A.row_idx) and np.array_equal(b2, b) and np.array_equal(x2, xstar)


def test_biregular_matrix_degrees():
    from workloads import biregular_matrix
    for omega in (1, 5, 50):
        A = biregular_matrix(300, 100, omega, np.random.default_rng(omega))
        assert np.all(np.diff(A.col_ptr) == 3 * omega)
        assert np.all(np.bincount(A.row_idx, minlength=300) == omega)
        for i in range(A.n):
            r = A.row_idx[A.col_ptr[i]:A.col_ptr[i + 1]]
            assert np.unique(r).size == r.size
        assert np.all(A.values == 1.0)
