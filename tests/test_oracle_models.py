"""Pins for the oracle's other losses and regularisers (introduction: the
table of three losses; numerical experiments: SVM dual with box constraints,
L2-regularised logistic regression).

Independent references: finite differences of the loss values, numerical
second differences for the curvature bounds, brute-force one-dimensional
minimisation for the block minimiser, library optimisers (L-BFGS) and
closed forms for the optima, and SVM strong duality (the primal objective
computed from the dual iterate)."""

import numpy as np
import pytest
from scipy import optimize

import oracle
from workloads import CSC, csc_to_dense, orthonormal_block_hadamard, random_csc

LOSSES = ["square", "logistic", "sqhinge"]


@pytest.mark.parametrize("loss", LOSSES)
def test_loss_derivative_is_the_derivative(loss):
    rng = np.random.default_rng(1)
    for _ in range(200):
        z = rng.normal() * 3
        y = rng.choice([-1.0, 1.0]) if loss != "square" else rng.normal()
        h = 1e-5
        fd = (oracle.loss_value(loss, z + h, y) - oracle.loss_value(loss, z - h, y)) / (2 * h)
        assert oracle.loss_deriv(loss, z, y) == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_loss_special_values():
    assert oracle.loss_value("logistic", 0.0, 1.0) == pytest.approx(np.log(2.0), rel=1e-15)
    assert oracle.loss_deriv("logistic", 0.0, -1.0) == pytest.approx(0.5, rel=1e-15)
    assert oracle.loss_value("logistic", 800.0, 1.0) == 0.0 or oracle.loss_value("logistic", 800.0, 1.0) < 1e-300
    assert oracle.loss_value("logistic", -800.0, 1.0) == pytest.approx(800.0, rel=1e-15)  # no overflow
    assert oracle.loss_value("sqhinge", 1.5, 1.0) == 0.0 and oracle.loss_deriv("sqhinge", 1.5, 1.0) == 0.0
    assert oracle.loss_value("sqhinge", -1.0, 1.0) == pytest.approx(2.0)
    assert oracle.loss_value("square", 3.0, 1.0) == pytest.approx(2.0)


@pytest.mark.parametrize("loss,bound", [("square", 1.0), ("logistic", 0.25), ("sqhinge", 1.0)])
def test_curvature_bound_is_the_supremum(loss, bound):
    """sup phi'' (the factor in L_i) by second differences of phi'."""
    zs = np.linspace(-8, 8, 16001)
    y = 1.0
    d = np.array([oracle.loss_deriv(loss, z, y) for z in zs])
    second = np.diff(d) / np.diff(zs)
    assert second.max() <= bound * (1 + 1e-6)
    assert second.max() >= bound * (1 - 1e-3)
    assert oracle.loss_curvature_bound(loss) == bound


def _brute_prox(v, bl, l1, l2, c, lo, hi):
    f = lambda u: 0.5 * bl * (u - v) ** 2 + l1 * abs(u) + 0.5 * l2 * u * u + c * u
    a = max(lo, -50.0)
    b = min(hi, 50.0)
    grid = np.linspace(a, b, 200001)
    vals = 0.5 * bl * (grid - v) ** 2 + l1 * np.abs(grid) + 0.5 * l2 * grid ** 2 + c * grid
    k = int(np.argmin(vals))
    lo_b, hi_b = grid[max(k - 1, 0)], grid[min(k + 1, grid.size - 1)]
    res = optimize.minimize_scalar(f, bounds=(lo_b, hi_b), method="bounded", options={"xatol": 1e-12})
    cands = [res.x, lo_b, hi_b, 0.0 if a <= 0.0 <= b else a]
    return min(cands, key=f)


def test_prox_matches_brute_force_minimisation():
    rng = np.random.default_rng(2)
    for _ in range(300):
        v = rng.normal() * 3
        bl = rng.uniform(0.1, 5)
        l1 = rng.choice([0.0, rng.uniform(0, 2)])
        l2 = rng.choice([0.0, rng.uniform(0, 3)])
        c = rng.choice([0.0, rng.normal()])
        lo, hi = rng.choice([(-np.inf, np.inf), (0.0, 1.0), (0.0, np.inf), (-0.5, 0.25)])
        got = oracle.model_prox(v, bl, l1, l2, c, lo, hi)
        want = _brute_prox(v, bl, l1, l2, c, lo, hi)
        assert got == pytest.approx(want, abs=2e-6)
        assert lo <= got <= hi


def test_square_l1_model_step_is_the_lasso_step():
    rng = np.random.default_rng(3)
    A = random_csc(40, 60, 4, rng)
    b = rng.standard_normal(40)
    lam = 0.2
    lasso = oracle.Solver(A, b, lam, tau=7, seed=4)
    model = oracle.ModelSolver(A, b, tau=7, seed=4, loss="square", l1=lam)
    assert model.beta == lasso.beta
    lasso.step(50)
    model.step(50)
    np.testing.assert_allclose(model.x, lasso.x, rtol=0, atol=1e-13)
    assert model.objective() == pytest.approx(lasso.objective(), rel=1e-13)


def _labels_problem(seed, m=120, n=40, d=6):
    rng = np.random.default_rng(seed)
    A = random_csc(m, n, d, rng, normalize=False)
    M = csc_to_dense(A)
    w = rng.standard_normal(n)
    y = np.sign(M @ w + 0.3 * rng.standard_normal(m))
    y[y == 0] = 1.0
    return A, M, y


def test_l2_logistic_reaches_the_lbfgs_optimum():
    """sum_j log(1 + exp(-y_j a_j^T x)) + lam ||x||^2 (the form of the logistic
    experiment): l2 = 2 lam."""
    A, M, y = _labels_problem(5)
    lam = 0.5

    def F(x):
        t = -y * (M @ x)
        return float(np.sum(np.logaddexp(0.0, t)) + lam * x @ x)

    def G(x):
        t = -y * (M @ x)
        return M.T @ (-y * 0.5 * (1 + np.tanh(t / 2))) + 2 * lam * x

    ref = optimize.minimize(F, np.zeros(A.n), jac=G, method="L-BFGS-B",
                            options={"gtol": 1e-12, "ftol": 1e-15, "maxiter": 10000})
    s = oracle.ModelSolver(A, y, tau=8, seed=1, loss="logistic", l2=2 * lam)
    s.step(3000 * s.steps_per_epoch())
    assert s.objective() == pytest.approx(ref.fun, rel=1e-10)
    np.testing.assert_allclose(s.x, ref.x, atol=1e-5)


@pytest.mark.parametrize("loss", ["logistic", "sqhinge"])
def test_l1_models_satisfy_kkt(loss):
    A, M, y = _labels_problem(7)
    l1 = 0.8
    s = oracle.ModelSolver(A, y, tau=5, seed=2, loss=loss, l1=l1)
    s.step(4000 * s.steps_per_epoch())
    z = M @ s.x
    if loss == "logistic":
        dphi = -y * 0.5 * (1 + np.tanh(-y * z / 2))
    else:
        dphi = -y * np.maximum(0.0, 1 - y * z)
    g = M.T @ dphi
    on = s.x != 0
    assert np.all(np.abs(g[~on]) <= l1 * (1 + 1e-7))
    np.testing.assert_allclose(g[on], -l1 * np.sign(s.x[on]), atol=1e-7)
    assert 0 < on.sum() < A.n


def test_svm_dual_closes_the_duality_gap():
    """SVM dual of the SVM experiment: minimise (1/(2 lam n^2)) x^T Z x - (1/n) sum x
    over 0 <= x <= 1, Z_ij = y_i y_j <A_i, A_j>.  In the form here the columns
    are the examples y_i A_i (features as rows), loss square with targets 0,
    scale 1/(lam n^2), linear term -1/n, box [0, 1].  At the dual optimum the
    primal hinge objective at w = (1/(lam n)) sum_i x_i y_i A_i equals the dual
    value (strong duality)."""
    rng = np.random.default_rng(9)
    d, n = 30, 200
    X = random_csc(d, n, 5, rng, normalize=False)      # column i: example A_i
    Xd = csc_to_dense(X)
    yl = np.sign(Xd.T @ rng.standard_normal(d) + 0.5 * rng.standard_normal(n))
    yl[yl == 0] = 1.0
    cols = CSC(m=d, n=n, col_ptr=X.col_ptr, row_idx=X.row_idx,
               values=X.values_f64() * np.repeat(yl, np.diff(X.col_ptr)))
    Yd = Xd * yl[None, :]
    lam = 0.01
    s = oracle.ModelSolver(cols, np.zeros(d), tau=8, seed=3, loss="square", scale=1.0 / (lam * n * n),
                           c=-1.0 / n, lo=0.0, hi=1.0)
    s.step(4000 * s.steps_per_epoch())
    xd = s.x
    assert np.all((xd >= 0) & (xd <= 1))
    dual = -s.objective()                                     # max of -f
    w = Yd @ xd / (lam * n)
    primal = np.mean(np.maximum(0.0, 1 - yl * (Xd.T @ w))) + 0.5 * lam * w @ w
    assert primal - dual >= -1e-12
    assert primal - dual <= 1e-8 * max(1.0, abs(primal))


def test_elastic_net_orthonormal_closed_form():
    """AᵀA = I: the minimiser of 0.5||Ax - b||^2 + l1||x||_1 + (l2/2)||x||^2 is
    soft(Aᵀb, l1)/(1 + l2) coordinate-wise."""
    A = orthonormal_block_hadamard(16, 4)
    M = csc_to_dense(A)
    rng = np.random.default_rng(4)
    b = rng.standard_normal(A.m) * 2
    l1, l2 = 0.7, 0.5
    s = oracle.ModelSolver(A, b, tau=4, seed=0, loss="square", l1=l1, l2=l2)
    s.step(500 * s.steps_per_epoch())
    atb = M.T @ b
    want = np.sign(atb) * np.maximum(np.abs(atb) - l1, 0) / (1 + l2)
    np.testing.assert_allclose(s.x, want, atol=1e-12)


def test_nonnegative_lasso_kkt():
    rng = np.random.default_rng(11)
    A = random_csc(50, 30, 5, rng)
    M = csc_to_dense(A)
    b = rng.standard_normal(50)
    l1 = 0.1
    s = oracle.ModelSolver(A, b, tau=6, seed=5, loss="square", l1=l1, lo=0.0)
    s.step(5000 * s.steps_per_epoch())
    g = M.T @ (M @ s.x - b)
    assert np.all(s.x >= 0)
    on = s.x > 0
    np.testing.assert_allclose(g[on], -l1, atol=1e-9)
    assert np.all(g[~on] >= -l1 - 1e-9)


def test_logistic_objective_at_zero_printed_value():
    """F(x_0) = 13,352,855 printed for the logistic experiment: with x_0 = 0
    every one of the 19,264,097 examples contributes log(1 + e^0)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")) as fh:
        g = json.load(fh)["kddb_logistic_F_x0"]
    m = g["examples"]
    A = CSC(m=m, n=1, col_ptr=np.array([0, 1], dtype=np.int64), row_idx=np.array([0], dtype=np.int32),
            values=np.array([1.0]))
    y = np.where(np.arange(m) % 2 == 0, 1.0, -1.0)
    s = oracle.ModelSolver(A, y, tau=1, seed=0, loss="logistic", l2=2.0)
    assert abs(s.objective() - g["F_x0_printed"]) <= g["printed_abs_tol"]
