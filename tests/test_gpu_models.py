"""Other losses and regularisers on the HIP path vs the float64 oracle
(introduction: the table of three losses; numerical experiments: SVM dual
with box constraints, L2-regularised logistic regression).

The library folds labels into the stored values and keeps margins; the
oracle keeps z = A x and applies the labels in the loss, so the two share
no arithmetic beyond the definitions.  Tolerances as for the LASSO path:
float64 1e-10 relative on F and 1e-9 on x, float32 1e-5 on F.
"""

import numpy as np
import pytest

import oracle
from workloads import CSC, csc_to_dense, make_config, random_csc, random_csc_ragged

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    import torch
    assert torch.cuda.is_available()
    import paper_1212_0873_amd as pc
    pc.load()
    return pc


def _say(msg):
    print(msg, flush=True)


def _classification(seed, m, n, dmin, dmax, dtype="f64"):
    rng = np.random.default_rng(seed)
    A = random_csc_ragged(m, n, dmin, dmax, rng, dtype=dtype)
    M = csc_to_dense(A) if m * n <= 4e6 else None
    w = np.zeros(n)
    sup = rng.choice(n, size=max(1, n // 20), replace=False)
    w[sup] = rng.standard_normal(sup.size)
    import scipy.sparse as sp
    S = sp.csc_matrix((A.values_f64(), A.row_idx, A.col_ptr), shape=(m, n))
    y = np.sign(S @ w + 0.1 * rng.standard_normal(m))
    y[y == 0] = 1.0
    return A, y, M


MODELS = [
    ("logistic_l1", "logistic", dict(), 0.05),
    ("logistic_l2", "logistic", dict(l2=2.0), 0.0),
    ("logistic_l1_l2", "logistic", dict(l2=0.5), 0.02),
    ("sqhinge_l1", "sqhinge", dict(), 0.05),
    ("sqhinge_box", "sqhinge", dict(lower=-0.3, upper=0.3), 0.0),
]


def _run_pair(pc, A, y, loss, extra, l1, tau, seed, steps, chunks, rtol_F, x_atol, lanes=0):
    kw = dict(scale=extra.get("scale", 1.0), l1=l1, l2=extra.get("l2", 0.0), c=extra.get("linear", 0.0),
              lo=extra.get("lower", -np.inf), hi=extra.get("upper", np.inf))
    ref = oracle.ModelSolver(A, y, tau=tau, seed=seed, loss=loss, **kw)
    model = dict(loss=loss, **extra)
    with pc.Problem(A, y, l1, tau, seed=seed, model=model) as p:
        if lanes:
            p.set_option("lanes_per_column", lanes)
        inf = p.info()
        assert inf["beta"] == pytest.approx(ref.beta, rel=1e-15)
        assert inf["loss"] == oracle.LOSSES[loss]
        worst = 0.0
        for _ in range(chunks):
            p.step(steps)
            ref.step(steps)
            F, _ = p.objective()
            Fr = ref.objective()
            worst = max(worst, abs(F - Fr) / abs(Fr))
            assert abs(F - Fr) <= rtol_F * abs(Fr), (F, Fr)
        if x_atol is not None:
            np.testing.assert_allclose(p.get_x(), ref.x, rtol=0, atol=x_atol)
        return worst


@pytest.mark.parametrize("name,loss,extra,l1", MODELS, ids=[m[0] for m in MODELS])
@pytest.mark.parametrize("tau", [7, 300])
def test_models_float64_match_oracle(pc, name, loss, extra, l1, tau):
    A, y, _ = _classification(3, 900, 700, 1, 30)
    worst = _run_pair(pc, A, y, loss, extra, l1, tau, 5, 3 * (-(-700 // tau)), 6, 1e-10, 1e-9)
    _say(f"{name} tau={tau}: worst rel F diff {worst:.2e}")


@pytest.mark.parametrize("name,loss,extra,l1", MODELS, ids=[m[0] for m in MODELS])
def test_models_float32_match_oracle(pc, name, loss, extra, l1):
    A, y, _ = _classification(4, 1500, 1000, 2, 25, dtype="f32")
    worst = _run_pair(pc, A, y, loss, extra, l1, 64, 2, 40, 5, 1e-5, None)
    _say(f"{name} f32: worst rel F diff {worst:.2e}")


@pytest.mark.parametrize("lanes", [1, 4, 16, 64])
def test_models_every_lane_count(pc, lanes):
    A, y, _ = _classification(8, 500, 400, 1, 45)
    _run_pair(pc, A, y, "logistic", dict(l2=0.3), 0.01, 50, 3, 16, 3, 1e-10, 1e-9, lanes=lanes)


def test_square_loss_models_match_oracle(pc):
    """Elastic net with a box and a linear term on the square loss."""
    inst = make_config("small_2000x1000", dtype="f64")
    extra = dict(l2=0.3, linear=0.01, lower=-0.5, upper=2.0)
    _run_pair(pc, inst.A, inst.b, "square", extra, inst.lam, 8, 0, 500, 6, 1e-10, 1e-9)


def test_svm_dual_matches_oracle(pc):
    """The SVM dual (box [0, 1], linear -1/n, scale 1/(lambda n^2)) on
    label-scaled example columns."""
    rng = np.random.default_rng(6)
    d, n = 300, 2000
    X = random_csc(d, n, 8, rng, normalize=False)
    Xd = csc_to_dense(X)
    yl = np.sign(Xd.T @ rng.standard_normal(d) + 0.5 * rng.standard_normal(n))
    yl[yl == 0] = 1.0
    cols = CSC(m=d, n=n, col_ptr=X.col_ptr, row_idx=X.row_idx,
               values=X.values_f64() * np.repeat(yl, np.diff(X.col_ptr)))
    lam = 1e-3
    extra = dict(scale=1.0 / (lam * n * n), linear=-1.0 / n, lower=0.0, upper=1.0)
    worst = _run_pair(pc, cols, np.zeros(d), "square", extra, 0.0, 64, 1, 60, 5, 1e-10, 1e-9)
    _say(f"svm dual: worst {worst:.2e}")


def test_lasso_through_the_model_entry_is_the_same_path(pc):
    """pcdm_create_model with {square, 1, lambda} runs the same arithmetic as
    pcdm_create: identical x after the same steps."""
    inst = make_config("small_2000x1000", dtype="f32")
    with pc.Problem(inst.A, inst.b, inst.lam, 8, seed=0) as a, \
            pc.Problem(inst.A, inst.b, inst.lam, 8, seed=0, model=dict(loss="square")) as b:
        a.step(700)
        b.step(700)
        assert np.array_equal(a.get_x(), b.get_x())
        Fa, ga = a.objective(gap=True)
        Fb, _ = b.objective()
        assert Fa == Fb


def test_model_error_paths(pc):
    from paper_1212_0873_amd import PCDMError
    A, y, _ = _classification(1, 60, 50, 2, 6)
    bad = y.copy()
    bad[3] = 0.5
    with pytest.raises(PCDMError, match="label"):
        pc.Problem(A, bad, 0.1, 4, model=dict(loss="logistic"))
    for model in (dict(loss="logistic", lower=0.5), dict(loss="sqhinge", upper=-1.0),
                  dict(loss="square", scale=0.0), dict(loss="square", l2=-1.0)):
        with pytest.raises(PCDMError):
            pc.Problem(A, y, 0.1, 4, model=model)
    with pytest.raises(PCDMError):
        pc.Problem(A, y, -0.1, 4, model=dict(loss="logistic"))
    with pc.Problem(A, y, 0.1, 4, model=dict(loss="logistic")) as p:
        with pytest.raises(PCDMError, match="duality gap"):
            p.objective(gap=True)
        with pytest.raises(PCDMError):
            p.step_async(1)
        with pytest.raises(PCDMError):
            p.grad_backward(np.ones(50))
        with pytest.raises(PCDMError):
            p.set_rhs(y)
        with pytest.raises(PCDMError):
            p.set_option("chunks_per_lane", 2)
        p.step(5)
        F, _ = p.objective()
        assert np.isfinite(F)


def test_logistic_l2_converges_to_the_oracle_optimum(pc):
    """Strongly convex: the GPU run and the oracle's long run reach the same
    minimiser (float64)."""
    A, y, _ = _classification(11, 800, 300, 2, 20)
    ref = oracle.ModelSolver(A, y, tau=16, seed=0, loss="logistic", l2=1.0)
    ref.step(3000 * ref.steps_per_epoch())
    with pc.Problem(A, y, 0.0, 64, seed=9, model=dict(loss="logistic", l2=1.0)) as p:
        p.step(3000 * (-(-300 // 64)))
        x = p.get_x()
        F, _ = p.objective()
    assert F == pytest.approx(ref.objective(), rel=1e-12)
    np.testing.assert_allclose(x, ref.x, atol=1e-7)
