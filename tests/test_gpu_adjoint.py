"""Adjoint (dL/db, dL/dlambda through the LASSO solution) on the GPU vs the
float64 oracle's support solve, plus finite differences at full size.

Each side differentiates its own converged solution (the oracle never sees a
GPU iterate); the two solutions agree to the solve tolerance, so the
gradients are compared at a tolerance that covers it.
"""

import numpy as np
import pytest

import oracle
from workloads import make_config, random_csc

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


def _sparse(A):
    import scipy.sparse as sp
    return sp.csc_matrix((A.values_f64(), A.row_idx, A.col_ptr), shape=(A.m, A.n))


def _val_loss_grad(V, xstar):
    """L(x) = ||V (x - x*)||^2 and its gradient 2 V^T V (x - x*)."""
    def f(x):
        d = V @ (x - xstar)
        return float(d @ d), 2.0 * (V.T @ d)
    return f


def _oracle_solution(inst, tau, tol=1e-13, seed=0):
    s = oracle.Solver(inst.A, inst.b, inst.lam, tau=tau, seed=seed)
    for _ in range(2000):
        s.step(5 * s.steps_per_epoch())
        gap, F, _ = s.gap()
        if gap <= tol * F:
            break
    return s.x.copy()


@pytest.fixture(scope="module")
def scaled():
    inst = make_config("train_1e5x1e6", scale=0.02, dtype="f64")  # 2000 x 20000, 10 nnz/col
    rng = np.random.default_rng(11)
    V = _sparse(random_csc(400, inst.A.n, 10, rng, normalize=False))
    return inst, V


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-7), ("f32", 1e-4)])
def test_adjoint_matches_oracle(pc, scaled, dtype, tol):
    inst, V = scaled
    A = inst.A.astype(dtype)
    loss = _val_loss_grad(V, inst.xstar)
    x_ref = _oracle_solution(type(inst)(A=A, b=inst.b, lam=inst.lam), tau=256)
    want_db, want_dl = oracle.lasso_adjoint(A, x_ref, loss(x_ref)[1])
    with pc.Problem(A, inst.b, inst.lam, 256, seed=1) as p:
        p.set_option("adj_tol", 1e-10)
        st = p.solve(rel_gap=1e-12 if dtype == "f64" else 1e-6, check_every=5, max_epochs=20000)
        assert st["converged"], st
        x = p.get_x()
        got_db, got_dl = p.grad_backward(loss(x)[1])
    _say(f"{dtype}: solve {st}, support {np.count_nonzero(x)} vs {np.count_nonzero(x_ref)}")
    assert np.array_equal(x != 0, x_ref != 0)
    scale = np.max(np.abs(want_db))
    err = np.max(np.abs(got_db - want_db)) / scale
    _say(f"  dL/db rel err {err:.2e}; dL/dlambda {got_dl:.9e} vs {want_dl:.9e}")
    assert err <= tol
    assert got_dl == pytest.approx(want_dl, rel=tol)


def test_autograd_function(pc, scaled):
    import torch
    from paper_1212_0873_amd.autograd import lasso
    inst, V = scaled
    A = inst.A
    x_ref = _oracle_solution(inst, tau=256)
    loss = _val_loss_grad(V, inst.xstar)
    want_db, want_dl = oracle.lasso_adjoint(A, x_ref, loss(x_ref)[1])
    Vt = torch.tensor(V.toarray(), dtype=torch.float64, device="cuda")
    with pc.Problem(A, inst.b, inst.lam, 256, seed=1) as p:
        p.set_option("adj_tol", 1e-10)
        b = torch.tensor(inst.b, device="cuda", requires_grad=True)
        lam = torch.tensor(inst.lam, dtype=torch.float64, device="cuda", requires_grad=True)
        x = lasso(p, b, lam, rel_gap=1e-12)
        d = Vt @ (x - torch.tensor(inst.xstar, device="cuda")).unsqueeze(1)
        L = (d * d).sum()
        L.backward()
    err = (b.grad.cpu().numpy() - want_db)
    assert np.max(np.abs(err)) <= 1e-7 * np.max(np.abs(want_db))
    assert lam.grad.item() == pytest.approx(want_dl, rel=1e-7)


def test_adjoint_empty_support_and_zero_gradient(pc):
    rng = np.random.default_rng(5)
    A = random_csc(50, 40, 4, rng)
    b = rng.standard_normal(50)
    lam_big = 1e6
    with pc.Problem(A, b, lam_big, 8, seed=0) as p:
        p.step(50)
        assert np.count_nonzero(p.get_x()) == 0
        db, dl = p.grad_backward(rng.standard_normal(40))
    assert np.all(db == 0) and dl == 0.0


def test_full_size_adjoint_finite_differences(pc):
    """1e5 x 1e6 training matrix (10 nnz/col, float64 path so that the finite
    differences resolve h = 1e-4): the adjoint converges and matches central
    differences of the warm-started solves along random directions of b and
    in lambda."""
    inst = make_config("train_1e5x1e6", dtype="f64", tau=4096)
    rng = np.random.default_rng(3)
    V = _sparse(random_csc(20000, inst.A.n, 10, rng, normalize=False))
    loss = _val_loss_grad(V, inst.xstar)
    h = 1e-4
    with pc.Problem(inst.A, inst.b, inst.lam, 4096, seed=2) as p:
        st = p.solve(rel_gap=1e-13, check_every=10, max_epochs=20000)
        _say(f"forward: {st}")
        assert st["converged"], st
        x0 = p.get_x()
        L0, g = loss(x0)
        db, dl = p.grad_backward(g)
        _say(f"support {np.count_nonzero(x0)}, dL/dlambda {dl:.6e}")

        def L_at(b, lam):
            p.set_rhs(b)
            p.set_option("lambda", lam)
            r = p.solve(rel_gap=1e-14, check_every=10, max_epochs=20000)
            assert r["converged"], r
            return loss(p.get_x())[0]

        for _ in range(2):
            d = rng.standard_normal(inst.A.m)
            d /= np.linalg.norm(d)
            fd = (L_at(inst.b + h * d, inst.lam) - L_at(inst.b - h * d, inst.lam)) / (2 * h)
            _say(f"dir: fd {fd:.8e} adjoint {db @ d:.8e}")
            assert fd == pytest.approx(db @ d, rel=1e-3, abs=1e-6 * max(1.0, abs(L0)))
        fd = (L_at(inst.b, inst.lam + h) - L_at(inst.b, inst.lam - h)) / (2 * h)
        _say(f"lambda: fd {fd:.8e} adjoint {dl:.8e}")
        assert fd == pytest.approx(dl, rel=1e-3)


def test_full_size_float32_adjoint_matches_oracle(pc):
    """1e5 x 1e6 training matrix with float32 values: the float32 forward
    solve (float32 A and r, float64 refresh and x) to a certified 1e-7 gap,
    then dL/db and dL/dlambda of the validation loss through the library's
    adjoint, against the oracle's float64 support solve at the oracle's own
    solution on the same stored values (same support and signs)."""
    import time
    inst = make_config("train_1e5x1e6", dtype="f32", tau=4096)
    rng = np.random.default_rng(3)
    V = _sparse(random_csc(20000, inst.A.n, 10, rng, normalize=False))
    loss = _val_loss_grad(V, inst.xstar)
    t0 = time.time()
    x_ref = _oracle_solution(inst, tau=4096, tol=1e-11)
    want_db, want_dl = oracle.lasso_adjoint(inst.A, x_ref, loss(x_ref)[1])
    _say(f"oracle: support {np.count_nonzero(x_ref)} ({time.time() - t0:.0f} s)")
    with pc.Problem(inst.A, inst.b, inst.lam, 4096, seed=2) as p:
        p.set_option("adj_tol", 1e-9)
        st = p.solve(rel_gap=1e-7, check_every=5, max_epochs=4000)
        _say(f"forward: {st}")
        assert st["converged"], st
        x = p.get_x()
        got_db, got_dl = p.grad_backward(loss(x)[1])
    assert np.array_equal(np.sign(x), np.sign(x_ref))
    err = np.max(np.abs(got_db - want_db)) / np.max(np.abs(want_db))
    _say(f"dL/db rel err {err:.2e}; dL/dlambda {got_dl:.9e} vs {want_dl:.9e}")
    assert err <= 1e-4
    assert got_dl == pytest.approx(want_dl, rel=1e-4)
