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


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_batch_gap_incremental_max(pc, dtype):
    """The batched gap takes ||A_j^T r_j||_inf from the columns whose kept
    bound, moved by ||a_i|| times the change of r, can still reach the
    maximum.  At every check it equals the gap computed by scipy at the
    batch's own x (to the float64 refresh's rounding), late checks sum only
    a fraction of the columns, and the full pass (max_passes = 1) on a second
    handle that follows the same float64 trajectory gives the same gaps."""
    probs = _problems(dtype, seed=5)
    total_n = sum(A.n for A, _, _, _ in probs)
    cands = []
    with pc.Batch(probs, seed=2) as B:
        for rnd in range(10):
            B.step(25 if rnd < 8 else 1)  # the last two checks: one step apart
            F, gap = B.objective()
            for j, (A, b, lam, tau) in enumerate(probs):
                g_ref, _ = _scipy_gap(A, b, B.get_x(j), lam)
                assert gap[j] == pytest.approx(g_ref, rel=1e-8, abs=1e-12 * abs(F[j])), (rnd, j)
            cands.append(sum(B.info(j)["max_candidates"] for j in range(len(probs))))
        hits = [B.info(j)["max_incremental"] for j in range(len(probs))]
    assert min(hits) == 10, hits
    assert max(cands) <= total_n and cands[-1] < total_n // 4, (cands, total_n)
    if dtype == "f64":
        # float64 steps: both handles follow the oracle's trajectory to 1e-9
        with pc.Batch(probs, seed=2) as B1:
            B1.set_option("max_passes", 1)
            for rnd in range(10):
                B1.step(25 if rnd < 8 else 1)
                F1, gap1 = B1.objective()
            assert all(B1.info(j)["max_incremental"] == 0 for j in range(len(probs)))
            assert all(B1.info(j)["max_candidates"] == A.n for j, (A, _, _, _) in enumerate(probs))
        np.testing.assert_allclose(gap1, gap, rtol=1e-7, atol=1e-12 * np.abs(F).max())


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("f64", 1e-10)])
def test_batched_path_shape_matches_oracle(pc, dtype, tol):
    """The batched regularisation-path workload at its real shape: 64
    problems with n_j log-uniform on [1e3, 1e6] (m_j = n_j/5, 10 entries per
    column), lambda_j on the geometric grid, tau_j = min(n_j, 4096), one
    batch.  Every problem against the oracle run alone with the batch's key
    (seed + j) for 490 steps (two epochs of the largest problem; hundreds of
    the smallest), F at five checks; float64 values also x; at the end every
    certified gap against scipy's at the batch's own x."""
    import time

    from workloads.configs import batched_path
    t0 = time.time()
    insts = batched_path(64, seed=0, dtype=dtype)
    probs = [(i.A, i.b, i.lam, min(i.A.n, 4096)) for i in insts]
    ns = [A.n for A, _, _, _ in probs]
    _say(f"{dtype}: 64 problems, n {min(ns)} .. {max(ns)}, sum n {sum(ns)} ({time.time() - t0:.0f} s)")
    refs = [oracle.Solver(A, b, lam, tau=tau, seed=11 + j) for j, (A, b, lam, tau) in enumerate(probs)]
    with pc.Batch(probs, seed=11) as B:
        for j, r in enumerate(refs):
            inf = B.info(j)
            assert inf["omega"] == r.omega and inf["beta"] == pytest.approx(r.beta, rel=1e-15), j
        for rnd in range(5):
            steps = 98
            B.step(steps)
            for r in refs:
                r.step(steps)
            F, gap = B.objective()
            worst = 0.0
            for j, r in enumerate(refs):
                Fr = r.objective()
                worst = max(worst, abs(F[j] - Fr) / abs(Fr))
                assert F[j] == pytest.approx(Fr, rel=tol), (rnd, j)
            _say(f"  check {rnd}: worst rel F error {worst:.2e} ({time.time() - t0:.0f} s)")
        if dtype == "f64":
            for j, r in enumerate(refs):
                np.testing.assert_allclose(B.get_x(j), r.x, atol=1e-9, err_msg=str(j))
        for j, (A, b, lam, tau) in enumerate(probs):
            g_ref, _ = _scipy_gap(A, b, B.get_x(j), lam)
            assert gap[j] == pytest.approx(g_ref, rel=1e-6, abs=1e-10 * abs(F[j])), j
        assert all(B.info(j)["k"] == 490 for j in range(64))


def _say(msg):
    print(msg, flush=True)
