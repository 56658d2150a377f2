"""Asynchronous variant on the HIP path (section "Numerical experiments",
billion-variable LASSO: cores read the current iterate when ready, apply
updates at once, and pick blocks uniformly and independently).

With one processor the launch is serial coordinate descent over its pick
stream, which the oracle reproduces: compared at the float64 bar (1e-10).
With many processors the trajectory depends on timing, so the checks are
what holds for any interleaving: no update is lost (the stored residual
equals A x - b recomputed), and the iterates converge to the optimum the
oracle certifies.
"""

import numpy as np
import pytest

import oracle
from workloads import make_config, planted_lasso, random_csc, random_csc_ragged

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


@pytest.mark.parametrize("dtype,lanes", [("f64", 0), ("f64", 1), ("f64", 64), ("f32", 0), ("bf16", 8)])
def test_one_processor_is_the_serial_pick_stream(pc, dtype, lanes):
    rng = np.random.default_rng(31)
    A = random_csc_ragged(300, 500, 1, 30, rng, dtype=dtype)
    inst = planted_lasso(A, 20, 0.01, 0.05, rng)
    ref = oracle.Solver(inst.A, inst.b, inst.lam, tau=1, seed=6)
    with pc.Problem(inst.A, inst.b, inst.lam, 1, seed=6) as p:
        p.set_option("async_processors", 1)
        if lanes:
            p.set_option("lanes_per_column", lanes)
        assert p.info()["beta"] == 1.0
        for launch in range(6):
            p.step_async(1, picks_per_epoch=700)
            ref.async_serial(launch, 700)
            F, _ = p.objective()
            if dtype == "f64":
                assert F == pytest.approx(ref.objective(), rel=1e-10)
            else:
                assert F == pytest.approx(ref.objective(), rel=1e-5)
        inf = p.info()
        assert inf["async_picks"] == 4200 and inf["async_processors"] == 1
        if dtype == "f64":
            np.testing.assert_allclose(p.get_x(), ref.x, rtol=0, atol=1e-9)


@pytest.mark.parametrize("dtype,reads,rounds,procs", [
    ("f64", 0, 0, 0), ("f64", 1, 0, 0), ("f64", 2, 0, 0), ("f32", 0, 1, 0), ("f32", 2, 0, 0),
    ("f64", 0, 0, 300), ("f64", 1, 0, 300), ("f64", 2, 0, 300), ("f32", 0, 0, 300), ("f64", 0, 0, 5000),
    ("bf16", 1, 0, 300), ("bf16", 0, 4, 0),
])
def test_no_update_is_lost(pc, dtype, reads, rounds, procs):
    """Many processors, refresh off: the residual the atomics maintained equals
    A x - b recomputed from the x the processors wrote (float64: to rounding;
    float32: to the atomics' rounding), and no x_i is left holding the lock
    pattern.  With 300 processors a launch of 6000 picks has 20 rounds, so
    blocks are picked again and again inside one launch, from every XCD."""
    rng = np.random.default_rng(5)
    A = random_csc(4000, 6000, 10, rng, dtype=dtype)
    inst = planted_lasso(A, 80, 0.01, 0.05, rng)
    S = _sparse(inst.A)
    with pc.Problem(inst.A, inst.b, inst.lam, 6000, seed=2) as p:
        p.set_option("refresh_every", 0)
        p.set_option("async_reads", reads)
        p.set_option("async_rounds", rounds)
        p.set_option("async_processors", procs)
        for _ in range(5):
            p.step_async(1)
        inf = p.info()
        _say(f"{dtype} reads={reads} rounds={rounds}: processors {inf['async_processors']}, "
             f"changed {inf['nonzero_updates']}")
        assert inf["async_processors"] == (procs or 6000)
        x = p.get_x()
        r = p.get_residual()
    assert np.all(np.isfinite(x))
    recomputed = S @ x - inst.b
    tol = 1e-12 if dtype == "f64" else 2e-5   # bf16 values are exact in float32: same bar
    assert np.max(np.abs(r - recomputed)) <= tol * max(1.0, np.max(np.abs(inst.b)))


@pytest.mark.parametrize("dtype,tau,reads", [("f64", 64, 0), ("f64", 64, 1), ("f64", 64, 2), ("f64", 1000, 0),
                                             ("f32", 1000, 0)])
def test_converges_to_the_certified_optimum(pc, dtype, tau, reads):
    """The 2000 x 1000 configuration: epochs of the asynchronous variant reach a
    certified gap, and F matches the oracle's optimum (oracle run to a 1e-13
    gap) within the gap."""
    inst = make_config("small_2000x1000", dtype=dtype)
    ref = oracle.Solver(inst.A, inst.b, inst.lam, tau=8, seed=0)
    for _ in range(200):
        ref.step(20 * ref.steps_per_epoch())
        gap, Fr, _ = ref.gap()
        if gap <= 1e-13 * Fr:
            break
    target = 1e-10 if dtype == "f64" else 1e-6
    with pc.Problem(inst.A, inst.b, inst.lam, tau, seed=1) as p:
        p.set_option("async_reads", reads)
        for epoch in range(1, 3001):
            p.step_async(1)
            if epoch % 10 == 0:
                F, gap = p.objective(gap=True)
                if gap <= target * F:
                    break
        _say(f"{dtype} tau={tau} reads={reads}: {epoch} epochs, F {F:.12e} vs oracle {Fr:.12e}, gap {gap:.2e}")
        assert gap <= target * F
    assert F == pytest.approx(Fr, rel=2 * target)


def test_async_options_and_counters(pc):
    from paper_1212_0873_amd import PCDMError
    rng = np.random.default_rng(0)
    A = random_csc(40, 60, 3, rng)
    with pc.Problem(A, rng.standard_normal(40), 0.1, 8, seed=0) as p:
        for key, val in (("async_processors", -1), ("async_reads", 3), ("async_rounds", 0.5)):
            with pytest.raises(PCDMError):
                p.set_option(key, val)
        p.step_async(1, picks_per_epoch=0)
        assert p.info()["async_picks"] == 0
        p.step_async(2)
        inf = p.info()
        assert inf["async_picks"] == 120 and inf["k"] == 0
        assert 1 <= inf["async_processors"] <= 8
