"""Other samplings on the HIP path vs the float64 oracle: tau-independent
picks, (tau, p_b)-binomial availability, the drop mask (fault model) and the
doubly uniform beta (section "Block Samplings"; Table "ESO").

Tolerances as for the tau-nice path: float64 kernels 1e-10 relative on F and
1e-9 absolute on x; float32 kernels 1e-5 on F.  Sampler draws are integers
and compared bit for bit.
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


@pytest.mark.parametrize("seed,k,tau,n", [
    (0, 0, 1, 1), (3, 1, 3, 5), (9, 2, 17, 17), (1, 7, 8, 1000), (5, 11, 4000, 4097),
    (11, 123456789, 1_000_000, 10_000_000), (13, 2, 1000, 2**31 - 2),
])
def test_independent_draws_bit_exact(pc, seed, k, tau, n):
    _say(f"independent draws seed={seed} k={k} tau={tau} n={n}")
    got = pc.sample_draw("independent", seed, k, tau, n).cpu().numpy().astype(np.int64)
    assert np.array_equal(got, oracle.draw_independent(seed, k, tau, n))


@pytest.mark.parametrize("seed,k,tau,n,pb", [
    (0, 0, 1, 1, 1.0), (3, 1, 3, 5, 0.5), (1, 7, 8, 1000, 0.25), (5, 11, 4000, 4097, 0.9),
    (11, 99, 1_000_000, 10_000_000, 0.75), (2, 5, 100, 1000, 1e-3),
])
def test_binomial_draws_bit_exact(pc, seed, k, tau, n, pb):
    _say(f"binomial draws seed={seed} k={k} tau={tau} n={n} pb={pb}")
    got = pc.sample_draw("binomial", seed, k, tau, n, pb=pb).cpu().numpy().astype(np.int64)
    assert np.array_equal(got, oracle.draw_binomial(seed, k, tau, n, pb))


def test_beta_matches_oracle_per_sampling(pc):
    """The library's beta for each sampling (its own evaluation of the doubly
    uniform moments) vs the oracle's, on one matrix and many tau."""
    rng = np.random.default_rng(2)
    A = random_csc(300, 2000, 6, rng)
    b = rng.standard_normal(300)
    om = oracle.omega(A)
    with pc.Problem(A, b, 0.1, 1, seed=0) as p:
        for tau in (1, 2, 3, 17, 256, 1999, 2000):
            p.set_option("tau", tau)
            for sampling, pb in (("nice", 1.0), ("independent", 1.0), ("binomial", 0.3), ("binomial", 1.0)):
                p.set_sampling(sampling, pb)
                inf = p.info()
                want = oracle.beta_for(sampling, om, tau, 2000, pb)
                assert inf["beta"] == pytest.approx(want, rel=1e-12), (tau, sampling, pb)
                if sampling == "independent":
                    assert inf["expected_set_size"] == pytest.approx(
                        oracle.independent_moments(tau, 2000)[0], rel=1e-12)


def _run_pair(pc, inst, tau, seed, sampling, pb, mask, steps, chunks, rtol_F, x_atol, dtype="f64"):
    A = inst.A if dtype == "f64" else inst.A.astype(dtype)
    ref = oracle.Solver(A, inst.b, inst.lam, tau=tau, seed=seed, sampling=sampling, pb=pb, mask=mask)
    with pc.Problem(A, inst.b, inst.lam, tau, seed=seed) as p:
        p.set_sampling(sampling, pb)
        if mask is not None:
            p.set_slot_mask(mask)
        assert p.info()["beta"] == pytest.approx(ref.beta, rel=1e-12)
        worst = 0.0
        for _ in range(chunks):
            p.step(steps)
            ref.step(steps)
            F, _ = p.objective()
            Fr = ref.objective()
            worst = max(worst, abs(F - Fr) / abs(Fr))
            assert abs(F - Fr) <= rtol_F * abs(Fr)
        if x_atol is not None:
            np.testing.assert_allclose(p.get_x(), ref.x, rtol=0, atol=x_atol)
        return worst


@pytest.mark.parametrize("sampling,pb,tau", [
    ("independent", 1.0, 1), ("independent", 1.0, 8), ("independent", 1.0, 1000),
    ("binomial", 0.5, 8), ("binomial", 0.9, 333), ("binomial", 0.05, 1000),
])
def test_small_config_float64(pc, sampling, pb, tau):
    """The 2000 x 1000 configuration: tau = n = 1000 with independent picks
    has many repeated picks per step (E|S| = 632)."""
    inst = make_config("small_2000x1000", dtype="f64")
    _say(f"small f64 {sampling} pb={pb} tau={tau}")
    spe = -(-1000 // tau)
    worst = _run_pair(pc, inst, tau, 0, sampling, pb, None, 5 * spe, 8, 1e-10, 1e-9)
    _say(f"  worst rel F diff {worst:.2e}")


@pytest.mark.parametrize("sampling", ["nice", "independent", "binomial"])
def test_ragged_float32(pc, sampling):
    rng = np.random.default_rng(7)
    A = random_csc_ragged(500, 777, 1, 37, rng, dtype="f32")
    inst = planted_lasso(A, 30, 0.01, 0.05, rng)
    worst = _run_pair(pc, inst, 100, 4, sampling, 0.7, None, 40, 5, 1e-5, None, dtype="f32")
    _say(f"ragged f32 {sampling}: worst {worst:.2e}")


@pytest.mark.parametrize("sampling", ["nice", "independent", "binomial"])
def test_drop_mask_matches_oracle(pc, sampling):
    """Slots 0, 5, 63, 64 and 199 down (tile edges included), mask shorter
    than tau, so slots >= 230 stay alive."""
    rng = np.random.default_rng(9)
    A = random_csc_ragged(600, 900, 2, 20, rng)
    inst = planted_lasso(A, 25, 0.01, 0.05, rng)
    mask = np.ones(230, np.uint8)
    mask[[0, 5, 63, 64, 199]] = 0
    worst = _run_pair(pc, inst, 256, 2, sampling, 0.6, mask, 12, 5, 1e-10, 1e-9)
    _say(f"mask {sampling}: worst {worst:.2e}")


def test_fault_injection_converges_and_mask_clears(pc):
    """A quarter of the slots down from the start: PCDM still reaches a
    certified 1e-9 gap (the tau-nice beta over-damps the smaller sets);
    removing the mask returns to the oracle's unmasked trajectory."""
    rng = np.random.default_rng(12)
    A = random_csc(800, 1200, 8, rng)
    inst = planted_lasso(A, 40, 0.01, 0.1, rng)
    mask = (rng.random(128) >= 0.25).astype(np.uint8)
    with pc.Problem(inst.A, inst.b, inst.lam, 128, seed=5) as p:
        p.set_slot_mask(mask)
        assert p.info()["mask_len"] == 128
        st = p.solve(rel_gap=1e-9, check_every=5, max_epochs=5000)
        _say(f"fault injection: {st}")
        assert st["converged"]
        p.set_slot_mask(None)
        assert p.info()["mask_len"] == 0
        x0 = p.get_x()
        k0 = p.info()["k"]
        ref = oracle.Solver(inst.A, inst.b, inst.lam, tau=128, seed=5, x0=x0)
        ref.k = k0
        p.step(30)
        ref.step(30)
        np.testing.assert_allclose(p.get_x(), ref.x, rtol=0, atol=1e-9)


def test_independent_claims_restart_after_set_x(pc):
    """Rewinding the step counter must not leave stale claims: a rewound run
    retraces the original trajectory exactly."""
    inst = make_config("small_2000x1000", dtype="f64")
    with pc.Problem(inst.A, inst.b, inst.lam, 500, seed=3) as p:
        p.set_sampling("independent")
        p.step(20)
        x1 = p.get_x()
        p.set_x(np.zeros(inst.A.n), k=0)
        p.step(20)
        np.testing.assert_allclose(p.get_x(), x1, rtol=0, atol=1e-12)


def test_invalid_sampling_options(pc):
    from paper_1212_0873_amd import PCDMError
    rng = np.random.default_rng(0)
    A = random_csc(20, 30, 3, rng)
    with pc.Problem(A, rng.standard_normal(20), 0.1, 4, seed=0) as p:
        for key, val in (("sampling", 3), ("sampling", 0.5), ("binomial_p", 0.0), ("binomial_p", 1.5)):
            with pytest.raises(PCDMError):
                p.set_option(key, val)
        with pytest.raises(PCDMError):
            p.set_slot_mask(np.ones(31, np.uint8))  # longer than n
    with pytest.raises(PCDMError):
        pc.sample_draw("binomial", 0, 0, 4, 10, pb=0.0)


def test_full_size_independent_steps_match_oracle(pc):
    """1e6 x 1e7 (2e8 nonzeros, float32 values), tau = 1e6 independent picks
    (E|S| = 951,626): three steps, F within 1e-5 of the oracle and x within
    1e-5 of its scale."""
    inst = make_config("lasso_1e6x1e7", dtype="f32", tau=10**6)
    _say("full size generated")
    tau = 10**6
    ref = oracle.Solver(inst.A, inst.b, inst.lam, tau=tau, seed=0, sampling="independent")
    with pc.Problem(inst.A, inst.b, inst.lam, tau, seed=0) as p:
        p.set_sampling("independent")
        assert p.info()["beta"] == pytest.approx(ref.beta, rel=1e-12)
        p.step(3)
        ref.step(3)
        x = p.get_x()
        F, _ = p.objective()
    Fr = ref.objective()
    _say(f"full size independent: F {F:.10e} oracle {Fr:.10e}, changed {ref.changed}")
    assert F == pytest.approx(Fr, rel=1e-5)
    scale = np.max(np.abs(ref.x))
    assert np.max(np.abs(x - ref.x)) <= 1e-5 * scale
    assert np.array_equal(x != 0, ref.x != 0) or np.sum((x != 0) != (ref.x != 0)) <= 10
