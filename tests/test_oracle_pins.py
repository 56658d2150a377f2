"""Pins of the float64 oracle against facts the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
own formula: they use printed values, closed forms, brute force and exact
enumeration over all tau-subsets.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle
from tests import pins
from workloads import (csc_to_dense, dense_to_csc, make_config, orthonormal_block_hadamard, planted_lasso,
                       random_csc, separable_matrix, tightness_matrix)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# --------------------------------------------------------------------------- #
# beta (Table ESO)
# --------------------------------------------------------------------------- #

def test_beta_rcv1_printed_values():
    """rcv1 paragraph of the SVM experiment: beta = 7.46 and PSF = 2.15 at tau = 16."""
    g = _gold("paper_printed_values.json")["rcv1_nice_beta"]
    beta = oracle.beta_nice(g["omega"], g["tau"], g["n"])
    assert abs(beta - g["beta_printed"]) <= g["printed_abs_tol"]
    assert abs(g["tau"] / beta - g["psf_printed"]) <= g["printed_abs_tol"]


def test_beta_special_cases():
    """Table ESO: serial (tau = 1) gives 1, fully parallel (tau = n) gives omega,
    separable f (omega = 1) gives 1 for every tau; n = 1 uses max(1, n-1)."""
    for n in (2, 7, 1000):
        for omega in (1, 2, n):
            assert oracle.beta_nice(omega, 1, n) == 1.0
            assert oracle.beta_nice(omega, n, n) == pytest.approx(omega, rel=1e-15)
            assert oracle.beta_nice(1, n // 2 + 1, n) == 1.0
    assert oracle.beta_nice(1, 1, 1) == 1.0
    # the conservative rule is never smaller (remark after the uniform-ESO theorem)
    for n, omega, tau in [(10, 3, 5), (1000, 35, 24), (50, 50, 7)]:
        assert oracle.beta_uniform(omega, tau) >= oracle.beta_nice(omega, tau, n)
        assert oracle.beta_uniform(omega, tau) == min(omega, tau)


@pytest.mark.parametrize("tau", [1, 2, 3, 4, 5, 6, 7, 8])
def test_eso_is_tight_on_tightness_matrix(tau):
    """Tightness construction after the DSO theorem (0-1 A, omega ones per row,
    k per column) with h = k^{-1/2} 1: the exact mean over all tau-subsets of
    0.5 h_S^T A^T A h_S equals (tau/2n) beta ||h||_L^2 for the tau-nice beta.
    A wrong beta (e.g. without the max(1, n-1) or with omega and tau swapped
    in one factor) breaks the equality."""
    n, omega, k = 8, 4, 2
    A = tightness_matrix(n, omega, k)
    M = csc_to_dense(A)
    L = oracle.lipschitz(A)
    assert oracle.omega(A) == omega
    h = np.full(n, k ** -0.5)
    Q = M.T @ M
    subs = pins.all_subsets(n, tau)
    mean = np.mean([0.5 * h[S] @ Q[np.ix_(S, S)] @ h[S] for S in subs])
    beta = oracle.beta_nice(omega, tau, n)
    rhs = tau / (2 * n) * beta * float(np.sum(L * h * h))
    assert mean == pytest.approx(rhs, rel=1e-12)
    # random h: the ESO inequality holds
    rng = np.random.default_rng(tau)
    for _ in range(20):
        h = rng.standard_normal(n)
        mean = np.mean([0.5 * h[S] @ Q[np.ix_(S, S)] @ h[S] for S in subs])
        assert mean <= tau / (2 * n) * beta * float(np.sum(L * h * h)) * (1 + 1e-12)


def test_eso_holds_on_random_sparse_quadratics():
    """Theorem 'ESO for nice samplings' for f = 0.5||Ax-b||^2 on random sparse
    A: E[f(x + h_[S])] <= f(x) + (tau/n)(<grad f, h> + beta/2 ||h||_L^2)."""
    rng = np.random.default_rng(3)
    for trial in range(6):
        m, n, d = 7, 9, 3
        A = random_csc(m, n, d, rng)
        M = csc_to_dense(A)
        b = rng.standard_normal(m)
        L = oracle.lipschitz(A)
        om = oracle.omega(A)
        x = rng.standard_normal(n)
        h = rng.standard_normal(n)
        f = lambda z: 0.5 * float((M @ z - b) @ (M @ z - b))
        grad = M.T @ (M @ x - b)
        for tau in range(1, n + 1):
            beta = oracle.beta_nice(om, tau, n)
            lhs = np.mean([f(x + np.bincount(S, weights=h[S], minlength=n))
                           for S in pins.all_subsets(n, tau)])
            rhs = f(x) + tau / n * (grad @ h + 0.5 * beta * float(np.sum(L * h * h)))
            assert lhs <= rhs + 1e-10 * max(1.0, abs(rhs))


# --------------------------------------------------------------------------- #
# structure: omega and L
# --------------------------------------------------------------------------- #

def test_omega_and_lipschitz_hand_built():
    """omega = max nonzeros in a row; L_i = ||a_i||^2 (contributions, item on
    partial separability)."""
    M = np.array([[1.0, 0.0, 2.0, 0.0],
                  [0.0, 3.0, -1.0, 0.5],
                  [4.0, 1.0, 0.0, 0.0]])
    A = dense_to_csc(M)
    assert oracle.omega(A) == 3
    np.testing.assert_array_equal(oracle.lipschitz(A), [17.0, 10.0, 5.0, 0.25])
    # explicit zeros are not counted as nonzeros of a row
    A.values = A.values.copy()
    A.values[A.row_idx == 1] = 0.0
    assert oracle.omega(A) == 2


# --------------------------------------------------------------------------- #
# the update
# --------------------------------------------------------------------------- #

def test_soft_threshold_truth_table():
    """Closed form of the l1 block problem: sign(u) max(|u|-c, 0)."""
    cases = [(3.0, 1.0, 2.0), (-3.0, 1.0, -2.0), (1.0, 1.0, 0.0), (-1.0, 1.0, 0.0),
             (0.5, 1.0, 0.0), (0.0, 0.0, 0.0), (2.5, 0.0, 2.5), (-0.0, 1.0, 0.0)]
    for u, c, want in cases:
        assert oracle.soft(u, c) == want


def test_update_minimises_block_model():
    """Step 4: h^(i)(x) minimises <grad_i f, t> + (beta L_i/2) t^2 + lam|x_i + t|.
    Checked coordinate by coordinate against a kink/stationary-point search."""
    rng = np.random.default_rng(11)
    A = random_csc(12, 10, 4, rng)
    M = csc_to_dense(A)
    b = rng.standard_normal(12)
    lam = 0.3
    for beta in (1.0, 1.7, 4.0):
        s = oracle.Solver(A, b, lam, tau=10, beta=beta, x0=rng.standard_normal(10) * 0.5)
        x0 = s.x.copy()
        r0 = M @ x0 - b
        s.step_with_set(np.arange(10))
        for i in range(10):
            t = pins.coordinate_min_1d(M[:, i], r0, x0[i], lam, beta * float(M[:, i] @ M[:, i]))
            assert s.x[i] - x0[i] == pytest.approx(t, abs=1e-13)


def test_serial_step_is_exact_coordinate_minimisation():
    """tau = 1 gives beta = 1 (serial row of Table ESO), so each step exactly
    minimises F along the sampled coordinate: afterwards that coordinate
    satisfies its own KKT condition (|a_i^T r| <= lam at 0, a_i^T r =
    -lam sign(x_i) otherwise)."""
    rng = np.random.default_rng(5)
    A = random_csc(40, 30, 5, rng)
    inst = planted_lasso(A, 4, 0.01, 0.1, rng)
    s = oracle.Solver(inst.A, inst.b, inst.lam, tau=1, seed=9)
    assert s.beta == 1.0
    M = csc_to_dense(A)
    for _ in range(300):
        i = int(oracle.sample_nice(s.seed, s.k, 1, s.n)[0])
        s.step(1)
        g = float(M[:, i] @ (M @ s.x - inst.b))
        if s.x[i] == 0.0:
            assert abs(g) <= inst.lam * (1 + 1e-12) + 1e-13
        else:
            assert g == pytest.approx(-inst.lam * np.sign(s.x[i]), abs=1e-12)


def test_separable_fully_parallel_step_hits_closed_form():
    """omega = 1 (disjoint row supports) gives beta = 1 at every tau; one fully
    parallel step from 0 solves every coordinate problem exactly:
    x_i = soft(a_i^T b / L_i, lam / L_i)."""
    rng = np.random.default_rng(2)
    A = separable_matrix(25, 3, rng)
    M = csc_to_dense(A)
    b = rng.standard_normal(A.m)
    lam = 0.4
    s = oracle.Solver(A, b, lam, tau=25)
    assert s.omega == 1 and s.beta == 1.0
    s.step(1)
    L = np.sum(M * M, axis=0)
    u = (M.T @ b) / L
    want = np.sign(u) * np.maximum(np.abs(u) - lam / L, 0.0)
    np.testing.assert_allclose(s.x, want, rtol=1e-13, atol=1e-15)
    # and that point is optimal: brute force on a 6-column slice agrees
    Fstar, _ = pins.brute_force_fstar(M[:, :6][:18], b[:18], lam)
    assert pins.lasso_F(M[:18, :6], b[:18], lam, s.x[:6]) == pytest.approx(Fstar, rel=1e-12)


@pytest.mark.parametrize("tau", [1, 3, 16])
def test_orthonormal_columns_converge_to_soft_of_Atb(tau):
    """A^T A = I makes F = 0.5||x - A^T b||^2 + lam||x||_1 + const, whose
    minimiser is soft(A^T b, lam).  Block-Hadamard columns have omega = 4 > 1,
    so beta > 1 for tau > 1."""
    rng = np.random.default_rng(4)
    A = orthonormal_block_hadamard(4, 4, rng)
    M = csc_to_dense(A)
    np.testing.assert_allclose(M.T @ M, np.eye(16), atol=1e-14)
    b = rng.standard_normal(16)
    lam = 0.25
    s = oracle.Solver(A, b, lam, tau=tau, seed=1)
    assert s.omega == 4
    s.step(400 * s.steps_per_epoch())
    want = np.sign(M.T @ b) * np.maximum(np.abs(M.T @ b) - lam, 0)
    np.testing.assert_allclose(s.x, want, atol=1e-10)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_converges_to_brute_force_optimum(seed):
    """F* of tiny instances by enumeration of all 3^n sign patterns; the oracle
    reaches it to 1e-12 relative, for tau-nice beta and several tau."""
    rng = np.random.default_rng(100 + seed)
    m, n = 9, 7
    A = random_csc(m, n, 4, rng)
    inst = planted_lasso(A, 2, 0.05, 0.2, rng)
    M = csc_to_dense(A)
    Fstar, xstar = pins.brute_force_fstar(M, inst.b, inst.lam)
    for tau in (1, 3, 7):
        s = oracle.Solver(inst.A, inst.b, inst.lam, tau=tau, seed=seed)
        s.step(3000 * s.steps_per_epoch())
        assert s.objective() == pytest.approx(Fstar, rel=1e-12)
        np.testing.assert_allclose(s.x, xstar, atol=1e-6)


def test_kkt_and_dual_gap_at_convergence():
    """At convergence |a_i^T r| <= lam off the support, a_i^T r = -lam sign(x_i)
    on it, and the duality gap vanishes; weak duality D <= F holds throughout."""
    rng = np.random.default_rng(7)
    A = random_csc(200, 100, 10, rng)
    inst = planted_lasso(A, 10, 0.01, 0.1, rng)
    s = oracle.Solver(inst.A, inst.b, inst.lam, tau=8, seed=3)
    prev_gap = None
    for _ in range(60):
        gap, F, D = s.gap()
        assert D <= F + 1e-12 * abs(F)
        s.step(20 * s.steps_per_epoch())
        prev_gap = gap
    gap, F, D = s.gap()
    assert gap <= 1e-10 * F
    assert prev_gap is not None
    g = oracle.gradient(inst.A, oracle.residual(inst.A, s.x, inst.b))
    on = s.x != 0
    assert np.all(np.abs(g[~on]) <= inst.lam * (1 + 1e-9))
    np.testing.assert_allclose(g[on], -inst.lam * np.sign(s.x[on]), rtol=1e-8)


def test_maintained_residual_matches_recomputed():
    """The stored r equals a freshly computed A x - b after many steps
    (<= 1e-12 ||b||_inf in float64)."""
    rng = np.random.default_rng(8)
    A = random_csc(300, 500, 12, rng)
    inst = planted_lasso(A, 20, 0.01, 0.05, rng)
    s = oracle.Solver(inst.A, inst.b, inst.lam, tau=37, seed=5)
    s.step(50 * s.steps_per_epoch())
    fresh = oracle.residual(inst.A, s.x, inst.b)
    assert np.max(np.abs(s.r - fresh)) <= 1e-12 * np.max(np.abs(inst.b))


def test_conservative_beta_is_monotone_for_every_set():
    """Theorem on proper uniform samplings: with beta = min(omega, tau) the
    step never increases F, for every set S of size tau (checked over all
    subsets at several points)."""
    rng = np.random.default_rng(9)
    A = random_csc(8, 7, 3, rng)
    M = csc_to_dense(A)
    b = rng.standard_normal(8)
    lam = 0.2
    om = oracle.omega(A)
    for tau in (2, 3, 5, 7):
        for _ in range(5):
            x0 = rng.standard_normal(7)
            F0 = pins.lasso_F(M, b, lam, x0)
            for S in pins.all_subsets(7, tau):
                s = oracle.Solver(A, b, lam, tau=tau, beta=oracle.beta_uniform(om, tau), x0=x0)
                s.step_with_set(S)
                assert pins.lasso_F(M, b, lam, s.x) <= F0 + 1e-12 * abs(F0)


def test_expected_decrease_bound():
    """Eq. (1) of the ESO section: E[F(x + h(x)_[S])] <= (1 - tau/n) F(x) +
    (tau/n) H_{beta,L}(x, h(x)), exact mean over all tau-subsets."""
    rng = np.random.default_rng(10)
    m, n = 8, 7
    A = random_csc(m, n, 3, rng)
    M = csc_to_dense(A)
    b = rng.standard_normal(m)
    lam = 0.15
    om = oracle.omega(A)
    L = np.sum(M * M, axis=0)
    for tau in range(1, n + 1):
        beta = oracle.beta_nice(om, tau, n)
        for _ in range(4):
            x0 = rng.standard_normal(n)
            full = oracle.Solver(A, b, lam, tau=n, beta=beta, x0=x0)
            full.step_with_set(np.arange(n))
            h = full.x - x0
            grad = M.T @ (M @ x0 - b)
            H = (0.5 * float((M @ x0 - b) @ (M @ x0 - b)) + grad @ h
                 + 0.5 * beta * float(np.sum(L * h * h)) + lam * np.abs(x0 + h).sum())
            Fs = []
            for S in pins.all_subsets(n, tau):
                s = oracle.Solver(A, b, lam, tau=tau, beta=beta, x0=x0)
                s.step_with_set(S)
                Fs.append(pins.lasso_F(M, b, lam, s.x))
            F0 = pins.lasso_F(M, b, lam, x0)
            assert np.mean(Fs) <= (1 - tau / n) * F0 + tau / n * H + 1e-12 * abs(F0)


# --------------------------------------------------------------------------- #
# sampler (tau-nice law)
# --------------------------------------------------------------------------- #

def test_sampler_generator_known_answers():
    """SplitMix64 and MurmurHash3 fmix32 reproduce their published outputs."""
    g = _gold("generator_vectors.json")
    for t, hx in enumerate(g["splitmix64_seed0"]["outputs_hex"]):
        assert oracle.splitmix64(0, t) == int(hx, 16)
    for x, hx in zip(g["murmur3_fmix32"]["inputs"], g["murmur3_fmix32"]["outputs_hex"]):
        assert oracle.fmix32(x) == int(hx, 16)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 15, 16, 17, 255, 256, 257, 1000, 4097, 65537])
def test_sampler_is_a_permutation(n):
    """S_k with tau = n is all of [0, n): distinct and in range."""
    for k in (0, 1, 12345):
        s = oracle.sample_nice(42, k, n, n)
        assert np.array_equal(np.sort(s), np.arange(n))


def test_sampler_prefix_and_determinism():
    a = oracle.sample_nice(1, 3, 50, 1000)
    assert np.array_equal(a, oracle.sample_nice(1, 3, 50, 1000))
    assert np.array_equal(a[:20], oracle.sample_nice(1, 3, 20, 1000))
    assert not np.array_equal(a, oracle.sample_nice(1, 4, 50, 1000))
    assert not np.array_equal(a, oracle.sample_nice(2, 3, 50, 1000))


def test_sampler_subset_law_is_uniform():
    """tau-nice: each of the C(n, tau) subsets equally likely (chi-square over
    all 20 subsets of n = 6, tau = 3, 40000 steps)."""
    n, tau, K = 6, 3, 40000
    counts = {}
    for k in range(K):
        key = tuple(sorted(oracle.sample_nice(77, k, tau, n).tolist()))
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == math.comb(n, tau)
    exp = K / math.comb(n, tau)
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    assert chi2 < 45.0  # 19 dof: P(chi2 > 45) ~ 7e-4


def test_sampler_inclusion_and_pair_probabilities():
    """p_i = tau/n (uniform samplings) and p_ij = tau(tau-1)/(n(n-1))
    (doubly uniform samplings with |S| = tau)."""
    n, tau, K = 40, 10, 20000
    inc = np.zeros(n)
    pair = np.zeros((n, n))
    for k in range(K):
        s = oracle.sample_nice(5, k, tau, n)
        inc[s] += 1
        pair[np.ix_(s, s)] += 1
    p = tau / n
    z = (inc / K - p) / math.sqrt(p * (1 - p) / K)
    assert np.max(np.abs(z)) < 4.5
    pij = tau * (tau - 1) / (n * (n - 1))
    off = pair[~np.eye(n, dtype=bool)] / K
    zz = (off - pij) / math.sqrt(pij * (1 - pij) / K)
    assert np.max(np.abs(zz)) < 5.0
    assert abs(off.mean() - pij) < 3 * math.sqrt(pij / (K * n * n))


def test_checkpoint_resume_follows_the_same_trajectory():
    """Fault/resume: the state of a run is (x, k) with the seed; a fresh run
    started from a checkpoint (x_k, k) draws the same S_k, S_k+1, ... and
    ends where the uninterrupted run ends (up to the rounding of r, which the
    resumed run recomputes from x)."""
    inst = make_config("small_2000x1000", dtype="f64")
    full = oracle.Solver(inst.A, inst.b, inst.lam, tau=8, seed=3)
    full.step(300)
    x_mid = full.x.copy()
    full.step(200)
    resumed = oracle.Solver(inst.A, inst.b, inst.lam, tau=8, seed=3, x0=x_mid)
    resumed.k = 300
    resumed.step(200)
    np.testing.assert_allclose(resumed.x, full.x, rtol=0, atol=1e-12)
    assert resumed.objective() == pytest.approx(full.objective(), rel=1e-13)
    # a wrong step counter draws other sets and leaves the trajectory
    wrong = oracle.Solver(inst.A, inst.b, inst.lam, tau=8, seed=3, x0=x_mid)
    wrong.step(200)
    assert np.max(np.abs(wrong.x - full.x)) > 1e-6
