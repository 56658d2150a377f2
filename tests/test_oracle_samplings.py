"""Pins for the oracle's other samplings: tau-independent, (tau, p_b)-binomial,
the drop mask, and the doubly uniform beta (section "Block Samplings";
Table "ESO", doubly uniform and binomial rows; theorem "ESO for doubly uniform
samplings").

What fixes them without trusting the oracle: the paper's printed q_k of the
tau-independent example, the q_k recurrence and the binomial moments it
states, exact enumeration of all pick tuples on tiny domains, the ESO written
as an expectation over that enumeration (equality on the tightness
construction), chi-square tests of the generators' laws, and convergence to
the brute-force optimum.
"""

from __future__ import annotations

import itertools
import json
import math
import os
from collections import Counter
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle
from tests import pins
from workloads import csc_to_dense, planted_lasso, random_csc, tightness_matrix

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")


def _gold(name):
    with open(GOLD) as fh:
        return json.load(fh)[name]


def q_independent(n: int, tau: int):
    """q_k = C(n,k) c_k with c_1 = (1/n)^tau and
    c_k = (k/n)^tau - sum_{i<k} C(k,i) c_i (the paper's definition of the
    tau-independent sampling), in exact rational arithmetic."""
    c = {}
    q = {}
    for k in range(1, tau + 1):
        ck = Fraction(k, n) ** tau - sum(math.comb(k, i) * c[i] for i in range(1, k))
        c[k] = ck
        q[k] = math.comb(n, k) * ck
    return q


def enumerate_independent(n: int, tau: int):
    """Exact law of S for tau-independent picks: every one of the n^tau pick
    tuples is equally likely; S is the set of distinct picks."""
    law = Counter()
    for t in itertools.product(range(n), repeat=tau):
        law[tuple(sorted(set(t)))] += 1
    total = n ** tau
    return {S: Fraction(c, total) for S, c in law.items()}


# --------------------------------------------------------------------------- #
# tau-independent sampling
# --------------------------------------------------------------------------- #

def test_independent_q_printed_values():
    """The printed example n = 1000, tau = 8: q_8 = 0.9723, q_7 = 0.0274,
    q_6 = 0.0003 (four decimals); the oracle's moments equal sum k q_k and
    sum k^2 q_k of that law."""
    g = _gold("independent_sampling_q")
    q = q_independent(g["n"], g["tau"])
    assert sum(q.values()) == 1
    for k, v in g["q"].items():
        assert abs(float(q[int(k)]) - v) <= g["printed_abs_tol"]
    e1, e2 = oracle.independent_moments(g["tau"], g["n"])
    assert e1 == pytest.approx(float(sum(k * v for k, v in q.items())), rel=1e-13)
    assert e2 == pytest.approx(float(sum(k * k * v for k, v in q.items())), rel=1e-13)


@pytest.mark.parametrize("n,tau", [(1, 1), (2, 1), (2, 2), (3, 3), (4, 2), (5, 4), (6, 3), (7, 5)])
def test_independent_law_by_enumeration(n, tau):
    """All n^tau pick tuples: the law of S is doubly uniform (equal mass on sets
    of equal size), its size law is the q_k of the definition, and the
    oracle's moments are its moments."""
    law = enumerate_independent(n, tau)
    by_size = {}
    for S, p in law.items():
        by_size.setdefault(len(S), set()).add(p)
    for k, ps in by_size.items():
        assert len(ps) == 1, "not doubly uniform"
        assert len([S for S in law if len(S) == k]) == math.comb(n, k)
    q = q_independent(n, tau)
    for k in range(1, tau + 1):
        mass = sum(p for S, p in law.items() if len(S) == k)
        assert mass == q[k]
    e1 = float(sum(len(S) * p for S, p in law.items()))
    e2 = float(sum(len(S) ** 2 * p for S, p in law.items()))
    got1, got2 = oracle.independent_moments(tau, n)
    assert got1 == pytest.approx(e1, rel=1e-13)
    assert got2 == pytest.approx(e2, rel=1e-13)


@pytest.mark.parametrize("n,tau", [(10**7, 1), (5 * 10**8, 1), (10**7, 1024), (5 * 10**8, 2**16),
                                   (10**7, 10**6), (10**3, 10**3)])
def test_independent_moments_large_n(n, tau):
    """Where tau << n the pair probability cancels catastrophically in the
    plain form; the moments must still satisfy E|S| <= tau, E|S|^2 >= E|S|^2
    (Jensen) and, to first order, E|S|^2/E|S| - 1 = (tau-1)(1 - O(tau/n)),
    checked against a series in exact rationals."""
    e1, e2 = oracle.independent_moments(tau, n)
    assert e1 <= tau * (1 + 1e-15)
    assert e2 >= e1 * e1 * (1 - 1e-12)
    if tau == 1:
        assert e1 == pytest.approx(1.0, rel=1e-15) and e2 == pytest.approx(1.0, rel=1e-14)
        return
    if tau <= 2**16 and n >= 10**7:
        # exact: 1 - a = sum_{j>=1} (-1)^{j+1} C(tau,j) n^-j, truncated where terms vanish
        def one_minus(p):  # 1 - (1 - p)^tau, p rational, by the binomial series
            s, term = Fraction(0), Fraction(1)
            for j in range(1, 8):
                term = term * (tau - j + 1) / j * p
                s += term if j % 2 else -term
            return s
        a1 = one_minus(Fraction(1, n))
        a2 = one_minus(Fraction(2, n))
        pair = 2 * a1 - a2  # 1 - 2(1-1/n)^tau + (1-2/n)^tau
        E1 = n * a1
        E2 = E1 + n * (n - 1) * pair
        assert e1 == pytest.approx(float(E1), rel=1e-12)
        assert (e2 / e1 - 1) == pytest.approx(float(E2 / E1 - 1), rel=1e-9)


def test_independent_draws_follow_the_law():
    """Raw picks are uniform on [0, n) (chi-square) and |S| follows q_k."""
    n, tau, K = 12, 5, 4000
    picks = np.concatenate([oracle.draw_independent(7, k, tau, n) for k in range(K)])
    assert picks.min() >= 0 and picks.max() < n
    cnt = np.bincount(picks, minlength=n)
    assert stats.chisquare(cnt).pvalue > 1e-4
    sizes = Counter(len(oracle.sample_set("independent", 7, k, tau, n)) for k in range(K))
    q = q_independent(n, tau)
    ks = sorted(q)
    obs = np.array([sizes.get(k, 0) for k in ks], dtype=float)
    exp = np.array([float(q[k]) * K for k in ks])
    keep = exp >= 5
    obs_k = np.append(obs[keep], obs[~keep].sum())
    exp_k = np.append(exp[keep], exp[~keep].sum())
    if exp_k[-1] == 0:
        obs_k, exp_k = obs_k[:-1], exp_k[:-1]
    assert stats.chisquare(obs_k, exp_k * obs_k.sum() / exp_k.sum()).pvalue > 1e-4


def test_independent_set_is_distinct_picks():
    for k in range(20):
        raw = oracle.draw_independent(3, k, 50, 200)
        assert np.array_equal(oracle.sample_set("independent", 3, k, 50, 200), np.unique(raw))


# --------------------------------------------------------------------------- #
# (tau, p_b)-binomial sampling
# --------------------------------------------------------------------------- #

def test_binomial_moments_and_conditional_uniformity():
    """E|S| = tau p_b and E|S|^2 = tau p_b (1 + tau p_b - p_b) (stated with the
    definition); given |S| = k the set is uniform over k-subsets (DU)."""
    n, tau, pb, K = 9, 4, 0.6, 20000
    sets = [tuple(oracle.sample_set("binomial", 11, k, tau, n, pb=pb)) for k in range(K)]
    sz = np.array([len(S) for S in sets], dtype=float)
    e1 = tau * pb
    e2 = tau * pb * (1 + tau * pb - pb)
    var = e2 - e1 * e1
    assert abs(sz.mean() - e1) < 5 * math.sqrt(var / K)
    # size law is Binomial(tau, p_b)
    obs = np.bincount(sz.astype(int), minlength=tau + 1)
    exp = stats.binom.pmf(np.arange(tau + 1), tau, pb) * K
    assert stats.chisquare(obs, exp).pvalue > 1e-4
    # within |S| = 2, all C(9,2) pairs equally likely
    pairs = Counter(S for S in sets if len(S) == 2)
    counts = np.array([pairs.get(c, 0) for c in itertools.combinations(range(n), 2)])
    assert stats.chisquare(counts).pvalue > 1e-4


def test_binomial_slots_are_nice_slots():
    """Available slots keep the tau-nice block of that slot (implicit
    selection); p_b = 1 is the tau-nice sampling."""
    for k in range(10):
        nice = oracle.sample_nice(5, k, 30, 100)
        bino = oracle.draw_binomial(5, k, 30, 100, 0.5)
        keep = bino >= 0
        assert np.array_equal(bino[keep], nice[keep])
        assert 0 < keep.sum() < 30
        assert np.array_equal(oracle.draw_binomial(5, k, 30, 100, 1.0), nice)


# --------------------------------------------------------------------------- #
# drop mask
# --------------------------------------------------------------------------- #

def test_drop_mask_removes_exactly_the_dead_slots():
    n, tau = 300, 40
    mask = np.ones(tau, dtype=np.uint8)
    mask[[0, 7, 39]] = 0
    for k in range(5):
        nice = oracle.sample_nice(2, k, tau, n)
        want = np.sort(nice[mask.astype(bool)])
        assert np.array_equal(oracle.sample_set("nice", 2, k, tau, n, mask=mask), want)
        raw = oracle.draw_independent(2, k, tau, n)
        want = np.unique(raw[mask.astype(bool)])
        assert np.array_equal(oracle.sample_set("independent", 2, k, tau, n, mask=mask), want)
    # a mask shorter than tau leaves the later slots alive; all zeros empties S
    short = np.zeros(5, dtype=np.uint8)
    assert np.array_equal(oracle.sample_set("nice", 2, 0, tau, n, mask=short),
                          np.sort(oracle.sample_nice(2, 0, tau, n)[5:]))
    assert oracle.sample_set("nice", 2, 0, tau, n, mask=np.zeros(tau, np.uint8)).size == 0


# --------------------------------------------------------------------------- #
# doubly uniform beta
# --------------------------------------------------------------------------- #

def test_du_beta_reduces_to_table_rows():
    """With tau-nice moments (tau, tau^2) the doubly uniform beta is the
    tau-nice row; with binomial moments it is the binomial row."""
    for n, om, tau, pb in [(100, 7, 10, 0.3), (677399, 291516, 16, 0.9), (10**7, 200, 10**6, 0.5)]:
        assert oracle.beta_du(om, n, tau, tau * tau) == pytest.approx(oracle.beta_nice(om, tau, n), rel=1e-14)
        e1 = tau * pb
        e2 = tau * pb * (1 + tau * pb - pb)
        assert oracle.beta_du(om, n, e1, e2) == pytest.approx(oracle.beta_binomial(om, tau, n, pb), rel=1e-13)
    assert oracle.beta_for("binomial", 7, 10, 100, 1.0) == oracle.beta_nice(7, 10, 100)


@pytest.mark.parametrize("tau", [1, 2, 3, 4])
def test_independent_eso_tight_on_tightness_matrix(tau):
    """The ESO of a doubly uniform sampling with its beta, as an exact
    expectation over all n^tau pick tuples: equality on the tightness
    construction (h = k^{-1/2} 1), inequality for random h."""
    n, omega, k = 8, 4, 2
    A = tightness_matrix(n, omega, k)
    M = csc_to_dense(A)
    Q = M.T @ M
    L = oracle.lipschitz(A)
    law = enumerate_independent(n, tau)
    e1, e2 = oracle.independent_moments(tau, n)
    beta = oracle.beta_du(omega, n, e1, e2)

    def mean_quad(h):
        return sum(float(p) * 0.5 * h[list(S)] @ Q[np.ix_(S, S)] @ h[list(S)] for S, p in law.items())

    h = np.full(n, k ** -0.5)
    assert mean_quad(h) == pytest.approx(e1 / (2 * n) * beta * float(np.sum(L * h * h)), rel=1e-12)
    rng = np.random.default_rng(tau)
    for _ in range(10):
        h = rng.standard_normal(n)
        assert mean_quad(h) <= e1 / (2 * n) * beta * float(np.sum(L * h * h)) * (1 + 1e-12)


# --------------------------------------------------------------------------- #
# the method with these samplings
# --------------------------------------------------------------------------- #

@pytest.mark.parametrize("sampling,pb", [("independent", 1.0), ("binomial", 0.5)])
def test_converges_to_brute_force_optimum(sampling, pb):
    """PCDM1 with the sampling's ESO beta reaches the brute-force F* (3^n
    sign patterns)."""
    rng = np.random.default_rng(4)
    inst = planted_lasso(random_csc(8, 7, 3, rng), 3, 0.05, 0.2, rng)
    M = csc_to_dense(inst.A)
    Fstar, _ = pins.brute_force_fstar(M, inst.b, inst.lam)
    s = oracle.Solver(inst.A, inst.b, inst.lam, tau=4, seed=1, sampling=sampling, pb=pb)
    s.step(6000)
    assert s.objective() == pytest.approx(Fstar, rel=1e-11, abs=1e-13)


def test_masked_run_equals_steps_on_the_surviving_sets():
    """A run with a drop mask is the run of steps on the sets the mask leaves,
    and still converges (the tau-nice beta over-damps the smaller sets)."""
    rng = np.random.default_rng(6)
    inst = planted_lasso(random_csc(60, 40, 4, rng), 5, 0.01, 0.1, rng)
    mask = np.ones(8, np.uint8)
    mask[[1, 5]] = 0
    a = oracle.Solver(inst.A, inst.b, inst.lam, tau=8, seed=3, mask=mask)
    b = oracle.Solver(inst.A, inst.b, inst.lam, tau=8, seed=3)
    a.step(30)
    for k in range(30):
        b.step_with_set(oracle.sample_set("nice", 3, k, 8, 40, mask=mask))
    assert np.array_equal(a.x, b.x)
    a.step(20000)
    gap, F, _ = a.gap()
    assert gap <= 1e-10 * F


def test_random_sparse_independent_eso_inequality():
    """Expected-decrease form of the ESO for f = 0.5||Ax-b||^2 on a random
    sparse A under the tau-independent law (exact enumeration)."""
    rng = np.random.default_rng(8)
    m, n, d = 6, 5, 2
    A = random_csc(m, n, d, rng)
    M = csc_to_dense(A)
    b = rng.standard_normal(m)
    L = oracle.lipschitz(A)
    om = oracle.omega(A)
    x = rng.standard_normal(n)
    grad = M.T @ (M @ x - b)
    f = lambda z: 0.5 * float((M @ z - b) @ (M @ z - b))
    for tau in range(1, 5):
        law = enumerate_independent(n, tau)
        e1, e2 = oracle.independent_moments(tau, n)
        beta = oracle.beta_du(om, n, e1, e2)
        for _ in range(5):
            h = rng.standard_normal(n)
            lhs = sum(float(p) * f(x + np.bincount(list(S), weights=h[list(S)], minlength=n))
                      for S, p in law.items())
            rhs = f(x) + e1 / n * (grad @ h + 0.5 * beta * float(np.sum(L * h * h)))
            assert lhs <= rhs + 1e-10 * max(1.0, abs(rhs))
