"""Pins for the oracle's one-processor run of the asynchronous variant
(section "Numerical experiments", billion-variable LASSO: cores read the
current iterate when ready and apply updates at once, picking blocks
uniformly and independently).

With one processor the run is serial coordinate descent over the pick
stream, so it is pinned by an independent serial loop whose every update is
the brute-force minimiser of the one-dimensional model, and by convergence to
the brute-force optimum.
"""

import numpy as np
import pytest

import oracle
from tests import pins
from workloads import csc_to_dense, planted_lasso, random_csc

ASYNC_STREAM = 0x5043444D4153594E


def _pick(seed, launch, u, n):
    kappa = oracle.splitmix64(seed ^ ASYNC_STREAM, launch)
    return (oracle.splitmix64(kappa, u) * n) >> 64


@pytest.mark.parametrize("beta", [1.0, 2.5])
def test_serial_run_equals_brute_force_coordinate_steps(beta):
    rng = np.random.default_rng(21)
    A = random_csc(30, 12, 4, rng)
    inst = planted_lasso(A, 4, 0.05, 0.1, rng)
    M = csc_to_dense(inst.A)
    L = (M * M).sum(axis=0)
    s = oracle.Solver(inst.A, inst.b, inst.lam, tau=1, seed=9, beta=beta)
    s.async_serial(launch=3, nupdates=300)
    x = np.zeros(12)
    r = -inst.b.copy()
    picks = [_pick(9, 3, u, 12) for u in range(300)]
    assert sorted(set(picks)) == list(range(12))
    for i in picks:
        t = pins.coordinate_min_1d(M[:, i], r, x[i], inst.lam, beta * L[i])
        x[i] += t
        r += t * M[:, i]
    np.testing.assert_allclose(s.x, x, rtol=0, atol=1e-12)
    np.testing.assert_allclose(s.r, M @ s.x - inst.b, rtol=0, atol=1e-12)


def test_serial_run_reaches_brute_force_optimum():
    rng = np.random.default_rng(5)
    A = random_csc(9, 8, 3, rng)
    inst = planted_lasso(A, 3, 0.05, 0.2, rng)
    Fstar, _ = pins.brute_force_fstar(csc_to_dense(inst.A), inst.b, inst.lam)
    s = oracle.Solver(inst.A, inst.b, inst.lam, tau=1, seed=2)
    for launch in range(40):
        s.async_serial(launch, 200)
    assert s.objective() == pytest.approx(Fstar, rel=1e-12, abs=1e-14)
