"""The 'theory versus reality' workload (0.5||Ax - b||^2 with omega equal
nonzeros per row, lambda = 0): the library's step count to a 1e-6 relative
objective error equals the oracle's on the same sets (float64 values)."""

import numpy as np
import pytest
import scipy.linalg

import oracle
from workloads import biregular_matrix, csc_to_dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    import torch
    assert torch.cuda.is_available()
    import paper_1212_0873_amd as pc
    pc.load()
    return pc


def _count(stepper, objective, Fstar, F0, chunk, limit=500_000):
    steps = 0
    while steps < limit:
        stepper(chunk)
        steps += chunk
        if objective() - Fstar <= 1e-6 * (F0 - Fstar):
            return steps
    return -1


@pytest.mark.parametrize("omega,tau", [(10, 1), (10, 64), (50, 1000)])
def test_steps_to_eps_match_oracle(pc, omega, tau):
    n, m = 1000, 3000
    A = biregular_matrix(m, n, omega, np.random.default_rng(omega))
    b = np.random.default_rng(1000 + omega).standard_normal(m)
    M = csc_to_dense(A)
    Fstar = 0.5 * float(np.sum((M @ scipy.linalg.lstsq(M, b)[0] - b) ** 2))
    F0 = 0.5 * float(b @ b)
    chunk = max(1, -(-n // (8 * tau)))
    ref = oracle.Solver(A, b, 0.0, tau=tau, seed=0)
    want = _count(ref.step, ref.objective, Fstar, F0, chunk)
    with pc.Problem(A, b, 0.0, tau, seed=0) as p:
        assert p.info()["omega"] == omega and p.info()["beta"] == pytest.approx(ref.beta, rel=1e-15)
        got = _count(p.step, lambda: p.objective()[0], Fstar, F0, chunk)
    print(f"omega {omega} tau {tau}: {got} steps (oracle {want}), theory speedup {tau / ref.beta:.2f}", flush=True)
    assert want > 0 and got == want
