"""Float64 oracle for PCDM1 with blocks of several coordinates: the group
LASSO  F(x) = 0.5||A x - b||^2 + lambda * sum_i ||x^(i)||_2  (test
infrastructure; only the test suite, the smoke check and the benchmark's CPU
leg may use it).

What it follows (Richtarik & Takac, "Parallel Coordinate Descent Methods
for Big Data Optimization"):
  * blocks x^(i) of N_i coordinates (section "Block structure, notation and
    assumptions"); here block i is the column range block_ptr[i] ..
    block_ptr[i+1]-1 of A;
  * block norms ||t||_(i) = <B_i t, t>^(1/2) with B_i = I, so the block
    Lipschitz constant of grad_i f (eq. for the block Lipschitz property) is
    L_i = lambda_max(A_i^T A_i), computed with a library symmetric eigen-solver;
  * Omega_i = lambda ||.||_2 (the group-lasso example of block separable
    Omega in the same section);
  * the update h^(i)(x) = argmin <grad_i f, t> + (beta L_i/2)||t||^2 +
    lambda||x^(i) + t|| (eq. h(x) with w = L), whose minimiser is the block
    soft threshold v = max(0, 1 - lambda/(beta L_i ||u||)) u with
    u = x^(i) - grad_i f / (beta L_i);
  * omega = max over rows of the number of blocks with a nonzero in the row
    (partial separability over blocks), beta of the tau-nice row of Table ESO
    with n = number of blocks;
  * every block of S_k is updated from the same x_k, then applied in
    ascending block order (PCDM1, Step 4);
  * duality gap with theta = r * min(1, lambda / max_i ||A_i^T r||).
The sampler is the C oracle's tau-nice sampler over block indices.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import beta_nice, sample_nice


def _csc(A):
    return sp.csc_matrix((A.values_f64(), A.row_idx, A.col_ptr), shape=(A.m, A.n))


def block_lipschitz(A, block_ptr) -> np.ndarray:
    """L_i = largest eigenvalue of A_i^T A_i (dense, float64)."""
    S = _csc(A)
    nb = len(block_ptr) - 1
    L = np.empty(nb)
    for i in range(nb):
        Ai = S[:, block_ptr[i]:block_ptr[i + 1]]
        G = (Ai.T @ Ai).toarray()
        L[i] = float(np.linalg.eigvalsh(G)[-1])
    return L


def block_omega(A, block_ptr) -> int:
    """max over rows of the number of distinct blocks with a nonzero there."""
    S = _csc(A)
    S.eliminate_zeros()
    nb = len(block_ptr) - 1
    col_block = np.repeat(np.arange(nb), np.diff(block_ptr))
    coo = S.tocoo()
    pairs = np.unique(np.stack([coo.row, col_block[coo.col]], axis=1), axis=0)
    return int(np.bincount(pairs[:, 0], minlength=A.m).max()) if pairs.size else 0


def block_soft(u: np.ndarray, t: float) -> np.ndarray:
    """argmin_v 0.5||v - u||^2 + t||v||: max(0, 1 - t/||u||) u."""
    nu = float(np.linalg.norm(u))
    if nu <= t:
        return np.zeros_like(u)
    return (1.0 - t / nu) * u


class GroupSolver:
    """Serial float64 PCDM1 on the group LASSO with the tau-nice sampler over
    blocks (tau blocks per step)."""

    def __init__(self, A, b, lam, block_ptr, tau, seed=0, beta=None):
        self.A = A
        self.S = _csc(A)
        self.m, self.n = A.m, A.n
        self.bp = np.asarray(block_ptr, dtype=np.int64)
        self.nb = len(self.bp) - 1
        self.b = np.asarray(b, dtype=np.float64)
        self.lam = float(lam)
        self.tau = int(tau)
        self.seed = int(seed)
        self.L = block_lipschitz(A, self.bp)
        self.omega = block_omega(A, self.bp)
        self.beta = beta_nice(self.omega, self.tau, self.nb) if beta is None else float(beta)
        self.x = np.zeros(self.n)
        self.r = -self.b.copy()
        self.k = 0
        self.blocks = [self.S[:, self.bp[i]:self.bp[i + 1]] for i in range(self.nb)]

    def step(self, nsteps: int = 1) -> None:
        for _ in range(int(nsteps)):
            S = np.sort(sample_nice(self.seed, self.k, self.tau, self.nb))
            deltas = []
            for i in S:                           # every block from the same r
                Ai = self.blocks[i]
                lo, hi = self.bp[i], self.bp[i + 1]
                g = Ai.T @ self.r
                bl = self.beta * self.L[i]
                v = block_soft(self.x[lo:hi] - g / bl, self.lam / bl)
                deltas.append(v - self.x[lo:hi])
            for i, d in zip(S, deltas):            # apply in ascending block order
                lo, hi = self.bp[i], self.bp[i + 1]
                if np.any(d != 0):
                    self.x[lo:hi] += d
                    self.r += self.blocks[i] @ d
            self.k += 1

    def residual(self) -> np.ndarray:
        return self.S @ self.x - self.b

    def objective(self) -> float:
        r = self.residual()
        norms = [np.linalg.norm(self.x[self.bp[i]:self.bp[i + 1]]) for i in range(self.nb)]
        return 0.5 * float(r @ r) + self.lam * float(np.sum(norms))

    def gap(self):
        r = self.residual()
        g = self.S.T @ r
        gmax = max(np.linalg.norm(g[self.bp[i]:self.bp[i + 1]]) for i in range(self.nb))
        s = min(1.0, self.lam / gmax) if gmax > 0 else 1.0
        F = self.objective()
        D = -0.5 * s * s * float(r @ r) - s * float(self.b @ r)
        return F - D, F, D

    def steps_per_epoch(self) -> int:
        return -(-self.nb // self.tau)
