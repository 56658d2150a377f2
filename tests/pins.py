"""Independent references used to pin the oracle (tiny dense problems only).

Nothing here calls the oracle's step: these are brute-force enumerations and
closed forms that a wrong oracle would disagree with.
"""

from __future__ import annotations

import itertools

import numpy as np


def lasso_F(M: np.ndarray, b: np.ndarray, lam: float, x: np.ndarray) -> float:
    r = M @ x - b
    return 0.5 * float(r @ r) + lam * float(np.abs(x).sum())


def brute_force_fstar(M: np.ndarray, b: np.ndarray, lam: float):
    """Minimum of 0.5||Mx-b||^2 + lam||x||_1 by enumerating all 3^n sign
    patterns s: on support S solve M_S^T M_S x_S = M_S^T b - lam s_S and keep
    the sign-consistent solutions (the KKT conditions of the LASSO)."""
    m, n = M.shape
    best_F, best_x = lasso_F(M, b, lam, np.zeros(n)), np.zeros(n)
    for s in itertools.product((-1, 0, 1), repeat=n):
        s = np.asarray(s, dtype=float)
        S = np.nonzero(s)[0]
        if S.size == 0:
            continue
        MS = M[:, S]
        G = MS.T @ MS
        if np.linalg.matrix_rank(G) < S.size:
            continue
        xs = np.linalg.solve(G, MS.T @ b - lam * s[S])
        if np.any(np.sign(xs) != s[S]):
            continue
        x = np.zeros(n)
        x[S] = xs
        F = lasso_F(M, b, lam, x)
        if F < best_F:
            best_F, best_x = F, x
    return best_F, best_x


def all_subsets(n: int, tau: int):
    return [np.asarray(c, dtype=np.int64) for c in itertools.combinations(range(n), tau)]


def coordinate_min_1d(a: np.ndarray, r: np.ndarray, x_i: float, lam: float, curvature: float) -> float:
    """argmin_t g t + (curvature/2) t^2 + lam |x_i + t| for g = a^T r, by
    comparing the stationary points of both smooth pieces and the kink."""
    g = float(a @ r)
    cands = [-x_i]  # kink: x_i + t = 0
    for sgn in (-1.0, 1.0):
        t = -(g + lam * sgn) / curvature
        if sgn * (x_i + t) > 0:
            cands.append(t)
    vals = [g * t + 0.5 * curvature * t * t + lam * abs(x_i + t) for t in cands]
    return float(cands[int(np.argmin(vals))])
