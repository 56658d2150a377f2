"""The inequality behind the incremental ||A^T r||_inf (CPU, numpy): a
float64 sum of the d products a_ji r_j, formed in any order, moves between
two residuals by at most ||a_i||_1 D with
D = ||r - r_old||_inf + 2 gamma max(||r||_inf, ||r_old||_inf),
gamma = (d + 2) 2^-52 (Hoelder's inequality plus the standard bound on the
rounding of a sum of products).  Checked on spread and concentrated changes
of r, on residuals spanning many binades, and for the lower bound of the new
maximum."""

import numpy as np
import pytest


def _sum(prods, order, rng):
    """float64 sum of the products in a given order: sequential, reversed,
    pairwise (numpy), or a random permutation."""
    if order == "seq":
        s = 0.0
        for p in prods:
            s += p
        return s
    if order == "rev":
        s = 0.0
        for p in prods[::-1]:
            s += p
        return s
    if order == "pairwise":
        return float(np.sum(prods))
    s = 0.0
    for p in prods[rng.permutation(prods.size)]:
        s += p
    return s


def _D(r, ro, d):
    gam = (d + 2) * 2.0 ** -52
    dlt = np.max(np.abs(r - ro)) * (1.0 + 2.0 ** -50)
    rmax = max(np.max(np.abs(r)), np.max(np.abs(ro)))
    return (dlt + 2.0 * gam * rmax) * (1.0 + 2.0 ** -40)


KINDS = ["spread", "concentrated", "wide_range", "tiny_move", "aligned", "cancel_no_move"]


@pytest.mark.parametrize("kind", KINDS)
def test_moved_bound_holds(kind):
    rng = np.random.default_rng(KINDS.index(kind) + 1)
    m, n, d = 400, 300, 20
    rows = np.stack([rng.choice(m, d, replace=False) for _ in range(n)])
    vals = rng.standard_normal((n, d)).astype(np.float32).astype(np.float64)  # stored values
    if kind == "cancel_no_move":
        # products that nearly cancel in every column: the sums are mostly
        # rounding, which the order of summation changes
        ro = rng.standard_normal(m)
        X = 1e3 * rng.standard_normal((n, d // 2))
        c = np.concatenate([X, -X], axis=1)
        vals = (c / ro[rows]).astype(np.float32).astype(np.float64)
    elif kind == "wide_range":
        vals *= 2.0 ** rng.integers(-30, 30, (n, d))
        ro = rng.standard_normal(m) * 2.0 ** rng.integers(-60, 60, m)
    else:
        ro = rng.standard_normal(m)
    r = ro.copy()
    if kind == "spread":
        r += 1e-3 * rng.standard_normal(m)
    elif kind == "concentrated":
        r[rng.choice(m, 3, replace=False)] += 1.0
    elif kind == "wide_range":
        r += ro * 1e-6 * rng.standard_normal(m)
    elif kind == "aligned":
        # Hoelder's equality case for column 0: r moves by delta sign(a_j) on
        # its rows, in the direction that grows |a_0^T r|
        s0 = float(vals[0] @ ro[rows[0]])
        r[rows[0]] += 1e-3 * np.sign(s0) * np.sign(vals[0])
    elif kind == "tiny_move":
        r += 1e-15 * rng.standard_normal(m)
    D = _D(r, ro, d)
    l1 = np.abs(vals).sum(1) * (1.0 + (d + 8) * 2.0 ** -52)
    orders = ["seq", "rev", "pairwise", "perm"]
    s_old = np.array([_sum(vals[i] * ro[rows[i]], orders[i % 4], rng) for i in range(n)])
    s_new = np.array([_sum(vals[i] * r[rows[i]], orders[(i + 1) % 4], rng) for i in range(n)])
    ub = np.abs(s_old) * (1.0 + 2.0 ** -40) + l1 * D
    assert np.all(np.abs(s_new) <= ub)
    lower = (np.max(np.abs(s_old)) - np.max(l1) * D) * (1.0 - 2.0 ** -40) - 2.0 ** -1000
    assert np.max(np.abs(s_new)) >= lower
    if kind == "tiny_move":
        # the bound is not vacuous: most columns are ruled out
        assert np.count_nonzero(ub >= lower) < n // 4


def test_max_norm_form_is_tighter_for_spread_changes():
    """For a change spread over all rows the Hoelder form moves a column with
    d = 20 entries far less than the Cauchy-Schwarz form would."""
    rng = np.random.default_rng(5)
    m, d = 100_000, 20
    a = rng.standard_normal(d)
    dr = 1e-6 * rng.standard_normal(m)
    holder = np.abs(a).sum() * np.max(np.abs(dr))
    cauchy = np.linalg.norm(a) * np.linalg.norm(dr)
    assert holder < cauchy / 10
