"""||A^T r||_inf of the duality gap and of ||A^T b||_inf on the HIP path.

For float32 and bf16 values the library takes two passes: a bound pass over
fl32(r) that gives every column a rigorous interval, then the exact float64
sums of the columns whose upper bound reaches the largest lower bound.  The
exact sums are those of the single pass, so both routes must return the same
number bit for bit ("max_passes" 1 vs 2), also where columns tie exactly or
to a few ulps, where r spans the whole float32 range (subnormals included),
and where r leaves it.  The result is also checked against the oracle's
sums and against dense float64 arithmetic on the host.
"""

import numpy as np
import pytest

import oracle
from workloads import CSC, csc_to_dense, make_config, random_csc, random_csc_ragged

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    import torch
    assert torch.cuda.is_available()
    import paper_1212_0873_amd as pc
    pc.load()
    return pc


def _routes(pc, A, b, lam, x):
    """(||A^T b||_inf, F, gap) with one and with two passes."""
    out = {}
    for passes in (1, 2):
        with pc.Problem(A, b, lam, 4, seed=0) as p:
            p.set_option("max_passes", passes)
            p.set_rhs(b)  # ||A^T b||_inf again, by this route
            atb = p.info()["atb_inf"]
            p.set_x(x, k=0)
            F, gap = p.objective(gap=True)
        out[passes] = (atb, F, gap)
    return out


def _check(pc, A, b, lam, x):
    out = _routes(pc, A, b, lam, x)
    assert out[1] == out[2], out
    atb = np.max(np.abs(oracle.gradient(A, -np.asarray(b, np.float64))))
    assert out[2][0] == pytest.approx(atb, rel=1e-13)
    return out


def _disjoint_support(A: CSC, want: int, rng) -> np.ndarray:
    """Up to `want` columns sharing no row, so that r = A x - b gets at most one
    term per row: the float64 residual is then the same bits however the
    refresh's atomic adds are ordered, and the two routes see the same r."""
    used = np.zeros(A.m, dtype=bool)
    cols = []
    for j in rng.permutation(A.n):
        rows = A.row_idx[A.col_ptr[j]:A.col_ptr[j + 1]]
        if not used[rows].any():
            used[rows] = True
            cols.append(j)
            if len(cols) == want:
                break
    return np.array(cols, dtype=np.int64)


def _pairs(A: CSC, scale: float, dtype: str) -> CSC:
    """Each column followed by a copy whose values are multiplied by `scale`
    (rounded to the storage type): exact ties for scale 1, near-ties else."""
    v = A.values_f64()
    cols, rows, vals = [0], [], []
    for j in range(A.n):
        s, e = A.col_ptr[j], A.col_ptr[j + 1]
        for sc in (1.0, scale):
            rows.append(A.row_idx[s:e])
            vals.append(v[s:e] * sc)
            cols.append(cols[-1] + (e - s))
    B = CSC(A.m, 2 * A.n, np.array(cols, np.int64), np.concatenate(rows).astype(np.int32),
            np.concatenate(vals))
    return B.astype(dtype)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_two_passes_equal_one_on_random_points(pc, dtype):
    rng = np.random.default_rng(1)
    for trial in range(4):
        A = random_csc_ragged(900, 700, 1, 40, rng).astype(dtype)
        b = rng.standard_normal(900) * 10.0 ** rng.integers(-3, 4)
        x = np.zeros(700)
        sup = _disjoint_support(A, 200, rng)
        x[sup] = rng.standard_normal(sup.size).astype(np.float32)
        _check(pc, A, b, 0.5, x)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("scale", [1.0, 1.0 + 2.0 ** -22, 1.0 - 2.0 ** -20, -1.0])
def test_ties_and_near_ties(pc, dtype, scale):
    rng = np.random.default_rng(2)
    A = _pairs(random_csc(500, 300, 6, rng), scale, dtype)
    b = rng.standard_normal(500)
    x = np.zeros(A.n)
    _check(pc, A, b, 0.3, x)
    x[_disjoint_support(A, 50, rng)] = 0.25
    _check(pc, A, b, 0.3, x)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_residual_across_the_float32_range(pc, dtype):
    """r = -b with entries from 1e-44 (float32 subnormals) to 1e30, zeros, and
    entries whose float32 rounding is inexact by a full half-ulp."""
    rng = np.random.default_rng(3)
    A = random_csc(400, 300, 8, rng).astype(dtype)
    exps = rng.uniform(-44, 30, 400)
    b = np.sign(rng.standard_normal(400)) * 10.0 ** exps
    b[::17] = 0.0
    b[1::23] = (1.0 + 2.0 ** -24) * 2.0 ** rng.integers(-100, 100, b[1::23].size)
    _check(pc, A, b, 1e-3, np.zeros(300))


def test_residual_beyond_float32(pc):
    """Entries of r beyond the float32 range make every column touching them a
    candidate: the exact pass decides."""
    rng = np.random.default_rng(4)
    A = random_csc(300, 200, 5, rng).astype("f32")
    b = rng.standard_normal(300)
    b[[3, 77, 150]] = [1e39, -3e40, 5e38]
    out = _check(pc, A, b, 1.0, np.zeros(200))
    M = csc_to_dense(A)
    assert out[2][0] == pytest.approx(np.max(np.abs(M.T @ b)), rel=1e-12)


def test_float64_values_take_one_pass(pc):
    rng = np.random.default_rng(5)
    A = random_csc_ragged(300, 200, 2, 12, rng)
    b = rng.standard_normal(300)
    out = _check(pc, A, b, 0.2, np.zeros(200))
    assert out[1][0] > 0


def test_max_passes_option_checked(pc):
    from paper_1212_0873_amd import PCDMError
    rng = np.random.default_rng(6)
    A = random_csc(50, 40, 3, rng).astype("f32")
    with pc.Problem(A, rng.standard_normal(50), 0.1, 2) as p:
        for bad in (-1, 4, 1.5):
            with pytest.raises(PCDMError):
                p.set_option("max_passes", bad)


def _sequence(pc, A, b, lam, xs, passes):
    """(||A^T b||, F, gap) at each point of xs, evaluated in order on one
    handle with the given route."""
    out, cands = [], []
    with pc.Problem(A, b, lam, 4, seed=0) as p:
        p.set_option("max_passes", passes)
        p.set_rhs(b)
        for x in xs:
            p.set_x(x, k=0)
            out.append(p.objective(gap=True))
            cands.append(p.info()["max_candidates"])
        hits = p.info()["max_incremental"]
    return out, hits, cands


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_incremental_route_equals_single_pass_along_a_sequence(pc, dtype):
    """Route 3 keeps r and per-column bounds from the last evaluation and sums
    exactly only the columns whose moved bound can still reach the maximum.
    Along a sequence of nearby points (small and large moves, a move back,
    no move) it returns the single pass's numbers bit for bit.  The points
    are supported on columns sharing no row, so the float64 residual is the
    same bits on every handle."""
    rng = np.random.default_rng(11)
    A = random_csc(1500, 1200, 6, rng).astype(dtype)
    b = rng.standard_normal(1500)
    sup = _disjoint_support(A, 150, rng)
    x0 = np.zeros(1200)
    x0[sup] = rng.standard_normal(sup.size)
    xs = [x0]
    for scale in (1e-6, 1e-3, 1e-6, 0.0, 1.0, 1e-9):
        x = xs[-1].copy()
        x[sup] += scale * rng.standard_normal(sup.size)
        xs.append(x.astype(np.float32).astype(np.float64))
    xs.append(xs[0])
    one, hits1, _ = _sequence(pc, A, b, 0.2, xs, 1)
    inc, hits3, cands = _sequence(pc, A, b, 0.2, xs, 3)
    assert inc == one
    assert hits1 == 0
    # set_rhs's ||A^T b|| leaves the state the first point moves from (a large
    # move: every column a candidate); the small moves and the unmoved point
    # are decided from the moved bounds with few exact sums
    assert hits3 >= 4 and max(cands[1], cands[2], cands[3], cands[4]) <= 1200 // 8, cands


def test_incremental_route_after_steps(pc):
    """Route 3 along a solve (steps between evaluations): the same objective
    and gap as the single pass evaluated right after it at the same point, to
    the refresh's rounding."""
    inst = make_config("small_2000x1000", dtype="f32")
    cands = []
    with pc.Problem(inst.A, inst.b, inst.lam, 64, seed=1) as p:
        for _ in range(12):
            p.step(16 * 5)
            p.set_option("max_passes", 3)
            F3, g3 = p.objective(gap=True)
            p.set_option("max_passes", 1)
            F1, g1 = p.objective(gap=True)
            cands.append(p.info()["max_candidates"])
            # each evaluation refreshes the float64 residual with atomic adds,
            # so the two see it to rounding only
            assert F3 == pytest.approx(F1, rel=1e-13)
            assert g3 == pytest.approx(g1, rel=1e-9, abs=1e-13 * abs(F1))
        hits = p.info()["max_incremental"]
    assert hits >= 1, cands
