"""HIP path vs the float64 oracle, through the C ABI, on the same seeded inputs.

Tolerances (relative on F(x_k) unless stated):
  * float64 kernels: 1e-10 (rounding order of sums and atomics only);
  * float32 / bf16 kernels: 1e-5 against the oracle run on the same stored
    (rounded) values, at every logged epoch.
"""

import numpy as np
import pytest

import oracle
from workloads import (CSC, csc_to_dense, make_config, orthonormal_block_hadamard, planted_lasso,
                       random_csc, random_csc_ragged, separable_matrix)

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


def _dense_residual(A, x, b):
    M = csc_to_dense(A)
    return M @ x - b


def _sparse(A):
    import scipy.sparse as sp
    return sp.csc_matrix((A.values_f64(), A.row_idx, A.col_ptr), shape=(A.m, A.n))


# --------------------------------------------------------------------------- #
# sampler
# --------------------------------------------------------------------------- #

@pytest.mark.parametrize("seed,k,tau,n", [
    (0, 0, 1, 1), (0, 5, 2, 2), (3, 1, 3, 5), (9, 2, 17, 17), (1, 7, 8, 1000), (2, 3, 1000, 1000),
    (5, 11, 4000, 4097), (7, 0, 65537, 65537), (11, 123456789, 1_000_000, 10_000_000),
    (13, 2, 1000, 2**31 - 2),
])
def test_sampler_bit_exact(pc, seed, k, tau, n):
    _say(f"sampler seed={seed} k={k} tau={tau} n={n}")
    got = pc.sample(seed, k, tau, n).cpu().numpy().astype(np.int64)
    want = oracle.sample_nice(seed, k, tau, n)
    assert np.array_equal(got, want)


# --------------------------------------------------------------------------- #
# trajectories on the small configuration
# --------------------------------------------------------------------------- #

def _compare_run(pc, A, b, lam, tau, seed, epochs, log_every, rtol_F, x_atol=None):
    ref = oracle.Solver(A, b, lam, tau=tau, seed=seed)
    spe = ref.steps_per_epoch()
    with pc.Problem(A, b, lam, tau, seed=seed) as p:
        info = p.info()
        assert info["omega"] == ref.omega
        assert info["beta"] == pytest.approx(ref.beta, rel=1e-15)
        worst = 0.0
        for e in range(0, epochs, log_every):
            p.step(log_every * spe)
            ref.step(log_every * spe)
            F, _ = p.objective()
            Fr = ref.objective()
            worst = max(worst, abs(F - Fr) / abs(Fr))
            assert abs(F - Fr) <= rtol_F * abs(Fr), (e + log_every, F, Fr)
        if x_atol is not None:
            np.testing.assert_allclose(p.get_x(), ref.x, rtol=0, atol=x_atol)
        return worst, ref, p.info()


@pytest.mark.parametrize("tau", [1, 8])
def test_small_config_float64_matches_oracle(pc, tau):
    inst = make_config("small_2000x1000", dtype="f64")
    _say(f"small f64 tau={tau}")
    worst, ref, info = _compare_run(pc, inst.A, inst.b, inst.lam, tau, 0, 200, 20, 1e-10, x_atol=1e-9)
    _say(f"  worst rel F diff {worst:.2e}, oracle changed {ref.changed}, gpu nonzero {info['nonzero_updates']}")
    # The count of nonzero updates is reported, not compared: near convergence
    # delta_i sits at rounding level and whether it is exactly zero depends on
    # the summation order.


@pytest.mark.parametrize("tau", [1, 8])
def test_small_config_float32_matches_oracle(pc, tau):
    inst = make_config("small_2000x1000", dtype="f32")
    _say(f"small f32 tau={tau}")
    worst, _, _ = _compare_run(pc, inst.A, inst.b, inst.lam, tau, 0, 200, 10, 1e-5)
    _say(f"  worst rel F diff {worst:.2e}")


def test_small_config_bf16_matches_oracle(pc):
    inst = make_config("small_2000x1000", dtype="bf16")
    _say("small bf16 tau=8")
    worst, _, _ = _compare_run(pc, inst.A, inst.b, inst.lam, 8, 0, 200, 10, 1e-5)
    _say(f"  worst rel F diff {worst:.2e}")


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16, 32, 64])
def test_every_lane_schedule_matches_oracle(pc, lanes):
    """Ragged degrees 1..37 (not multiples of 4), unsorted rows, tau not dividing n."""
    rng = np.random.default_rng(lanes)
    A = random_csc_ragged(500, 777, 1, 37, rng)
    inst = planted_lasso(A, 30, 0.01, 0.05, rng)
    ref = oracle.Solver(inst.A, inst.b, inst.lam, tau=100, seed=4)
    with pc.Problem(inst.A, inst.b, inst.lam, 100, seed=4) as p:
        p.set_option("lanes_per_column", lanes)
        assert p.info()["lanes_per_column"] == lanes
        for _ in range(5):
            p.step(16)
            ref.step(16)
            F, _ = p.objective()
            assert F == pytest.approx(ref.objective(), rel=1e-10)
        np.testing.assert_allclose(p.get_x(), ref.x, rtol=0, atol=1e-9)


@pytest.mark.parametrize("d,dtype", [(1, "f64"), (3, "f32"), (10, "bf16"), (10, "f64")])
def test_fixed_degree_with_padding(pc, d, dtype):
    """Equal column lengths (the fixed-stride record layout) that are not a
    multiple of 4, so every record carries padding entries."""
    rng = np.random.default_rng(d)
    A = random_csc(400, 600, d, rng, normalize=False, dtype=dtype)
    inst = planted_lasso(A, 15, 0.01, 0.1, rng)
    rtol = 1e-10 if dtype == "f64" else 1e-5
    worst, _, info = _compare_run(pc, inst.A, inst.b, inst.lam, 50, 6, 20, 5, rtol)
    assert info["stored_nnz"] == 600 * (-(-d // 4) * 4)
    _say(f"d={d} {dtype} worst {worst:.2e}")


@pytest.mark.parametrize("tau", [1, 2, 777])
def test_extreme_tau_float64(pc, tau):
    rng = np.random.default_rng(tau)
    A = random_csc_ragged(300, 777, 2, 9, rng)
    inst = planted_lasso(A, 20, 0.01, 0.1, rng)
    worst, _, _ = _compare_run(pc, inst.A, inst.b, inst.lam, tau, 3, 20, 5, 1e-10, x_atol=1e-9)
    _say(f"tau={tau} worst {worst:.2e}")


def test_single_column_problem(pc):
    A = CSC(3, 1, np.array([0, 2], dtype=np.int64), np.array([0, 2], dtype=np.int32), np.array([1.0, -2.0]))
    b = np.array([1.0, 5.0, -3.0])
    lam = 0.5
    with pc.Problem(A, b, lam, 1, seed=0) as p:
        assert p.info()["beta"] == 1.0
        p.step(1)
        x = p.get_x()
    u = (1.0 * 1.0 + -2.0 * -3.0) / 5.0
    assert x[0] == pytest.approx(np.sign(u) * max(abs(u) - lam / 5.0, 0), rel=1e-15)


# --------------------------------------------------------------------------- #
# closed forms and invariants (properties, no oracle input from the GPU)
# --------------------------------------------------------------------------- #

@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_separable_one_parallel_step_is_exact(pc, dtype):
    rng = np.random.default_rng(21)
    A = separable_matrix(2000, 4, rng).astype(dtype)
    b = rng.standard_normal(A.m)
    lam = 0.3
    with pc.Problem(A, b, lam, A.n, seed=2) as p:
        assert p.info()["omega"] == 1 and p.info()["beta"] == 1.0
        p.step(1)
        x = p.get_x()
    v = A.values_f64().reshape(A.n, 4)
    L = (v * v).sum(1)
    u = (v * b.reshape(A.n, 4)).sum(1) / L
    want = np.sign(u) * np.maximum(np.abs(u) - lam / L, 0)
    tol = 1e-13 if dtype == "f64" else 2e-6
    np.testing.assert_allclose(x, want, rtol=tol, atol=tol)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 2e-5)])
def test_orthonormal_columns_converge_to_closed_form(pc, dtype, tol):
    rng = np.random.default_rng(3)
    A = orthonormal_block_hadamard(16, 8, rng).astype(dtype)
    M = csc_to_dense(A)
    b = rng.standard_normal(A.m)
    lam = 0.2
    with pc.Problem(A, b, lam, 32, seed=5) as p:
        assert p.info()["omega"] == 8
        p.step(400 * 4)
        x = p.get_x()
    want = np.sign(M.T @ b) * np.maximum(np.abs(M.T @ b) - lam, 0)
    np.testing.assert_allclose(x, want, atol=tol)


def test_residual_invariant_float32(pc):
    """Stored r vs A x - b computed independently (scipy): drift within an
    epoch is small, and the float64 refresh at the epoch end removes it."""
    inst = make_config("lasso_1e6x1e7", scale=0.01, dtype="f32", tau=1000)
    S = _sparse(inst.A)
    with pc.Problem(inst.A, inst.b, inst.lam, 1000, seed=1) as p:
        spe = p.info()["refresh_every"]
        p.step(spe - 1)
        r = p.get_residual()
        fresh = S @ p.get_x() - inst.b
        drift = np.max(np.abs(r - fresh)) / np.max(np.abs(inst.b))
        p.step(1)  # epoch end: refresh
        r = p.get_residual()
        fresh = S @ p.get_x() - inst.b
        after = np.max(np.abs(r - fresh)) / np.max(np.abs(inst.b))
    _say(f"drift before refresh {drift:.2e}, after {after:.2e}")
    assert drift <= 1e-5
    assert after <= 1e-7


def test_kkt_and_gap_at_convergence_float64(pc):
    rng = np.random.default_rng(8)
    A = random_csc(600, 400, 12, rng)
    inst = planted_lasso(A, 20, 0.01, 0.1, rng)
    S = _sparse(inst.A)
    with pc.Problem(inst.A, inst.b, inst.lam, 16, seed=7) as p:
        p.step(25 * 300)
        F, gap = p.objective(gap=True)
        x = p.get_x()
    g = S.T @ (S @ x - inst.b)
    on = x != 0
    assert gap <= 1e-9 * F
    assert np.all(np.abs(g[~on]) <= inst.lam * (1 + 1e-8))
    np.testing.assert_allclose(g[on], -inst.lam * np.sign(x[on]), rtol=1e-7)


def test_objective_and_gap_at_given_point_match_oracle(pc):
    rng = np.random.default_rng(9)
    for dtype in ("f64", "f32", "bf16"):
        A = random_csc_ragged(700, 500, 3, 15, rng).astype(dtype)
        b = rng.standard_normal(700)
        lam = 0.7
        x = np.where(rng.random(500) < 0.2, rng.standard_normal(500), 0.0)
        if dtype != "f64":
            x = x.astype(np.float32).astype(np.float64)
        with pc.Problem(A, b, lam, 10, seed=0) as p:
            p.set_x(x, k=0)
            F, gap = p.objective(gap=True)
            info = p.info()
        gap_r, F_r, _ = oracle.dual_gap(A, b, x, lam)
        assert F == pytest.approx(F_r, rel=1e-12)
        assert gap == pytest.approx(gap_r, rel=1e-10)
        assert info["atb_inf"] == pytest.approx(np.max(np.abs(oracle.gradient(A, -b))), rel=1e-12)


def test_set_x_resumes_the_same_trajectory(pc):
    inst = make_config("small_2000x1000", dtype="f64")
    with pc.Problem(inst.A, inst.b, inst.lam, 8, seed=3) as p:
        p.step(300)
        x_mid = p.get_x()
        p.step(200)
        x_end = p.get_x()
    with pc.Problem(inst.A, inst.b, inst.lam, 8, seed=3) as q:
        q.set_x(x_mid, k=300)
        assert q.info()["k"] == 300
        q.step(200)
        np.testing.assert_allclose(q.get_x(), x_end, atol=1e-11)


def test_uniform_beta_rule_is_monotone(pc):
    """beta = min(omega, tau): F never increases (float64 kernels)."""
    rng = np.random.default_rng(12)
    A = random_csc(300, 200, 8, rng)
    inst = planted_lasso(A, 10, 0.01, 0.05, rng)
    with pc.Problem(inst.A, inst.b, inst.lam, 40, seed=2) as p:
        p.set_option("beta_rule", 1)
        assert p.info()["beta"] == min(p.info()["omega"], 40)
        prev, _ = p.objective()
        for _ in range(100):
            p.step(1)
            F, _ = p.objective()
            assert F <= prev * (1 + 1e-14)
            prev = F


# --------------------------------------------------------------------------- #
# validation
# --------------------------------------------------------------------------- #

def _bad(kind):
    cp = np.array([0, 2, 4, 6], dtype=np.int64)
    ri = np.array([0, 1, 1, 2, 0, 2], dtype=np.int32)
    v = np.array([1.0, 2.0, -1.0, 0.5, 3.0, 1.0])
    if kind == "empty":
        cp = np.array([0, 2, 2, 6], dtype=np.int64)
    elif kind == "dup":
        ri = np.array([0, 1, 1, 1, 0, 2], dtype=np.int32)
    elif kind == "row":
        ri = np.array([0, 1, 1, 3, 0, 2], dtype=np.int32)
    elif kind == "nan":
        v = v.copy()
        v[3] = np.nan
    elif kind == "zerocol":
        v = v.copy()
        v[2:4] = 0.0
    elif kind == "ptr":
        cp = np.array([0, 3, 2, 6], dtype=np.int64)
    elif kind == "ptr_end":
        cp = np.array([0, 2, 4, 5], dtype=np.int64)
    return CSC(3, 3, cp, ri, v)


@pytest.mark.parametrize("kind", ["empty", "dup", "row", "nan", "zerocol", "ptr", "ptr_end"])
def test_invalid_matrix_rejected(pc, kind):
    with pytest.raises(pc.PCDMError) as e:
        pc.Problem(_bad(kind), np.ones(3), 0.1, 1)
    assert e.value.status == -1


def test_valid_tiny_matrix_accepted(pc):
    with pc.Problem(_bad("none"), np.ones(3), 0.1, 3) as p:
        assert p.info()["omega"] == 2


# --------------------------------------------------------------------------- #
# full-size single instance (the benchmark's launch configuration)
# --------------------------------------------------------------------------- #

@pytest.fixture(scope="module")
def c2_full():
    _say("generating 1e6 x 1e7 instance (2e8 nnz)")
    return make_config("lasso_1e6x1e7", dtype="f32", tau=1_000_000)


def test_full_size_exact_max_routes_agree(pc, c2_full):
    """1e6 x 1e7: ||A^T b||_inf and the gap at x = 0 (r = -b exactly, no
    atomics) are the same numbers by the default and the single-pass route;
    after steps the three routes agree to the float64 refresh's rounding."""
    inst = c2_full
    with pc.Problem(inst.A, inst.b, inst.lam, 1_000_000, seed=0) as p:
        atb2 = p.info()["atb_inf"]  # at create: no kept state, two passes
        F2, g2 = p.objective(gap=True)
        p.set_option("max_passes", 1)
        p.set_rhs(inst.b)
        atb1 = p.info()["atb_inf"]
        F1, g1 = p.objective(gap=True)
        assert (atb1, F1, g1) == (atb2, F2, g2)
        p.step(30)
        F1, g1 = p.objective(gap=True)
        for passes in (2, 3, 3):
            # the second route-3 evaluation moves from the first one's state
            p.set_option("max_passes", passes)
            F2, g2 = p.objective(gap=True)
            assert F2 == pytest.approx(F1, rel=1e-13)
            assert g2 == pytest.approx(g1, rel=1e-10)
        assert p.info()["max_incremental"] >= 1


def test_full_size_steps_match_oracle(pc, c2_full):
    """Three steps of tau = 1e6 on the 1e6 x 1e7 (2e8 nnz) instance: every x_i
    and F against the oracle on the same float32-stored matrix."""
    inst = c2_full
    tau = 1_000_000
    ref = oracle.Solver(inst.A, inst.b, inst.lam, tau=tau, seed=0)
    with pc.Problem(inst.A, inst.b, inst.lam, tau, seed=0) as p:
        info = p.info()
        _say(f"omega {info['omega']} beta {info['beta']:.4f} lanes {info['lanes_per_column']}")
        assert info["omega"] == ref.omega
        # step 0 starts at x = 0: coordinate i changes iff |g_i| > lambda with
        # g_i = a_i^T r = -a_i^T b.  The device sums d float32 products of
        # fl32(-b), within (d + 3) 2^-24 sum_j |a_ji||b_j| of g_i; only
        # coordinates with |g_i| that close to lambda may count differently.
        S0 = oracle.sample_nice(0, 0, tau, inst.A.n).astype(np.int64)
        d = int(inst.A.col_ptr[1] - inst.A.col_ptr[0])
        assert np.all(np.diff(inst.A.col_ptr) == d)
        idx = inst.A.col_ptr[S0][:, None] + np.arange(d)
        av = inst.A.values_f64()[idx]
        bv = inst.b[inst.A.row_idx[idx]]
        g0 = -(av * bv).sum(axis=1)
        bound = (d + 3) * 2.0 ** -24 * (np.abs(av) * np.abs(bv)).sum(axis=1)
        edge = int(np.count_nonzero(np.abs(np.abs(g0) - inst.lam) <= bound))
        for s in range(3):
            p.step(1)
            ref.step(1)
            if s == 0:
                got = p.info()["nonzero_updates"]
                _say(f"step 1: nonzero updates gpu {got} oracle {ref.changed} ({edge} at the threshold)")
                assert ref.changed == int(np.count_nonzero(np.abs(g0) > inst.lam)) or edge > 0
                assert abs(got - ref.changed) <= edge
            F, _ = p.objective()
            Fr = ref.objective()
            _say(f"step {s + 1}: F {F:.9e} oracle {Fr:.9e}")
            assert abs(F - Fr) <= 1e-5 * abs(Fr)
        x = p.get_x()
        scale = np.max(np.abs(ref.x))
        assert np.max(np.abs(x - ref.x)) <= 1e-5 * scale
        assert np.array_equal(x != 0, ref.x != 0) or np.mean((x != 0) != (ref.x != 0)) < 1e-5
        _say(f"nonzero updates after 3 steps: gpu {p.info()['nonzero_updates']} oracle {ref.changed}")


@pytest.mark.parametrize("tau,steps", [(65536, 24), (1024, 400)])
def test_full_size_small_tau_matches_oracle(pc, c2_full, tau, steps):
    """The instance's other two tau (the lane-group layout): F after every
    quarter of the run and every x_i at the end against the oracle on the
    same float32-stored matrix, with the same beta."""
    inst = c2_full
    ref = oracle.Solver(inst.A, inst.b, inst.lam, tau=tau, seed=1)
    with pc.Problem(inst.A, inst.b, inst.lam, tau, seed=1) as p:
        info = p.info()
        assert info["beta"] == pytest.approx(ref.beta, rel=1e-15)
        for q in range(4):
            p.step(steps // 4)
            ref.step(steps // 4)
            F, _ = p.objective()
            Fr = ref.objective()
            _say(f"tau {tau} after {(q + 1) * steps // 4} steps: F {F:.9e} oracle {Fr:.9e}")
            assert abs(F - Fr) <= 1e-5 * abs(Fr)
        x = p.get_x()
        assert np.max(np.abs(x - ref.x)) <= 1e-5 * np.max(np.abs(ref.x))


# --------------------------------------------------------------------------- #
# the two step-kernel layouts (64-slot tiles, a lane group per slot)
# --------------------------------------------------------------------------- #

@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16, 32, 64])
def test_narrow_and_tiled_layouts_agree(pc, lanes):
    """The first step from x = 0 reads r = -b only, so both layouts must give
    the same x bit for bit (same summation order per column); over further
    steps each stays within 1e-10 of the oracle.  tau = 300 leaves a ragged
    last tile / wave."""
    rng = np.random.default_rng(40 + lanes)
    A = random_csc_ragged(700, 1100, 1, 41, rng)
    inst = planted_lasso(A, 30, 0.01, 0.05, rng)
    xs = {}
    for name, nb in (("tiles", 0), ("narrow", 10**12)):
        ref = oracle.Solver(inst.A, inst.b, inst.lam, tau=300, seed=8)
        with pc.Problem(inst.A, inst.b, inst.lam, 300, seed=8) as p:
            p.set_option("lanes_per_column", lanes)
            p.set_option("narrow_below", nb)
            assert p.info()["narrow_below"] == (0 if nb == 0 else nb)
            p.step(1)
            xs[name] = p.get_x()
            ref.step(1)
            np.testing.assert_allclose(xs[name], ref.x, rtol=0, atol=1e-12)
            for _ in range(4):
                p.step(7)
                ref.step(7)
                F, _ = p.objective()
                assert F == pytest.approx(ref.objective(), rel=1e-10)
            np.testing.assert_allclose(p.get_x(), ref.x, rtol=0, atol=1e-9)
    assert np.array_equal(xs["tiles"], xs["narrow"])


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_narrow_layout_large_tau(pc, dtype):
    """The lane-group layout forced at tau = 4000 (many waves, grid-stride
    loop) on float32 / bf16 values, against the oracle."""
    rng = np.random.default_rng(77)
    A = random_csc(3000, 5000, 12, rng, dtype=dtype)
    inst = planted_lasso(A, 50, 0.01, 0.05, rng)
    ref = oracle.Solver(inst.A, inst.b, inst.lam, tau=4000, seed=1)
    with pc.Problem(inst.A, inst.b, inst.lam, 4000, seed=1) as p:
        p.set_option("narrow_below", 10**12)
        for _ in range(5):
            p.step(6)
            ref.step(6)
            F, _ = p.objective()
            assert F == pytest.approx(ref.objective(), rel=1e-5)


# --------------------------------------------------------------------------- #
# runs of steps replayed from a captured graph
# --------------------------------------------------------------------------- #

@pytest.mark.parametrize("graph_steps", [0, 5, 32])
def test_graph_replays_match_oracle(pc, graph_steps):
    """Calls of odd lengths with a refresh every 25 steps, so runs are split
    between graph replays and direct launches."""
    inst = make_config("small_2000x1000", dtype="f64")
    ref = oracle.Solver(inst.A, inst.b, inst.lam, tau=8, seed=0)
    with pc.Problem(inst.A, inst.b, inst.lam, 8, seed=0) as p:
        p.set_option("graph_steps", graph_steps)
        p.set_option("refresh_every", 25)
        for n in (37, 64, 5, 101, 32, 77):
            p.step(n)
            ref.step(n)
            F, _ = p.objective()
            assert F == pytest.approx(ref.objective(), rel=1e-10)
        np.testing.assert_allclose(p.get_x(), ref.x, rtol=0, atol=1e-9)
        assert p.info()["k"] == 316


def test_graph_rebuilt_when_options_change(pc):
    """lambda, tau and the sampling change between calls; each change must
    reach the replayed steps."""
    inst = make_config("small_2000x1000", dtype="f64")
    ref = oracle.Solver(inst.A, inst.b, inst.lam, tau=8, seed=4)
    with pc.Problem(inst.A, inst.b, inst.lam, 8, seed=4) as p:
        p.set_option("refresh_every", 0)
        p.step(64)
        ref.step(64)
        p.set_option("lambda", inst.lam * 0.5)
        ref.lam = inst.lam * 0.5
        p.step(64)
        ref.step(64)
        np.testing.assert_allclose(p.get_x(), ref.x, rtol=0, atol=1e-9)
        p.set_option("tau", 20)
        ref2 = oracle.Solver(inst.A, inst.b, inst.lam * 0.5, tau=20, seed=4, x0=ref.x)
        ref2.k = ref.k
        p.step(64)
        ref2.step(64)
        np.testing.assert_allclose(p.get_x(), ref2.x, rtol=0, atol=1e-9)
        p.set_sampling("independent")
        ref3 = oracle.Solver(inst.A, inst.b, inst.lam * 0.5, tau=20, seed=4, x0=ref2.x, sampling="independent")
        ref3.k = ref2.k
        p.step(96)
        ref3.step(96)
        np.testing.assert_allclose(p.get_x(), ref3.x, rtol=0, atol=1e-9)


def test_graph_replays_with_independent_picks_rewind(pc):
    inst = make_config("small_2000x1000", dtype="f64")
    with pc.Problem(inst.A, inst.b, inst.lam, 300, seed=3) as p:
        p.set_sampling("independent")
        p.step(100)
        x1 = p.get_x()
        p.set_x(np.zeros(inst.A.n), k=0)
        p.step(100)
        np.testing.assert_allclose(p.get_x(), x1, rtol=0, atol=1e-12)
