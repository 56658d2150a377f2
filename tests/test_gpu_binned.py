"""Partial derivatives by rows (option gather_route = 2): the step's entries
dealt into bins by (row range, window of 2^18 rows), r read window by window,
per-range partial sums added per slot.  Against the oracle on the same
stored values (float32 / bf16: F within 1e-5 at every check, x within
1e-5 of max|x|), on shapes that exercise several windows per range, ragged
tau (a partial binning workgroup and slot block), tiny row counts, graph
replays, and the overflow fallback (a step whose bins overflow is taken by
the plain gather)."""

import numpy as np
import pytest

import oracle
from workloads import planted_lasso, random_csc, random_csc_ragged

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


def _instance(m, n, d, seed, dtype, balanced=True):
    rng = np.random.default_rng(seed)
    A = random_csc(m, n, d, rng, balanced=balanced, normalize=True, dtype=dtype)
    return planted_lasso(A, max(1, n // 100), 0.01, 0.05, rng)


def _run(pc, inst, tau, rounds, steps, cap=0, graph_steps=32, seed=3):
    ref = oracle.Solver(inst.A, inst.b, inst.lam, tau=tau, seed=seed)
    with pc.Problem(inst.A, inst.b, inst.lam, tau, seed=seed) as p:
        p.set_option("gather_route", 2)
        if cap:
            p.set_option("bin_capacity", cap)
        p.set_option("graph_steps", graph_steps)
        assert p.info()["gather_route"] == 2
        worst = 0.0
        for rnd in range(rounds):
            p.step(steps)
            ref.step(steps)
            F, _ = p.objective()
            Fr = ref.objective()
            worst = max(worst, abs(F - Fr) / abs(Fr))
            assert F == pytest.approx(Fr, rel=1e-5), rnd
        x = p.get_x()
        assert p.info()["gather_route"] == 2
    xerr = np.max(np.abs(x - ref.x)) / max(np.max(np.abs(ref.x)), 1e-300)
    _say(f"  worst rel F {worst:.2e}, x err {xerr:.2e} of max|x|, {np.count_nonzero(ref.x)} nonzero")
    assert xerr <= 1e-5
    return x


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_binned_several_windows_ragged_tau(pc, dtype):
    """3e6 rows: 8 ranges of 375,000 rows, two windows each (the second
    partial); tau = 50,001 leaves a partial binning workgroup and a partial
    slot block."""
    inst = _instance(3_000_000, 200_000, 20, 1, dtype)
    _run(pc, inst, 50_001, rounds=4, steps=3)


def test_binned_tiny_rows_all_columns(pc):
    """m = 5000 (ranges of 625 rows, one window), tau = n: every column in
    every step, with graph replays of 8 steps between direct launches."""
    inst = _instance(5000, 3000, 12, 2, "f32", balanced=False)
    _run(pc, inst, 3000, rounds=3, steps=20, graph_steps=8)


def test_binned_long_run_with_refreshes(pc):
    """Several epochs (float64 refreshes between graph replays) on 1e6 rows."""
    inst = _instance(1_000_000, 100_000, 20, 4, "f32")
    _run(pc, inst, 16384, rounds=3, steps=40)


def test_binned_overflow_falls_back_to_the_plain_gather(pc):
    """Capacity 1 entry per bin: every step overflows and is taken by the
    plain gather; the trajectory still follows the oracle."""
    inst = _instance(2_500_000, 60_000, 20, 5, "f32")
    _run(pc, inst, 20_000, rounds=3, steps=2, cap=1)


def test_binned_partial_overflow(pc):
    """A capacity near the mean count: some steps overflow and some do not."""
    inst = _instance(2_500_000, 60_000, 20, 6, "f32")
    # mean entries per bin: 1024 * 20 / (8 * 2) = 1280
    _run(pc, inst, 20_000, rounds=4, steps=2, cap=1290)


def test_binned_route_eligibility(pc):
    rng = np.random.default_rng(7)
    A = random_csc_ragged(400, 300, 1, 9, rng).astype("f32")  # unequal column lengths
    inst = planted_lasso(A, 5, 0.01, 0.1, rng)
    with pc.Problem(inst.A, inst.b, inst.lam, 64, seed=0) as p:
        assert p.info()["gather_route"] == 1
        with pytest.raises(pc.PCDMError, match="equal column lengths"):
            p.set_option("gather_route", 2)
    inst = _instance(2000, 1000, 8, 8, "f64")
    with pc.Problem(inst.A, inst.b, inst.lam, 64, seed=0) as p:
        with pytest.raises(pc.PCDMError, match="float32 or bf16"):
            p.set_option("gather_route", 2)
    inst = _instance(2000, 1000, 8, 9, "f32")
    with pc.Problem(inst.A, inst.b, inst.lam, 64, seed=0) as p:
        assert p.info()["gather_route"] == 1  # automatic: small r, small tau
        p.set_option("gather_route", 2)
        assert p.info()["gather_route"] == 2
        p.set_sampling("independent")  # not eligible: steps fall back to route 1
        assert p.info()["gather_route"] == 1
        p.set_sampling("nice")
        assert p.info()["gather_route"] == 2
        p.set_slot_mask(np.ones(64, dtype=np.uint8))
        assert p.info()["gather_route"] == 1
        p.set_slot_mask(None)
        assert p.info()["gather_route"] == 2
        p.set_option("gather_route", 1)
        assert p.info()["gather_route"] == 1


# --------------------------------------------------------------------------- #
# residual scatter by row blocks (option scatter_route = 2)
# --------------------------------------------------------------------------- #

def _run_s(pc, inst, tau, rounds, steps, cap=0, graph_steps=32, seed=5, gather_route=1, narrow=None):
    ref = oracle.Solver(inst.A, inst.b, inst.lam, tau=tau, seed=seed)
    with pc.Problem(inst.A, inst.b, inst.lam, tau, seed=seed) as p:
        p.set_option("scatter_route", 2)
        p.set_option("gather_route", gather_route)
        if cap:
            p.set_option("scatter_capacity", cap)
        if narrow is not None:
            p.set_option("narrow_below", narrow)
        p.set_option("graph_steps", graph_steps)
        assert p.info()["scatter_route"] == 2
        worst = 0.0
        for rnd in range(rounds):
            p.step(steps)
            ref.step(steps)
            F, _ = p.objective()
            Fr = ref.objective()
            worst = max(worst, abs(F - Fr) / abs(Fr))
            assert F == pytest.approx(Fr, rel=1e-5), rnd
        x = p.get_x()
        r_lib = p.get_residual()
        nz = p.info()["nonzero_updates"]
    xerr = np.max(np.abs(x - ref.x)) / max(np.max(np.abs(ref.x)), 1e-300)
    _say(f"  worst rel F {worst:.2e}, x err {xerr:.2e} of max|x|, {nz} nonzero updates")
    assert xerr <= 1e-5
    return r_lib


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_row_block_scatter_ragged_tau(pc, dtype):
    """1e6 rows (245 blocks of 4096), tau = 50,001: a partial last packing
    workgroup and a partial last row block."""
    inst = _instance(1_000_000, 200_000, 20, 11, dtype)
    _run_s(pc, inst, 50_001, rounds=4, steps=3)


def test_row_block_scatter_tiny_rows_graphs(pc):
    """m = 5000 (two row blocks), tau = n, graph replays of 8 steps."""
    inst = _instance(5000, 3000, 12, 12, "f32", balanced=False)
    _run_s(pc, inst, 3000, rounds=3, steps=20, graph_steps=8)


def test_row_block_scatter_overflow_goes_to_atomics(pc):
    """Capacity 1 per run: almost every product is added with an atomic in
    the packing kernel; the trajectory is unchanged."""
    inst = _instance(300_000, 60_000, 20, 13, "f32")
    _run_s(pc, inst, 20_000, rounds=3, steps=3, cap=1)


def test_row_block_scatter_with_rows_gather_and_narrow_layout(pc):
    """Both routes by rows together; then the lane-group layout of small tau."""
    inst = _instance(2_500_000, 60_000, 20, 14, "f32")
    _run_s(pc, inst, 20_000, rounds=3, steps=2, gather_route=2)
    inst = _instance(100_000, 30_000, 20, 15, "f32")
    _run_s(pc, inst, 1000, rounds=3, steps=30, narrow=10**9)


def test_row_block_scatter_keeps_the_residual(pc):
    """Over several epochs (float64 refreshes in between) the maintained r
    stays the residual of the iterate: r = A x - b to float32 accuracy."""
    import scipy.sparse as sp
    inst = _instance(1_000_000, 100_000, 20, 16, "f32")
    rng = np.random.default_rng(0)
    with pc.Problem(inst.A, inst.b, inst.lam, 16384, seed=1) as p:
        p.set_option("scatter_route", 2)
        p.set_option("refresh_every", 0)  # no refresh: r is only what the scatters made it
        p.step(25)
        x = p.get_x()
        r = p.get_residual()
    M = sp.csc_matrix((inst.A.values_f64(), inst.A.row_idx, inst.A.col_ptr), shape=(inst.A.m, inst.A.n))
    want = M @ x - inst.b
    err = np.max(np.abs(r - want)) / np.max(np.abs(inst.b))
    _say(f"  drift of r after 25 steps without refresh: {err:.2e} of max|b|")
    assert err <= 1e-5


def test_row_block_scatter_eligibility(pc):
    inst = _instance(2000, 1000, 8, 17, "f64")
    with pc.Problem(inst.A, inst.b, inst.lam, 64, seed=0) as p:
        assert p.info()["scatter_route"] == 1
        with pytest.raises(pc.PCDMError, match="float32 or bf16"):
            p.set_option("scatter_route", 2)
    inst = _instance(2000, 1000, 8, 18, "f32")
    with pc.Problem(inst.A, inst.b, inst.lam, 64, seed=0) as p:
        p.set_option("scatter_route", 2)
        assert p.info()["scatter_route"] == 2
        p.set_option("tau", 500)
        assert p.info()["scatter_route"] == 2
        p.set_option("scatter_route", 1)
        assert p.info()["scatter_route"] == 1
