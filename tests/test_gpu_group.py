"""Blocks of several coordinates (group LASSO) on the HIP path vs the float64
block oracle (section "Block structure, notation and assumptions"; group-lasso
example of block separable Omega; eq. h(x); Table ESO over blocks).

The library computes L_i = lambda_max(A_i^T A_i) by Jacobi rotations on the
device; the oracle by a library eigen-solver.  Tolerances as for the
coordinate path: float64 1e-10 on F and 1e-9 on x, float32 1e-5 on F.
"""

import numpy as np
import pytest

import oracle
from oracle import group
from workloads import csc_to_dense, orthonormal_block_hadamard, planted_lasso, random_csc, random_csc_ragged

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


def _random_blocks(n, rng, lo=1, hi=16):
    sizes = []
    left = n
    while left:
        s = min(left, int(rng.integers(lo, hi + 1)))
        sizes.append(s)
        left -= s
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def _pair(pc, inst, bp, tau, seed, steps, chunks, rtol_F, x_atol, lanes=0):
    ref = group.GroupSolver(inst.A, inst.b, inst.lam, bp, tau=tau, seed=seed)
    with pc.Problem(inst.A, inst.b, inst.lam, tau, seed=seed, blocks=bp) as p:
        if lanes:
            p.set_option("lanes_per_column", lanes)
        inf = p.info()
        assert inf["nblocks"] == len(bp) - 1
        assert inf["omega"] == ref.omega
        assert inf["beta"] == pytest.approx(ref.beta, rel=1e-15)
        worst = 0.0
        for _ in range(chunks):
            p.step(steps)
            ref.step(steps)
            F, _ = p.objective()
            Fr = ref.objective()
            worst = max(worst, abs(F - Fr) / abs(Fr))
            assert abs(F - Fr) <= rtol_F * abs(Fr), (F, Fr)
        if x_atol is not None:
            np.testing.assert_allclose(p.get_x(), ref.x, rtol=0, atol=x_atol)
    return worst


@pytest.mark.parametrize("tau", [1, 7, 40])
def test_blocks_float64_match_oracle(pc, tau):
    rng = np.random.default_rng(tau)
    A = random_csc_ragged(600, 500, 1, 30, rng)
    inst = planted_lasso(A, 40, 0.01, 0.2, rng)
    bp = _random_blocks(500, rng)
    nb = len(bp) - 1
    tau = min(tau, nb)
    worst = _pair(pc, inst, bp, tau, 3, 2 * (-(-nb // tau)), 8, 1e-10, 1e-9)
    _say(f"blocks f64 tau={tau} nb={nb}: worst {worst:.2e}")


def test_all_blocks_in_one_step(pc):
    rng = np.random.default_rng(11)
    A = random_csc(300, 200, 5, rng)
    inst = planted_lasso(A, 20, 0.01, 0.2, rng)
    bp = _random_blocks(200, rng, 2, 6)
    _pair(pc, inst, bp, len(bp) - 1, 0, 3, 6, 1e-10, 1e-9)


def test_single_column_blocks(pc):
    rng = np.random.default_rng(12)
    A = random_csc(200, 150, 6, rng)
    inst = planted_lasso(A, 10, 0.01, 0.1, rng)
    _pair(pc, inst, np.arange(151, dtype=np.int64), 16, 2, 20, 5, 1e-10, 1e-9)


@pytest.mark.parametrize("lanes", [1, 4, 32])
def test_blocks_lane_counts(pc, lanes):
    rng = np.random.default_rng(20 + lanes)
    A = random_csc_ragged(400, 300, 1, 40, rng)
    inst = planted_lasso(A, 20, 0.01, 0.2, rng)
    bp = _random_blocks(300, rng)
    _pair(pc, inst, bp, 9, 1, 10, 4, 1e-10, 1e-9, lanes=lanes)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_blocks_low_precision(pc, dtype):
    rng = np.random.default_rng(30)
    A = random_csc(2000, 3000, 10, rng, dtype=dtype)
    inst = planted_lasso(A, 60, 0.01, 0.1, rng)
    bp = _random_blocks(3000, rng, 1, 8)
    worst = _pair(pc, inst, bp, 64, 4, 30, 5, 1e-5, None)
    _say(f"blocks {dtype}: worst {worst:.2e}")


def test_orthonormal_closed_form(pc):
    A = orthonormal_block_hadamard(64, 4)
    M = csc_to_dense(A)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(A.m) * 3
    bp = _random_blocks(A.n, rng, 1, 7)
    lam = 1.2
    with pc.Problem(A, b, lam, 5, seed=2, blocks=bp) as p:
        st = p.solve(rel_gap=1e-12, check_every=10)
        assert st["converged"], st
        x = p.get_x()
    atb = M.T @ b
    want = np.concatenate([group.block_soft(atb[bp[i]:bp[i + 1]], lam) for i in range(len(bp) - 1)])
    np.testing.assert_allclose(x, want, atol=1e-10)


def test_objective_and_gap_at_a_point(pc):
    rng = np.random.default_rng(7)
    A = random_csc(300, 240, 6, rng)
    inst = planted_lasso(A, 20, 0.01, 0.2, rng)
    bp = _random_blocks(240, rng, 1, 10)
    ref = group.GroupSolver(inst.A, inst.b, inst.lam, bp, tau=4, seed=0)
    x = rng.standard_normal(240) * (rng.random(240) < 0.3)
    ref.x = x.copy()
    gap_r, F_r, _ = ref.gap()
    with pc.Problem(inst.A, inst.b, inst.lam, 4, seed=0, blocks=bp) as p:
        p.set_x(x)
        F, gap = p.objective(gap=True)
    assert F == pytest.approx(F_r, rel=1e-12)
    assert gap == pytest.approx(gap_r, rel=1e-10, abs=1e-12 * abs(F_r))


def test_block_error_paths(pc):
    from paper_1212_0873_amd import PCDMError
    rng = np.random.default_rng(0)
    A = random_csc(40, 40, 3, rng)
    b = rng.standard_normal(40)
    # blocks over 16 columns, not starting at 0, not ending at n, an empty block
    for bp in ([0, 20, 40], [1, 20, 40], [0, 12, 39], [0, 10, 10, 24, 40], [0, 17, 40]):
        with pytest.raises(PCDMError):
            pc.Problem(A, b, 0.1, 1, blocks=np.array(bp, dtype=np.int64))
    bp = np.arange(0, 41, 4, dtype=np.int64)
    with pytest.raises(PCDMError):
        pc.Problem(A, b, 0.1, 11, blocks=bp)          # tau > blocks
    with pc.Problem(A, b, 0.1, 3, blocks=bp) as p:
        with pytest.raises(PCDMError):
            p.set_sampling("independent")
        with pytest.raises(PCDMError):
            p.set_slot_mask(np.ones(3, np.uint8))
        with pytest.raises(PCDMError):
            p.step_async(1)
        with pytest.raises(PCDMError):
            p.grad_backward(np.ones(40))
        with pytest.raises(PCDMError):
            p.set_option("tau", 11)
        p.set_option("tau", 10)
        assert p.info()["beta"] == pytest.approx(oracle.beta_nice(p.info()["omega"], 10, 10))
        p.step(3)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_gap_two_passes_equal_one(pc, dtype):
    """The block-norm maximum of the group gap: bound pass over fl32(r) plus
    exact norms of the candidate blocks gives the single pass's number.  x is
    supported on blocks that share no row, so the float64 residual does not
    depend on the order of the refresh's atomic adds."""
    rng = np.random.default_rng(40)
    A = random_csc(900, 600, 4, rng).astype(dtype)
    b = rng.standard_normal(900) * 10.0 ** rng.uniform(-20, 20, 900)
    bp = _random_blocks(600, rng, 1, 6)
    used = np.zeros(900, dtype=bool)
    x = np.zeros(600)
    for i in rng.permutation(len(bp) - 1):
        rows = np.concatenate([A.row_idx[A.col_ptr[c]:A.col_ptr[c + 1]] for c in range(bp[i], bp[i + 1])])
        if not used[rows].any():
            used[rows] = True
            x[bp[i]:bp[i + 1]] = rng.standard_normal(bp[i + 1] - bp[i]).astype(np.float32)
    out = {}
    for passes in (1, 2, 3):
        with pc.Problem(A, b, 0.3, 5, seed=0, blocks=bp) as p:
            p.set_option("max_passes", passes)
            p.set_x(x)
            out[passes] = p.objective(gap=True)
    assert out[1] == out[2] == out[3], out
    ref = group.GroupSolver(A, b, 0.3, bp, tau=5, seed=0)
    ref.x = x.copy()
    gap_r, F_r, _ = ref.gap()
    assert out[2][0] == pytest.approx(F_r, rel=1e-12)
    assert out[2][1] == pytest.approx(gap_r, rel=1e-9, abs=1e-12 * abs(F_r))
