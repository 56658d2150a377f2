"""pcdm_grad_backward_noalloc (temporaries in the library's fixed device
region, no allocation) against pcdm_grad_backward (temporaries from
hipMalloc) on the same handles: two calls in a row, the second on a smaller
problem, so the second reuses a region the first left filled.  A problem
whose temporaries exceed the region is rejected before any work."""

import numpy as np
import pytest

from workloads import make_config

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


def _solved(pc, scale, dtype):
    inst = make_config("train_1e5x1e6", scale=scale, dtype="f64")
    A = inst.A.astype(dtype)
    p = pc.Problem(A, inst.b, inst.lam, 256, seed=1)
    p.set_option("adj_tol", 1e-12)
    st = p.solve(rel_gap=1e-12 if dtype == "f64" else 1e-6, check_every=5, max_epochs=20000)
    assert st["converged"], st
    return p


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_allocating_entry_point(pc, dtype):
    import torch
    for call, scale in enumerate([0.02, 0.01]):  # 2000 x 20000, then 1000 x 10000
        p = _solved(pc, scale, dtype)
        try:
            gen = torch.Generator(device="cpu").manual_seed(100 + call)
            dL_dx = torch.randn(p.n, generator=gen, dtype=torch.float64).cuda()
            want_db, want_dl = p.grad_backward(dL_dx)
            got_db, got_dl = p.grad_backward_noalloc(dL_dx)
            torch.cuda.synchronize()
            support = int(np.count_nonzero(p.get_x()))
        finally:
            p.close()
        want = want_db.cpu().numpy()
        got = got_db.cpu().numpy()
        scale_db = max(np.max(np.abs(want)), 1e-300)
        err = np.max(np.abs(got - want)) / scale_db
        _say(f"{dtype} call {call} (m={want.size}, support {support}): dL/db rel diff {err:.2e}, "
             f"dL/dlambda {got_dl:.12e} vs {want_dl:.12e}")
        assert support > 0
        # same kernels and sampler; only the order of float64 atomic adds into
        # A_S v differs, and both solves stop at a normal-equation residual of
        # 1e-12 relative
        assert err <= 1e-8
        assert got_dl == pytest.approx(want_dl, rel=1e-8, abs=1e-12 * scale_db)


def test_noalloc_rejects_problems_beyond_its_region(pc):
    from workloads import CSC
    m, n = 64, 3_000_000  # temporaries of about 13 n bytes > 32 MiB
    rng = np.random.default_rng(0)
    A = CSC(m, n, np.arange(n + 1, dtype=np.int64), rng.integers(0, m, n).astype(np.int32),
            np.ones(n, dtype=np.float32))
    import torch
    with pc.Problem(A, np.ones(m), 0.1, 1024, seed=0) as p:
        with pytest.raises(pc.PCDMError, match="fixed scratch"):
            p.grad_backward_noalloc(torch.ones(n, dtype=torch.float64, device="cuda"))
