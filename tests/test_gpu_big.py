"""The 2e8 x 5e8 (1e10 nonzero) instance and its generator.

The instance is written on the device by the counter-based recipe of
workloads/csrc/gen_common.h; the host build of the same recipe regenerates
any column, so the oracle gets its inputs without reading device memory.
"""

import numpy as np
import pytest

import oracle
from workloads import biggen
from workloads.lasso import _abs_rmatvec_max

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


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_device_generator_matches_host_build(pc, dtype):
    import torch
    m, n, d, K = 2000, 5000, 20, 50
    A, b, xs = biggen.device_instance(m, n, d, K, 0.01, seed=3, dtype=dtype)
    H, hb, hx = biggen.host_instance(m, n, d, K, 0.01, seed=3, dtype=dtype)
    assert np.array_equal(A.col_ptr.cpu().numpy(), H.col_ptr)
    assert np.array_equal(A.row_idx.cpu().numpy(), H.row_idx)
    dv = A.values.float().cpu().numpy().astype(np.float64)
    hv = H.values_f64()
    ulp = np.spacing(np.abs(hv).astype(np.float32)).astype(np.float64) * (256 if dtype == "bf16" else 1)
    assert np.all(np.abs(dv - hv) <= ulp)
    np.testing.assert_array_equal(xs.cpu().numpy(), hx)
    np.testing.assert_allclose(b.cpu().numpy(), hb, rtol=1e-12, atol=1e-15)


def test_scaled_recipe_matches_oracle(pc):
    """The big recipe at 2e5 x 5e5 (1e7 nnz): device-built problem vs the
    oracle on the host-built one, three steps of tau = 2^16."""
    m, n, d, K = 200_000, 500_000, 20, 1000
    A, b, _ = biggen.device_instance(m, n, d, K, 0.01, seed=5, dtype="f32")
    H, hb, _ = biggen.host_instance(m, n, d, K, 0.01, seed=5, dtype="f32")
    lam = 0.05 * _abs_rmatvec_max(H, hb)
    tau = 1 << 16
    ref = oracle.Solver(H, hb, lam, tau=tau, seed=0)
    with pc.Problem(A, b, lam, tau, seed=0) as p:
        assert p.info()["omega"] == ref.omega
        for s in range(3):
            p.step(1)
            ref.step(1)
            F, _ = p.objective()
            assert F == pytest.approx(ref.objective(), rel=1e-5), s


# --------------------------------------------------------------------------- #
# the full 2e8 x 5e8 instance (1e10 nonzeros), tau = 2^20, float32 values (the
# launch configuration the benchmark times) and bf16 values
# --------------------------------------------------------------------------- #

BIG = dict(m=200_000_000, n=500_000_000, d=20, K=100_000, sigma=0.01, seed=0)
BIG_TAU = 1 << 20
CHUNK = 1 << 22


def _host_pass(out, dtype):
    """b, omega and ||A^T b||_inf of the whole instance on the host: every
    column regenerated from the recipe (threads) with the stored values of
    the dtype, the statistics by the oracle.  Runs beside the device work."""
    try:
        m, n, d, K, sigma, seed = (BIG[k] for k in ("m", "n", "d", "K", "sigma", "seed"))
        b = biggen.host_b(seed, m, n, d, K, sigma, dtype)
        st = oracle.ColumnStats(m, b)
        for i0 in range(0, n, CHUNK):
            cnt = min(CHUNK, n - i0)
            cp, rows, vals = biggen.host_columns(seed, m, n, d, i0, cnt, dtype)
            st.add(cp, rows, vals)
        out["b"], out["stats"] = b, st
    except BaseException as e:  # reported by the test that joins
        out["error"] = e


@pytest.fixture(scope="module", params=["f32", "bf16"])
def big(pc, request):
    """The instance generated on the device and handed to the library (its
    own omega, beta and ||A^T b||_inf; lambda = 0.05 ||A^T b||_inf from the
    library's value), with the host pass running beside it."""
    import threading
    import time

    import torch
    dtype = request.param
    host = {}
    th = threading.Thread(target=_host_pass, args=(host, dtype), daemon=True)
    t0 = time.time()
    th.start()
    m, n, d, K, sigma, seed = (BIG[k] for k in ("m", "n", "d", "K", "sigma", "seed"))
    A, b, _ = biggen.device_instance(m, n, d, K, sigma, seed=seed, dtype=dtype)
    torch.cuda.synchronize()
    _say(f"generated 1e10 {dtype} entries on the device ({time.time() - t0:.0f} s)")
    p = pc.Problem(A, b, 1.0, BIG_TAU, seed=seed)
    del A, b
    torch.cuda.empty_cache()
    inf = p.info()
    p.set_option("lambda", 0.05 * inf["atb_inf"])
    _say(f"created ({time.time() - t0:.0f} s): omega {inf['omega']}, beta {inf['beta']:.6f}, "
         f"||A^T b||_inf {inf['atb_inf']:.15e}, gather route {inf['gather_route']}")
    # automatic route: by rows here (r = 800 MB, beyond the Infinity Cache, and tau = 2^20);
    # the plan below sets each step's route explicitly
    assert inf["gather_route"] == 2
    yield {"p": p, "host": host, "thread": th, "t0": t0, "dtype": dtype}
    p.close()
    torch.cuda.empty_cache()


def _host(big):
    import time
    th = big["thread"]
    while th.is_alive():
        th.join(timeout=20)
        _say(f"  host pass running ({time.time() - big['t0']:.0f} s)")
    if "error" in big["host"]:
        raise big["host"]["error"]
    return big["host"]


def test_full_size_create_matches_host_pass(big):
    """omega, ||A^T b||_inf and beta of the library at 1e10 nonzeros against
    the oracle's statistics over every host-regenerated column."""
    p = big["p"]
    inf = p.info()
    st = _host(big)["stats"]
    _say(f"host: omega {st.omega}, ||A^T b||_inf {st.atb_inf:.15e} over {st.ncols} columns")
    assert st.ncols == BIG["n"]
    assert inf["omega"] == st.omega
    # one float64 dot per column in either order of 20 terms: both within
    # 22 ulp-of-sum of the exact value
    assert inf["atb_inf"] == pytest.approx(st.atb_inf, rel=1e-13)
    assert inf["beta"] == pytest.approx(oracle.beta_nice(st.omega, BIG_TAU, BIG["n"]), rel=1e-15)


def test_full_size_steps_match_oracle(big):
    """Three steps of tau = 2^20 at 1e10 nonzeros (the second one with the
    partial derivatives taken by rows), then three of tau = 2^16 (the
    lane-group layout) from the state they reach: after every step F (float64
    refresh on the device) against the oracle's F on its own float64 r and x,
    every coordinate of S_k against the oracle's, coordinates outside every
    S_k still 0, and the count of nonzero updates of step 0 (from x = 0 a
    coordinate changes iff |g_i| > lambda) against the oracle's, up to the
    coordinates whose |g_i| lies within the float32 error bound of lambda.
    The oracle holds r and x whole and steps on S_k's regenerated columns,
    with its own lambda (0.05 of its ||A^T b||_inf) and beta."""
    import torch
    p = big["p"]
    m, n, d, seed = BIG["m"], BIG["n"], BIG["d"], BIG["seed"]
    host = _host(big)
    st = host["stats"]
    lam = 0.05 * st.atb_inf
    ref = oracle.ColumnSetSolver(m, n, host["b"], lam, oracle.beta_nice(st.omega, BIG_TAU, n))
    touched = np.zeros(0, dtype=np.int64)
    # (step, tau, gather route)
    plan = [(0, BIG_TAU, 2), (1, BIG_TAU, 1), (2, BIG_TAU, 2), (3, 1 << 16, 1), (4, 1 << 16, 1), (5, 1 << 16, 1)]
    for k, tau, route in plan:
        if tau != p.info()["tau"]:
            p.set_option("tau", tau)
            ref.beta = oracle.beta_nice(st.omega, tau, n)
            assert p.info()["beta"] == pytest.approx(ref.beta, rel=1e-15)
        S = np.sort(oracle.sample_nice(seed, k, tau, n).astype(np.int64))
        cp, rows, vals = biggen.host_column_list(seed, m, n, d, S, big["dtype"])
        if k == 0:
            g = ref.gradient(S, cp, rows, vals)
            # float32 r = fl32(-b) and float32 sums of d products: |error| <=
            # (d + 3) u sum |a_ji||r_j| with u = 2^-24
            absdot = np.add.reduceat(np.abs(vals) * np.abs(ref.r[rows]), cp[:-1])
            edge = int(np.count_nonzero(np.abs(np.abs(g) - lam) <= (d + 3) * 2.0 ** -24 * absdot))
        changed = ref.step_with_columns(S, cp, rows, vals)
        p.set_option("gather_route", route)
        assert p.info()["gather_route"] == route
        p.step(1)
        if k == 0:
            got = p.info()["nonzero_updates"]
            _say(f"step 0: nonzero updates {got} vs oracle {changed} ({edge} within the float32 bound of lambda)")
            assert abs(got - changed) <= edge
        F, _ = p.objective()
        F_ref = ref.objective()
        x = p.get_x_tensor()
        got_x = x[torch.as_tensor(S, device="cuda")].cpu().numpy()
        touched = np.union1d(touched, S)
        probe = np.setdiff1d(np.random.default_rng(k).choice(n, 20000, replace=False), touched)[:8192]
        outside = x[torch.as_tensor(probe, device="cuda")].cpu().numpy()
        del x
        want_x = ref.x[S]
        xerr = np.max(np.abs(got_x - want_x)) / max(np.max(np.abs(ref.x)), 1e-300)
        _say(f"step {k} (tau {tau}): F {F:.12e} vs oracle {F_ref:.12e} (rel {abs(F - F_ref) / F_ref:.2e}); "
             f"x on S_k max err {xerr:.2e} of max|x|; {np.count_nonzero(want_x)} nonzero on S_k")
        assert F == pytest.approx(F_ref, rel=1e-5)
        assert xerr <= 1e-5
        assert np.all(outside == 0.0)
