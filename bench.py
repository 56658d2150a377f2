#!/usr/bin/env python3
"""Throughput of the synchronous PCDM step (LASSO) on one MI355X.

A "step" is one synchronous PCDM1 iteration over tau sampled coordinates
(sample, partial derivatives, damped soft-threshold, residual scatter), with
the float64 residual refresh the library runs once per epoch.  The default
workload is the 2e8 x 5e8 LASSO with 20 nonzeros per column (1e10 nnz,
float32 values, balanced rows, written on the device by the counter-based
recipe) at tau = 2^20; inputs are synthetic and seeded, and resident in HBM
before the timed region.

Prints one JSON line: updates/s, the dominant kernel's roofline figure (HIP
event time of every launch in the timed region), the float64 CPU oracle's
rate on a bounded sample of the same workload, and the wall time until the
certified duality gap falls below 1e-6 of the objective.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
import types
from typing import Optional

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coord updates/s + HBM GB/s (% roofline); time to 1e-6 rel. objective gap"
HBM_PEAK_GBPS = 8000.0
WORKLOAD_NAMES = {
    "small_2000x1000": "lasso_2000x1000_d20_uniform",
    "lasso_1e6x1e7": "lasso_1e6x1e7_d20_balanced",
    "lasso_3.33e6x1e7": "lasso_3.33e6x1e7_d20_balanced",
    "train_1e5x1e6": "lasso_1e5x1e6_d10_uniform",
    "lasso_2e8x5e8": "lasso_2e8x5e8_d20_balanced",
}
KERNEL_SOURCES = ("kernels.hpp", "sampler.hpp", "binned_kernels.hpp", "pcdm.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1212_0873_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, workload: str, dtype: str, tau: int):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{WORKLOAD_NAMES[workload]}_{dtype}_tau{tau}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.startswith("#"):
                k, v = line.strip().split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def algorithmic_bytes(d_avg: float, s_val: int):
    """Bytes the method must move per coordinate update (no re-reads):
    gather: column pointers 2x8, column entries d*(4+s_val), r gathers d*4,
    x read + invL read + x write 3x4; scatter (delta != 0 only): r
    read-modify-write d*8."""
    gather = 16 + d_avg * (4 + s_val) + d_avg * 4 + 12
    scatter = d_avg * 8
    return gather, scatter


def cpu_model() -> Optional[str]:
    try:
        with open("/proc/cpuinfo") as fh:
            return next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        return None


def big_host_pass(cfg: dict, dtype: str, out: dict, chunk: int = 1 << 22) -> None:
    """The oracle's own set-up for an instance built on the device: b, omega
    and ||A^T b||_inf over every column regenerated on the host (threads).
    Not timed; it gives the oracle its lambda and beta."""
    try:
        import oracle
        from workloads import biggen
        m, n, d = cfg["m"], cfg["n"], cfg["d"]
        b = biggen.host_b(0, m, n, d, cfg["xstar_nnz"], cfg["noise_std"], dtype)
        st = oracle.ColumnStats(m, b)
        for i0 in range(0, n, chunk):
            cp, rows, vals = biggen.host_columns(0, m, n, d, i0, min(chunk, n - i0), dtype)
            st.add(cp, rows, vals)
            out["progress"] = min(1.0, (i0 + chunk) / n)
        out["b"], out["stats"] = b, st
    except BaseException as e:  # re-raised by the caller
        out["error"] = e


def big_cpu_baseline(cfg: dict, dtype: str, host: dict, tau: int, seconds: float,
                     min_updates: int = 10_000_000) -> dict:
    """The float64 oracle's PCDM1 steps on the same instance from x = 0: it
    holds r and x whole and steps on S_k's columns, regenerated on the host
    before each timed step (regeneration outside the timer).  Steps until
    both `seconds` of timed work and `min_updates` updates are done."""
    import numpy as np

    import oracle
    from workloads import biggen
    m, n, d = cfg["m"], cfg["n"], cfg["d"]
    st = host["stats"]
    lam = cfg["lam_factor"] * st.atb_inf
    beta = oracle.beta_nice(st.omega, tau, n)
    ref = oracle.ColumnSetSolver(m, n, host["b"], lam, beta)
    steps = 0
    timed = 0.0
    while timed < seconds or steps * tau < min_updates:
        S = np.sort(oracle.sample_nice(0, steps, tau, n).astype(np.int64))
        cp, rows, vals = biggen.host_column_list(0, m, n, d, S, dtype)
        t_c = time.perf_counter()
        ref.step_with_columns(S, cp, rows, vals)
        timed += time.perf_counter() - t_c
        steps += 1
    return {"value": steps * tau / timed, "unit": "coord updates/s", "cores": 1, "kind": "oracle",
            "cpu_model": cpu_model(), "host_threads_available": os.cpu_count(),
            "sample": f"{steps} steps of tau={tau} from x=0 on the same {m} x {n} instance ({n * d} nonzeros) "
                      f"({steps * tau} updates, {timed:.1f} s timed, float64, one thread); the oracle holds "
                      f"r ({m}) and x ({n}) in float64 and reads S_k's columns regenerated on the host "
                      f"(not timed); its lambda and beta are its own (omega {st.omega}, "
                      f"||A^T b||_inf {st.atb_inf:.6e} from a threaded pass over every regenerated column, "
                      f"also not timed)"}


def gap_check(args):
    return "auto" if args.gap_check == "auto" else int(args.gap_check)


def time_to_gap(p, target: float, limit_s: float, check_every="auto") -> dict:
    """Wall time from the handle's current state until the certified float64
    duality gap (F - D)/D <= target (``Problem.solve``: gap evaluations inside
    the timed region, every `check_every` epochs or on the cost-aware
    schedule "auto")."""
    st = p.solve(rel_gap=target, check_every=check_every, max_seconds=limit_s)
    return {"target_rel_gap": target, "reached": bool(st["converged"]), "seconds": st["seconds"],
            "epochs": st["epochs"], "rel_gap": st["rel_gap"], "F": st["F"], "check_every_epochs": check_every,
            "gap_evaluations": st["checks"], "includes_gap_evaluations": True,
            "evaluated_at": [(e, float(f"{g:.3g}"), round(c * 1e3, 1)) for e, g, c in st["evaluations"]]}


def oracle_time_to_gap(A, b, lam, tau: int, target: float, limit_s: float) -> dict:
    """The float64 oracle on one core from x = 0 until its certified gap
    (F - D)/D <= target, with the gap evaluations on the schedule the GPU
    solve uses (from the measured cost of the last evaluation and of the
    epochs before it); for instances small enough to solve on the host."""
    import oracle
    from paper_1212_0873_amd.api import next_check_interval
    ref = oracle.Solver(A, b, lam, tau=tau, seed=0)
    spe = ref.steps_per_epoch()
    epochs = checks = 0
    interval = 1
    rel = float("inf")
    last = None
    t0 = t_prev = time.perf_counter()
    while time.perf_counter() - t0 < limit_s:
        ref.step(interval * spe)
        epochs += interval
        t_mid = time.perf_counter()
        gap, F, D = ref.gap()
        checks += 1
        t_end = time.perf_counter()
        rel = gap / max(abs(D), 1e-300)
        if rel <= target:
            break
        trend = (last, (epochs, rel)) if last is not None else None
        interval = next_check_interval(t_end - t_mid, (t_mid - t_prev) / interval, epochs, trend=trend,
                                       target=target)
        last = (epochs, rel)
        t_prev = t_end
    return {"target_rel_gap": target, "reached": bool(rel <= target), "seconds": time.perf_counter() - t0,
            "epochs": epochs, "gap_evaluations": checks, "rel_gap": rel, "cores": 1}


def run_batched(args) -> int:
    """The batched path: `count` uneven LASSO problems on a lambda grid, all
    solved to a certified 1e-6 gap in one batch (graph-replayed steps) vs the
    same problems solved one after the other with the single-problem path."""
    import numpy as np
    import torch

    import paper_1212_0873_amd as pc
    from workloads.configs import batched_path

    torch.cuda.set_device(0)
    t0 = time.time()
    insts = batched_path(count=args.count, dtype=args.dtype)
    probs = [(i.A, i.b, i.lam, i.tau) for i in insts]
    sum_n = sum(i.A.n for i in insts)
    sum_nnz = sum(i.A.nnz for i in insts)
    print(f"[bench] generated {len(insts)} problems, sum n {sum_n}, sum nnz {sum_nnz} in "
          f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    with pc.Batch(probs, seed=0) as tune:
        sched = tune.autotune(2)
    with pc.Batch(probs, seed=0) as B:
        B.set_option("lanes_per_column", sched["lanes_per_column"])
        B.set_option("chunks_per_lane", sched["chunks_per_lane"])
        torch.cuda.synchronize()
        t_b = time.perf_counter()
        st = B.solve(rel_gap=1e-6, check_every_steps=args.check_steps)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t_b
    upd_b = sum(i.tau * (st["done_at"][j] or st["steps"]) for j, i in enumerate(insts))
    seq_t = 0.0
    seq_ok = True
    for j, (A, b, lam, tau) in enumerate(probs):
        with pc.Problem(A, b, lam, tau, seed=j) as p:
            p.set_option("lanes_per_column", sched["lanes_per_column"])
            p.set_option("chunks_per_lane", sched["chunks_per_lane"])
            r = time_to_gap(p, 1e-6, args.gap_seconds, gap_check(args))
        seq_t += r["seconds"]
        seq_ok &= r["reached"]
    out = {"metric": METRIC, "mode": "batched", "value": upd_b / tb, "unit": "coord updates/s",
           "n_gpus": 1, "dtype": args.dtype, "data": "synthetic",
           "config": {"workload": f"lasso_path_{len(insts)}_uneven_d10", "count": len(insts), "sum_n": sum_n,
                      "sum_nnz": sum_nnz, "tau": "min(n_j, 4096)", "schedule": sched,
                      "graph_steps": 32, "check_every_steps": args.check_steps},
           "batched_time_to_gap_s": tb, "batched_converged": st["converged"], "batched_steps": st["steps"],
           "sequential_time_to_gap_s": seq_t, "sequential_converged": seq_ok,
           "speedup_vs_sequential": seq_t / tb}
    print(json.dumps(out), flush=True)
    return 0


def run_dtypes(args) -> int:
    """Time to a certified 1e-6 gap on one instance with float64, float32 and
    bf16 values (same seeded matrix; bf16 and float32 are its roundings), and
    the bf16 problem's objective error against the float64 one."""
    import torch

    import paper_1212_0873_amd as pc
    from workloads import make_config

    torch.cuda.set_device(0)
    inst = make_config(args.config, dtype="f64", tau=args.tau)
    tau = min(args.tau, inst.A.n)
    print(f"[bench] generated {args.config} (nnz {inst.A.nnz})", file=sys.stderr, flush=True)
    res = {}
    for dt in ("f64", "f32", "bf16"):
        A = inst.A.astype(dt) if dt != "f64" else inst.A
        with pc.Problem(A, inst.b, inst.lam, tau, seed=0) as p:
            r = time_to_gap(p, 1e-6, args.gap_seconds, gap_check(args))
            res[dt] = r
        del A
        print(f"[bench] {dt}: {r}", file=sys.stderr, flush=True)
    F64 = res["f64"]["F"]
    out = {"metric": METRIC, "mode": "dtypes", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": WORKLOAD_NAMES[args.config], "tau": tau},
           "time_to_gap_s": {k: v["seconds"] for k, v in res.items()},
           "epochs": {k: v["epochs"] for k, v in res.items()},
           "reached": {k: v["reached"] for k, v in res.items()},
           "objective_rel_diff_vs_f64": {k: (v["F"] - F64) / F64 for k, v in res.items()}}
    print(json.dumps(out), flush=True)
    return 0


def copy_bandwidth_gbps(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """Read + write bandwidth of a plain device-to-device copy (torch)."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes * reps / dt / 1e9


def random_gather_ceiling(m: int, nthreads: int = 1_000_000, reps: int = 20) -> Optional[dict]:
    """Rates of independent random 4-byte reads and of random float atomic
    adds on a table of m floats (the size of the residual), measured with the
    calibration kernels of libpcdm_calib.so: the ceilings of the random-line
    requests that the gathers and the scatter of a coordinate step issue.
    HIP events on the launch stream."""
    import ctypes
    import torch
    from paper_1212_0873_amd import build as hipbuild
    if not os.path.exists(hipbuild.CALIB_LIB):
        return None
    lib = ctypes.CDLL(hipbuild.CALIB_LIB)
    lib.pcdm_calib_random_gather.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32,
                                             ctypes.c_void_p, ctypes.c_void_p]
    lib.pcdm_calib_random_gather.restype = ctypes.c_int
    reads = int(lib.pcdm_calib_reads_per_thread())
    table = torch.rand(m, dtype=torch.float32, device="cuda")
    out = torch.empty(nthreads, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    sptr = ctypes.c_void_p(stream.cuda_stream)

    def launch(salt, rows=m):
        rc = lib.pcdm_calib_random_gather(table.data_ptr(), rows, nthreads, salt, out.data_ptr(), sptr)
        if rc != 0:
            raise RuntimeError(f"pcdm_calib_random_gather failed: {rc}")

    lib.pcdm_calib_random_atomic.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32,
                                             ctypes.c_void_p]
    lib.pcdm_calib_random_atomic.restype = ctypes.c_int

    def launch_atomic(salt):
        rc = lib.pcdm_calib_random_atomic(table.data_ptr(), m, nthreads, salt, sptr)
        if rc != 0:
            raise RuntimeError(f"pcdm_calib_random_atomic failed: {rc}")

    def timed(fn):
        for k in range(3):
            fn(k)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k in range(reps):
            fn(100 + k)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    dt = timed(launch)
    dta = timed(launch_atomic)
    # the same reads on smaller tables: one that each XCD's 4 MB L2 holds whole,
    # and one beyond the L2s but inside the 256 MB Infinity Cache
    by_size = {}
    for small in (1 << 19, 1 << 24):
        if small < m:
            by_size[4 * small] = nthreads * reads / timed(lambda salt: launch(salt, small))
    del table, out
    torch.cuda.empty_cache()
    return {"table_bytes": 4 * m, "reads_per_launch": nthreads * reads, "avg_launch_us": dt * 1e6,
            "reads_per_s": nthreads * reads / dt, "atomic_avg_launch_us": dta * 1e6,
            "atomics_per_s": nthreads * reads / dta,
            "reads_per_s_smaller_tables": {f"{b >> 20} MiB": v for b, v in by_size.items()}}


def read_l2_counters(kernel: str, workload: str, dtype: str, tau: int) -> Optional[dict]:
    """L2 request counters per launch from a committed rocprofv3 summary, if it
    was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"pmc_l2_{kernel}_{WORKLOAD_NAMES[workload]}_{dtype}_tau{tau}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.startswith("#"):
                k, v = line.strip().split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return {k: float(kv[k]) for k in ("tcc_req_per_launch", "tcc_hit_per_launch", "tcc_miss_per_launch",
                                          "calib_tcc_req_per_read")}
    except (KeyError, ValueError):
        return None


def gpu_clocks() -> Optional[str]:
    """Current clock levels as rocm-smi reports them (best effort)."""
    import subprocess
    try:
        r = subprocess.run(["rocm-smi", "--showclocks"], capture_output=True, text=True, timeout=20)
    except Exception:  # noqa: BLE001 - the tool may be absent
        return None
    lines = [ln.strip() for ln in r.stdout.splitlines() if "clock level" in ln.lower()]
    return "; ".join(lines) if lines else None


def measure_rate(p, tau: int, min_seconds: float = 1.0, warmup: int = 20) -> dict:
    """Updates/s of the current handle over at least min_seconds of steps, and
    the average gather/scatter launch time from HIP events (a separate run, so
    the events do not perturb the rate)."""
    import torch
    p.step(warmup)
    torch.cuda.synchronize()
    steps = 16
    while True:
        t0 = time.perf_counter()
        p.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
        steps = int(steps * max(2.0, 1.2 * min_seconds / max(dt, 1e-6)))
    p.set_option("kernel_timing", 1)
    p.step(min(steps, 2000))
    ng, gms = p.kernel_time("gather")
    ns, sms = p.kernel_time("scatter")
    p.set_option("kernel_timing", 0)
    return {"steps": steps, "seconds": dt, "us_per_step": dt / steps * 1e6,
            "slot_updates_per_s": tau * steps / dt,
            "gather_avg_us": gms / max(ng, 1) * 1e3, "scatter_avg_us": sms / max(ns, 1) * 1e3}


def run_taus(args) -> int:
    """tau sweep on the 1e6 x 1e7 instance and its 3.33e6-row variant (omega
    about 61): updates/s, kernel times and time to a certified 1e-6 gap per
    tau; the fixed cost of a step (tau = 1); a plain copy's bandwidth."""
    import numpy as np
    import torch

    import paper_1212_0873_amd as pc
    from workloads import make_config

    torch.cuda.set_device(0)
    out = {"metric": METRIC, "mode": "taus", "n_gpus": 1, "dtype": args.dtype, "data": "synthetic",
           "device": torch.cuda.get_device_name(0), "copy_gbps": copy_bandwidth_gbps(),
           "gpu_clocks": gpu_clocks(), "workloads": {}}
    print(f"[bench] copy {out['copy_gbps']:.0f} GB/s", file=sys.stderr, flush=True)
    for cfg in ("lasso_1e6x1e7", "lasso_3.33e6x1e7"):
        inst = make_config(cfg, dtype=args.dtype)
        A = inst.A
        d_avg = A.nnz / A.n
        b_gather, _ = algorithmic_bytes(d_avg, {"f32": 4, "bf16": 2, "f64": 8}[args.dtype])
        res = {}
        with pc.Problem(A, inst.b, inst.lam, 1, seed=0) as p:
            r1 = measure_rate(p, 1, min_seconds=0.5)
            res["1"] = {"us_per_step": r1["us_per_step"], "gather_avg_us": r1["gather_avg_us"],
                        "scatter_avg_us": r1["scatter_avg_us"], "note": "fixed cost of one step"}
            for tau in (1024, 65536, 1_000_000):
                p.set_option("tau", tau)
                p.set_option("refresh_every", -(-A.n // tau))
                p.set_x(np.zeros(A.n), k=0)
                inf = p.info()
                r = measure_rate(p, tau)
                r["beta"] = inf["beta"]
                r["epoch_steps"] = inf["refresh_every"]
                r["gather_alg_gbps"] = b_gather * tau / (r["gather_avg_us"] * 1e-6) / 1e9
                p.set_x(np.zeros(A.n), k=0)
                r["time_to_gap"] = time_to_gap(p, 1e-6, args.gap_seconds, gap_check(args))
                res[str(tau)] = r
                print(f"[bench] {cfg} tau={tau}: {r}", file=sys.stderr, flush=True)
            omega = p.info()["omega"]
        out["workloads"][WORKLOAD_NAMES[cfg]] = {"m": A.m, "n": A.n, "nnz": A.nnz, "omega": omega, "taus": res}
        del inst, A
    print(json.dumps(out), flush=True)
    return 0


def run_samplings(args) -> int:
    """The samplings on one instance: tau-nice, tau-independent (the paper's
    own runs), (tau, 0.9)-binomial and tau-nice with 10% of the slots down:
    distinct coordinate updates/s, kernel times, time to a certified 1e-6 gap."""
    import numpy as np
    import torch

    import paper_1212_0873_amd as pc
    from workloads import make_config

    torch.cuda.set_device(0)
    inst = make_config(args.config, dtype=args.dtype, tau=args.tau)
    A = inst.A
    tau = min(args.tau, A.n)
    rng = np.random.default_rng(0)
    dead = (rng.random(tau) < 0.1)
    cases = [("nice", 1.0, None), ("independent", 1.0, None), ("binomial", 0.9, None),
             ("nice", 1.0, (~dead).astype(np.uint8))]
    res = {}
    with pc.Problem(A, inst.b, inst.lam, tau, seed=0) as p:
        for sampling, pb, mask in cases:
            name = sampling + ("_mask10" if mask is not None else "") + (f"_p{pb}" if sampling == "binomial" else "")
            p.set_sampling(sampling, pb)
            p.set_slot_mask(mask)
            p.set_x(np.zeros(A.n), k=0)
            inf = p.info()
            r = measure_rate(p, tau)
            es = inf["expected_set_size"] * (1.0 if mask is None else float(mask.mean()))
            r["expected_set_size"] = es
            r["distinct_updates_per_s"] = r["slot_updates_per_s"] * es / tau
            r["beta"] = inf["beta"]
            p.set_x(np.zeros(A.n), k=0)
            r["time_to_gap"] = time_to_gap(p, 1e-6, args.gap_seconds, gap_check(args))
            res[name] = r
            print(f"[bench] {name}: {r}", file=sys.stderr, flush=True)
    out = {"metric": METRIC, "mode": "samplings", "n_gpus": 1, "dtype": args.dtype, "data": "synthetic",
           "config": {"workload": WORKLOAD_NAMES[args.config], "tau": tau}, "samplings": res}
    print(json.dumps(out), flush=True)
    return 0


def async_time_to_gap(p, target: float, limit_s: float, check_every="auto") -> dict:
    """Wall time of asynchronous epochs (n picks each, float64 refresh after
    each) until the certified gap (F - D)/D <= target, checked every
    `check_every` epochs or on the cost-aware schedule of the synchronous
    solve ("auto"); the evaluations are inside the timed region."""
    import torch

    from paper_1212_0873_amd.api import next_check_interval
    auto = check_every == "auto"
    interval = 1 if auto else int(check_every)
    torch.cuda.synchronize()
    t0 = t_prev = time.perf_counter()
    epochs = checks = 0
    rel = float("inf")
    F = None
    last = None
    while time.perf_counter() - t0 < limit_s:
        p.step_async(interval)
        epochs += interval
        torch.cuda.synchronize()
        t_mid = time.perf_counter()
        F, gap = p.objective(gap=True)
        checks += 1
        t_end = time.perf_counter()
        rel = gap / max(abs(F - gap), 1e-300)
        if rel <= target:
            break
        if auto:
            trend = (last, (epochs, rel)) if last is not None else None
            interval = next_check_interval(t_end - t_mid, (t_mid - t_prev) / interval, epochs, trend=trend,
                                           target=target)
            last = (epochs, rel)
        t_prev = t_end
    return {"target_rel_gap": target, "reached": bool(rel <= target), "seconds": time.perf_counter() - t0,
            "epochs": epochs, "rel_gap": rel, "F": F, "check_every_epochs": check_every, "gap_evaluations": checks}


def run_async(args) -> int:
    """Asynchronous variant vs synchronous steps on one instance, per tau:
    picks/s, and time to a certified 1e-6 gap from x = 0."""
    import numpy as np
    import torch

    import paper_1212_0873_amd as pc
    from workloads import make_config

    torch.cuda.set_device(0)
    inst = make_config(args.config, dtype=args.dtype)
    A = inst.A
    res = {}
    with pc.Problem(A, inst.b, inst.lam, 1024, seed=0) as p:
        for tau in (1024, 65536, 1_000_000):
            tau = min(tau, A.n)
            p.set_option("tau", tau)
            p.set_option("refresh_every", -(-A.n // tau))
            p.set_x(np.zeros(A.n), k=0)
            sync = time_to_gap(p, 1e-6, args.gap_seconds, gap_check(args))
            r_tau = {"beta": p.info()["beta"], "sync_time_to_gap": sync}
            for label, reads, rounds in (("default", -1, 4), ("cached_r1", 0, 1), ("cached_r4", 0, 4),
                                         ("acquire", 1, 0), ("atomic", 2, 0)):
                p.set_option("async_reads", reads)
                p.set_option("async_rounds", rounds)
                p.set_x(np.zeros(A.n), k=0)
                p.step_async(1)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                p.step_async(2)
                torch.cuda.synchronize()
                rate = 2 * A.n / (time.perf_counter() - t0)
                p.set_x(np.zeros(A.n), k=0)
                r_tau[label] = {"picks_per_s": rate, "processors": p.info()["async_processors"],
                                "time_to_gap": async_time_to_gap(p, 1e-6, args.gap_seconds, gap_check(args))}
                print(f"[bench] async tau={tau} {label}: {r_tau[label]}", file=sys.stderr, flush=True)
            res[str(tau)] = r_tau
    out = {"metric": METRIC, "mode": "async", "n_gpus": 1, "dtype": args.dtype, "data": "synthetic",
           "config": {"workload": WORKLOAD_NAMES[args.config]}, "taus": res}
    print(json.dumps(out), flush=True)
    return 0


def run_models(args) -> int:
    """Other losses on instances shaped like the paper's last two experiments:
    L2-regularised logistic regression (sum_j log(1 + exp(-y_j a_j^T x)) +
    ||x||^2, i.e. l2 = 2) on 19,264,097 examples x 29,890,095 features with 19
    nonzeros per feature (5.7e8 nonzeros, written on the device; labels the
    signs of a planted linear model plus noise), reported as F(x0)/F(x_k) and
    seconds per epoch as in the paper's table; and the SVM dual (box [0, 1])
    on 677,399 examples x 47,236 features with 73 nonzeros per example."""
    import numpy as np
    import torch

    import paper_1212_0873_amd as pc
    from workloads import CSC, biggen, random_csc

    torch.cuda.set_device(0)
    out = {"metric": METRIC, "mode": "models", "n_gpus": 1, "dtype": args.dtype, "data": "synthetic"}
    m_ex, n_feat, d = 19_264_097, 29_890_095, 19
    t0 = time.time()
    A, b, _ = biggen.device_instance(m_ex, n_feat, d, 3_000_000, 0.1, seed=0, dtype=args.dtype)
    y = torch.where(b >= 0, 1.0, -1.0).to(torch.float64)
    del b
    torch.cuda.synchronize()
    print(f"[bench] logistic instance written in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    res = {}
    for tau in (65536, 1 << 20):
        with pc.Problem(A, y, 0.0, tau, seed=0, model=dict(loss="logistic", l2=2.0)) as p:
            spe = -(-n_feat // tau)
            F0, _ = p.objective()
            rows = []
            for epoch in range(1, 4):
                p.set_option("kernel_timing", 1)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                p.step(spe)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t1
                kt = {k: p.kernel_time(k)[1] for k in ("gather", "scatter", "refresh")}
                p.set_option("kernel_timing", 0)
                F, _ = p.objective()
                rows.append({"epoch": epoch, "F0_over_F": F0 / F, "seconds": dt, "updates_per_s": spe * tau / dt,
                             "kernel_ms": kt})
            res[str(tau)] = {"beta": p.info()["beta"], "omega": p.info()["omega"], "F0": F0, "epochs": rows}
            print(f"[bench] logistic tau={tau}: {res[str(tau)]}", file=sys.stderr, flush=True)
    out["logistic_l2"] = {"workload": "logistic_19264097x29890095_d19", "nnz": n_feat * d, "tau": res}
    del A, y
    torch.cuda.empty_cache()

    rng = np.random.default_rng(0)
    d_feat, n_ex, per = 47_236, 677_399, 73
    X = random_csc(d_feat, n_ex, per, rng, normalize=False, dtype="f64")
    w = rng.standard_normal(d_feat)
    import scipy.sparse as sp
    S = sp.csc_matrix((X.values, X.row_idx, X.col_ptr), shape=(d_feat, n_ex))
    lab = np.where(S.T @ w + 0.5 * rng.standard_normal(n_ex) >= 0, 1.0, -1.0)
    vals = (X.values * np.repeat(lab, np.diff(X.col_ptr))).astype(np.float32)
    cols = CSC(m=d_feat, n=n_ex, col_ptr=X.col_ptr, row_idx=X.row_idx, values=vals)
    del X, S
    lam = 1e-3
    res = {}
    for tau in (4096, 65536):
        model = dict(loss="square", scale=1.0 / (lam * n_ex * n_ex), linear=-1.0 / n_ex, lower=0.0, upper=1.0)
        with pc.Problem(cols, np.zeros(d_feat), 0.0, tau, seed=0, model=model) as p:
            spe = -(-n_ex // tau)
            rows = []
            for epoch in range(1, 6):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                p.step(spe)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t1
                F, _ = p.objective()
                rows.append({"epoch": epoch, "dual_objective": -F, "seconds": dt,
                             "updates_per_s": spe * tau / dt})
            res[str(tau)] = {"beta": p.info()["beta"], "omega": p.info()["omega"], "epochs": rows}
            print(f"[bench] svm dual tau={tau}: {res[str(tau)]}", file=sys.stderr, flush=True)
    out["svm_dual"] = {"workload": "svm_dual_677399x47236_d73", "lambda": lam, "tau": res}
    print(json.dumps(out), flush=True)
    return 0


def run_path(args) -> int:
    """A 64-point regularisation path on one instance of the batched
    workload's largest size (n = 1e6 columns, m = 2e5, 10 nonzeros per
    column): lambda_j = 0.5 * 0.01^(j/63) * ||A^T b||_inf, each solved to a
    certified 1e-6 gap, (a) warm-started in order, (b) cold from x = 0 one
    after the other, (c) cold, all 64 as one batch of copies of (A, b)."""
    import numpy as np
    import torch

    import paper_1212_0873_amd as pc
    from workloads import planted_lasso, random_csc

    torch.cuda.set_device(0)
    rng = np.random.default_rng(0)
    n, m, d = 1_000_000, 200_000, 10
    A = random_csc(m, n, d, rng, normalize=False, dtype=args.dtype)
    inst = planted_lasso(A, n // 100, 0.01, 0.5, rng)
    tau = 4096
    lam_max = inst.lam / 0.5
    lams = [0.5 * 0.01 ** (j / 63) * lam_max for j in range(64)]
    out = {"metric": METRIC, "mode": "path", "n_gpus": 1, "dtype": args.dtype, "data": "synthetic",
           "config": {"workload": "lasso_path_2e5x1e6_d10", "points": 64, "tau": tau, "target_rel_gap": 1e-6}}
    with pc.Problem(inst.A, inst.b, lams[0], tau, seed=0) as p:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        path = p.solve_path(lams, rel_gap=1e-6, keep_x=False)
        torch.cuda.synchronize()
        out["warm_seconds"] = time.perf_counter() - t0
        out["warm_epochs"] = sum(st["epochs"] for st in path)
        out["warm_converged"] = all(st["converged"] for st in path)
    print(f"[bench] warm path {out['warm_seconds']:.2f}s", file=sys.stderr, flush=True)
    cold_t = 0.0
    cold_e = 0
    with pc.Problem(inst.A, inst.b, lams[0], tau, seed=0) as p:
        for lam in lams:
            p.set_option("lambda", lam)
            p.set_x(np.zeros(n), k=0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = p.solve(rel_gap=1e-6, check_every=1)
            torch.cuda.synchronize()
            cold_t += time.perf_counter() - t0
            cold_e += st["epochs"]
    out["cold_seconds"] = cold_t
    out["cold_epochs"] = cold_e
    print(f"[bench] cold path {cold_t:.2f}s", file=sys.stderr, flush=True)
    with pc.Batch([(inst.A, inst.b, lam, tau) for lam in lams], seed=0) as B:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = B.solve(rel_gap=1e-6, check_every_steps=64)
        torch.cuda.synchronize()
        out["batched_cold_seconds"] = time.perf_counter() - t0
        out["batched_converged"] = st["converged"]
    out["warm_speedup_vs_cold"] = out["cold_seconds"] / out["warm_seconds"]
    print(json.dumps(out), flush=True)
    return 0


def run_group(args) -> int:
    """Group LASSO on the 1e6 x 1e7 instance with blocks of 4 consecutive
    columns (2.5e6 blocks): set-up time (block Gram matrices and their largest
    eigenvalues), coordinate updates/s and time to a certified 1e-6 gap at
    tau = 2.5e5 blocks (1e6 coordinates per step), lambda = 0.05 max_i
    ||A_i^T b||."""
    import numpy as np
    import scipy.sparse as sp
    import torch

    import paper_1212_0873_amd as pc
    from workloads import make_config

    torch.cuda.set_device(0)
    inst = make_config("lasso_1e6x1e7", dtype=args.dtype)
    A = inst.A
    size = 4
    bp = np.arange(0, A.n + 1, size, dtype=np.int64)
    S = sp.csc_matrix((A.values_f64(), A.row_idx, A.col_ptr), shape=(A.m, A.n))
    atb = S.T @ inst.b
    lam = 0.05 * float(np.max(np.sqrt(np.add.reduceat(atb * atb, bp[:-1]))))
    del S, atb
    tau = 250_000
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p = pc.Problem(A, inst.b, lam, tau, seed=0, blocks=bp)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    inf = p.info()
    spe = -(-inf["nblocks"] // tau)
    p.step(10)
    p.set_option("kernel_timing", 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.step(200)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ng, gms = p.kernel_time("gather")
    ns, sms = p.kernel_time("scatter")
    p.set_option("kernel_timing", 0)
    p.set_x(np.zeros(A.n), k=0)
    ttg = time_to_gap(p, 1e-6, args.gap_seconds, gap_check(args))
    p.close()
    out = {"metric": METRIC, "mode": "group", "n_gpus": 1, "dtype": args.dtype, "data": "synthetic",
           "config": {"workload": "group_lasso_1e6x1e7_d20_blocks4", "nblocks": inf["nblocks"], "tau_blocks": tau,
                      "omega_blocks": inf["omega"], "beta": inf["beta"], "lambda": lam},
           "create_seconds": create_s, "coord_updates_per_s": 200 * tau * size / dt, "ms_per_step": dt / 200 * 1e3,
           "gather_avg_us": gms / max(ng, 1) * 1e3, "scatter_avg_us": sms / max(ns, 1) * 1e3, "time_to_gap": ttg}
    print(json.dumps(out), flush=True)
    return 0


def run_adjoint(args) -> int:
    """The differentiation pattern on the 1e5 x 1e6 training matrix (10
    nonzeros per column, tau = 4096): forward solve from x = 0 to a certified
    1e-6 gap, then d loss/d b and d loss/d lambda of the validation loss
    ||V (x - x*)||^2 (V: 2e4 x 1e6, 10 nonzeros per column) through the
    solution by pcdm_grad_backward; forward and adjoint wall times (HIP
    synchronised), float32 and float64 values."""
    import numpy as np
    import scipy.sparse as sp
    import torch

    import paper_1212_0873_amd as pc
    from workloads import make_config, random_csc

    torch.cuda.set_device(0)
    res = {}
    for dtype in ("f32", "f64"):
        inst = make_config("train_1e5x1e6", dtype=dtype, tau=4096)
        rng = np.random.default_rng(3)
        Vc = random_csc(20000, inst.A.n, 10, rng, normalize=False)
        V = sp.csc_matrix((Vc.values_f64(), Vc.row_idx, Vc.col_ptr), shape=(Vc.m, Vc.n))
        with pc.Problem(inst.A, inst.b, inst.lam, 4096, seed=2) as p:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = p.solve(rel_gap=1e-6)
            torch.cuda.synchronize()
            t_fwd = time.perf_counter() - t0
            x = p.get_x()
            e = V @ (x - inst.xstar)
            g = torch.from_numpy(2.0 * (V.T @ e)).cuda()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            converged = True
            try:
                db, dl = p.grad_backward(g)
            except pc.PCDMError:
                converged = False
                dl = None
            torch.cuda.synchronize()
            t_adj = time.perf_counter() - t1
        res[dtype] = {"forward_seconds": t_fwd, "forward_epochs": st["epochs"], "forward_rel_gap": st["rel_gap"],
                      "support": int(np.count_nonzero(x)), "adjoint_seconds": t_adj,
                      "adjoint_converged": converged, "adjoint_over_forward": t_adj / t_fwd,
                      "dL_dlambda": dl, "validation_loss": float(e @ e)}
        print(f"[bench] adjoint {dtype}: {res[dtype]}", file=sys.stderr, flush=True)
    out = {"metric": METRIC, "mode": "adjoint", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "train_1e5x1e6_d10", "tau": 4096, "validation": "2e4 x 1e6, d = 10",
                      "forward_target_rel_gap": 1e-6},
           "results": res}
    print(json.dumps(out), flush=True)
    return 0


def steps_to_eps(p, Fstar: float, F0: float, eps: float, chunk: int, limit: int) -> int:
    """PCDM steps until F(x_k) - F* <= eps (F(x_0) - F*), checked every
    `chunk` steps (the count is exact to within one chunk); -1 if `limit`
    steps do not get there."""
    steps = 0
    while steps < limit:
        p.step(chunk)
        steps += chunk
        F, _ = p.objective()
        if F - Fstar <= eps * (F0 - Fstar):
            return steps
    return -1


def run_theory(args) -> int:
    """'Theory versus reality': 0.5||Ax - b||^2 (lambda = 0) with A 3000 x 1000
    holding exactly omega equal nonzeros (ones) in every row and 3 omega in
    every column (random pattern), b ~ N(0, 1), for omega in {5, 10, 50, 100}
    and tau from 1 to 1000.  Steps of PCDM1 with tau-nice sampling until
    F(x_k) - F* <= 1e-6 (F(x_0) - F*), F* from a dense float64 least-squares
    solve; the empirical speedup (steps at tau = 1) / (steps at tau) beside the
    theoretical factor tau / beta.  The paper shows this only as a figure, so
    it is a report (no gate)."""
    import numpy as np
    import scipy.linalg
    import torch

    import paper_1212_0873_amd as pc
    from workloads import biregular_matrix, csc_to_dense

    torch.cuda.set_device(0)
    n, m, eps = 1000, 3000, 1e-6
    taus = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1000]
    rows = []
    t0 = time.perf_counter()
    for omega in (5, 10, 50, 100):
        A = biregular_matrix(m, n, omega, np.random.default_rng(omega))
        b = np.random.default_rng(1000 + omega).standard_normal(m)
        M = csc_to_dense(A)
        xs = scipy.linalg.lstsq(M, b)[0]
        Fstar = 0.5 * float(np.sum((M @ xs - b) ** 2))
        F0 = 0.5 * float(b @ b)
        base = None
        for tau in taus:
            with pc.Problem(A.astype("f64"), b, 0.0, tau, seed=0) as p:
                beta = p.info()["beta"]
                chunk = max(1, -(-n // (8 * tau)))
                k = steps_to_eps(p, Fstar, F0, eps, chunk, 2_000_000)
            if tau == 1:
                base = k
            rows.append({"omega": omega, "tau": tau, "beta": beta, "steps": k, "chunk": chunk,
                         "theory_speedup": tau / beta,
                         "empirical_speedup": (base / k) if (base and k > 0) else None})
            print(f"[bench] omega {omega} tau {tau}: beta {beta:.4f}, {k} steps, theory {tau / beta:.2f}, "
                  f"empirical {rows[-1]['empirical_speedup']}", file=sys.stderr, flush=True)
    out = {"mode": "theory", "unit": "steps to F - F* <= 1e-6 (F(x_0) - F*)", "data": "synthetic",
           "dtype": "f64", "seconds": time.perf_counter() - t0,
           "config": {"m": m, "n": n, "lambda": 0.0, "values": "ones, omega per row, 3 omega per column",
                      "b": "N(0,1)", "sampling": "tau-nice", "seed": 0},
           "parity": "unpinned (the paper prints a figure only)", "results": rows}
    print(json.dumps(out), flush=True)
    return 0

def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--config", default=None, choices=sorted(WORKLOAD_NAMES),
                    help="workload (default: lasso_2e8x5e8 in the single mode, lasso_1e6x1e7 in the "
                         "dtypes, samplings and async modes)")
    ap.add_argument("--tau", type=int, default=None,
                    help="default: 2^20 on lasso_2e8x5e8, 1e6 on the other workloads")
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16", "f64"])
    ap.add_argument("--lanes", type=int, default=0, help="lanes per column (0 = automatic)")
    ap.add_argument("--gather-route", type=int, default=0, choices=[0, 1, 2],
                    help="partial derivatives: 0 automatic, 1 by columns, 2 by rows (option gather_route)")
    ap.add_argument("--scatter-route", type=int, default=0, choices=[0, 1, 2],
                    help="residual scatter: 0 automatic, 1 atomics, 2 row blocks (option scatter_route)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample length")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-gap", action="store_true", help="skip the time-to-gap run")
    ap.add_argument("--gap-seconds", type=float, default=60.0)
    ap.add_argument("--gap-check", default="auto",
                    help='epochs between duality-gap evaluations in the time-to-gap runs, or "auto"')
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for counter scaling)")
    ap.add_argument("--mode", default="single", choices=["single", "batched", "dtypes", "taus", "samplings", "async", "models", "path", "group",
                             "adjoint", "theory"],
                    help="single: one instance (default); batched: the uneven lambda path; "
                         "dtypes: time to gap with float64 / float32 / bf16 values; taus: tau sweep "
                         "on both 1e7-column instances; samplings: nice / independent / binomial / "
                         "masked slots; async: asynchronous variant vs synchronous steps; models: "
                         "logistic regression and the SVM dual; path: warm-started regularisation path; "
                         "group: group LASSO with blocks of 4 columns; adjoint: forward solve and "
                         "d loss/d (b, lambda) on the training matrix; theory: iterations to 1e-6 "
                         "against tau / beta on 3000 x 1000 matrices with omega ones per row")
    ap.add_argument("--count", type=int, default=64, help="problems in the batched mode")
    ap.add_argument("--check-steps", type=int, default=64, help="batched mode: steps between gap checks")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        msg = ("bench.py measures one GPU only: the method's data-parallel step runs on one "
               "MI355X here; multi-GPU sharding is a design note, not a built path")
        if int(os.environ.get("RANK", "0")) == 0:
            print(msg, file=sys.stderr)
        return 2

    from workloads.configs import CONFIGS
    host_modes = ("dtypes", "samplings", "async")
    if args.config is None:
        args.config = "lasso_1e6x1e7" if args.mode in host_modes else "lasso_2e8x5e8"
    if args.tau is None:
        args.tau = 1 << 20 if args.config == "lasso_2e8x5e8" else 1_000_000
    if args.mode in host_modes and CONFIGS[args.config].get("device_gen"):
        print(f"--mode {args.mode} builds its instance on the host; {args.config} is generated on the "
              f"device only (use the single mode)", file=sys.stderr)
        return 2

    if args.mode == "batched":
        return run_batched(args)
    if args.mode == "dtypes":
        return run_dtypes(args)
    if args.mode == "taus":
        return run_taus(args)
    if args.mode == "samplings":
        return run_samplings(args)
    if args.mode == "async":
        return run_async(args)
    if args.mode == "models":
        return run_models(args)
    if args.mode == "path":
        return run_path(args)
    if args.mode == "group":
        return run_group(args)
    if args.mode == "adjoint":
        return run_adjoint(args)
    if args.mode == "theory":
        return run_theory(args)

    import numpy as np
    import torch

    import paper_1212_0873_amd as pc
    from workloads import make_config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev_name = torch.cuda.get_device_name(0)

    copy_gbps = copy_bandwidth_gbps()
    if args.copy_calibration:
        nb = 1 << 30
        src = torch.empty(nb // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nb}), file=sys.stderr, flush=True)
        del src, dst

    from workloads.configs import CONFIGS
    cfg = CONFIGS[args.config]
    t0 = time.time()
    host_thread = None
    host = {}
    if cfg.get("device_gen"):
        # too large to build on the host: written on the device by the
        # counter-based recipe; the host regenerates columns for the oracle
        from workloads import biggen
        if not args.no_cpu:
            if args.dtype == "f64":
                raise SystemExit("the host pass of the 1e10 instance reads float32 / bf16 stored values")
            import threading
            host_thread = threading.Thread(target=big_host_pass, args=(cfg, args.dtype, host), daemon=True)
            host_thread.start()
        Ad, bd, _ = biggen.device_instance(cfg["m"], cfg["n"], cfg["d"], cfg["xstar_nnz"], cfg["noise_std"],
                                           seed=0, dtype=args.dtype)
        torch.cuda.synchronize()
        A = types.SimpleNamespace(m=cfg["m"], n=cfg["n"], nnz=cfg["n"] * cfg["d"])
        tau = min(args.tau, A.n)
        gen_s = time.time() - t0
        p = pc.Problem(Ad, bd, 0.0, tau, seed=0)
        lam = cfg["lam_factor"] * p.info()["atb_inf"]
        p.set_option("lambda", lam)
        del Ad, bd
        torch.cuda.empty_cache()
        inst = types.SimpleNamespace(lam=lam)
        if host_thread is not None:
            # the host pass (all CPU threads) ends before anything is timed
            while host_thread.is_alive():
                host_thread.join(timeout=20)
                print(f"[bench] host pass over the regenerated columns: {host.get('progress', 0):.0%} "
                      f"at {time.time() - t0:.0f}s", file=sys.stderr, flush=True)
            if "error" in host:
                raise host["error"]
    else:
        inst = make_config(args.config, dtype=args.dtype, tau=args.tau)
        A = inst.A
        tau = min(args.tau, A.n)
        gen_s = time.time() - t0
        p = pc.Problem(A, inst.b, inst.lam, tau, seed=0)
    print(f"[bench] generated {args.config}: m={A.m} n={A.n} nnz={A.nnz} in {gen_s:.1f}s "
          f"(create done at {time.time() - t0:.1f}s)", file=sys.stderr, flush=True)

    if args.lanes:
        p.set_option("lanes_per_column", args.lanes)
    if args.gather_route:
        p.set_option("gather_route", args.gather_route)
    if args.scatter_route:
        p.set_option("scatter_route", args.scatter_route)
    info = p.info()
    spe = info["refresh_every"]
    s_val = {"f32": 4, "bf16": 2, "f64": 8}[args.dtype]
    d_avg = A.nnz / A.n
    b_gather, b_scatter = algorithmic_bytes(d_avg, s_val)

    # warmup, then exactly K timed steps
    p.step(args.warmup)
    torch.cuda.synchronize()
    x_warm = p.get_x_tensor()  # to replay the same steps below
    p.set_option("reset_counters", 1)
    p.set_option("kernel_timing", 1)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    p.step(args.steps)
    torch.cuda.synchronize()
    t_el = time.perf_counter() - t_start
    info2 = p.info()
    ng, gms = p.kernel_time("gather")
    ns, sms = p.kernel_time("scatter")
    nr, rms = p.kernel_time("refresh")
    p.set_option("kernel_timing", 0)
    updates = tau * args.steps
    nz = info2["nonzero_updates"]
    value = updates / t_el
    # the same K steps again (from the same x and step counter) without
    # per-kernel events, so that runs of steps are replayed from HIP graphs as
    # in a solve (the events above turn the replay off and add a few
    # microseconds per launch); then the timed window's end state is restored
    x_end = p.get_x_tensor()
    t_reps = []
    for _ in range(5):
        p.set_x(x_warm, k=args.warmup)
        torch.cuda.synchronize()
        t_g = time.perf_counter()
        p.step(args.steps)
        torch.cuda.synchronize()
        t_reps.append(time.perf_counter() - t_g)
    t_graph = sorted(t_reps)[len(t_reps) // 2]
    p.set_x(x_end, k=args.warmup + args.steps)
    del x_warm, x_end
    gather_avg_s = gms / 1e3 / max(ng, 1)
    gather_bytes = b_gather * tau
    achieved = gather_bytes / gather_avg_s / 1e9
    step_alg_bytes = b_gather * updates + b_scatter * nz
    workload = WORKLOAD_NAMES[args.config]
    # the partial derivatives by rows take three launches per step (their
    # summed time is the "gather" clock); their counters sit in files of their own
    by_rows = info["gather_route"] == 2
    pmc_name = "gather_by_rows" if by_rows else "gather"
    traffic = read_traffic(pmc_name, args.config, args.dtype, tau)
    ceiling = random_gather_ceiling(A.m)
    l2c = read_l2_counters(pmc_name, args.config, args.dtype, tau)
    l2 = {"random_read_ceiling": ceiling, "requests_per_launch": None, "hit_rate": None,
          "request_rate_per_s": None, "frac_of_random_ceiling": None}
    if l2c:
        rate = l2c["tcc_req_per_launch"] / gather_avg_s
        l2.update({"requests_per_launch": l2c["tcc_req_per_launch"],
                   "hit_rate": l2c["tcc_hit_per_launch"] / l2c["tcc_req_per_launch"],
                   "request_rate_per_s": rate})
        if ceiling:
            l2["frac_of_random_ceiling"] = rate / (ceiling["reads_per_s"] * l2c["calib_tcc_req_per_read"])

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "coord updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": workload, "m": A.m, "n": A.n, "nnz": A.nnz, "tau": tau,
                   "omega": info["omega"], "beta": info["beta"], "lambda": inst.lam,
                   "lanes_per_column": info["lanes_per_column"], "refresh_every": spe,
                   "gather_route": {1: "columns", 2: "rows"}[info["gather_route"]],
                   "scatter_route": {1: "atomics", 2: "row blocks"}[info["scatter_route"]],
                   "device": dev_name},
        "roofline": {"bound": "hbm", "kernel": "k_bin + k_bin_dot + k_bin_prox" if by_rows else "k_gather",
                     "achieved": achieved,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic, "alg_bytes_per_update": b_gather,
                     "launches": ng, "avg_launch_us": gather_avg_s * 1e6,
                     "measured_gbps": (traffic / gather_avg_s / 1e9) if traffic else None,
                     "measured_frac": (traffic / gather_avg_s / 1e9 / HBM_PEAK_GBPS) if traffic else None,
                     "measured_over_algorithmic": (traffic / gather_bytes) if traffic else None,
                     "step_achieved": step_alg_bytes / t_el / 1e9,
                     "step_frac": step_alg_bytes / t_el / 1e9 / HBM_PEAK_GBPS,
                     "copy_gbps": copy_gbps,
                     "frac_of_copy": achieved / copy_gbps,
                     "measured_frac_of_copy": (traffic / gather_avg_s / 1e9 / copy_gbps) if traffic else None,
                     "l2_requests": l2},
        "scatter_atomics": {"atomics": nz * d_avg, "per_s": nz * d_avg / max(sms / 1e3, 1e-12),
                            "frac_of_random_atomic_ceiling":
                                (nz * d_avg / max(sms / 1e3, 1e-12) / ceiling["atomics_per_s"]) if ceiling else None,
                            "note": "nonzero updates x mean column length over the summed scatter launch time"},
        "graph_replay": {"steps": args.steps, "ms_per_step": t_graph * 1e3 / args.steps,
                         "value": updates / t_graph,
                         "ms_per_step_runs": [t * 1e3 / args.steps for t in t_reps],
                         "note": "the same K steps from the same state, timed without per-kernel events "
                                 "(HIP graph replay); median of 5 runs"},
        "gpu_clocks": gpu_clocks(),
        "hbm_gbps_algorithmic_step": step_alg_bytes / t_el / 1e9,
        "nonzero_update_fraction": nz / updates,
        "kernel_ms": {"gather": gms, "scatter": sms, "refresh": rms,
                      "launches": {"gather": ng, "scatter": ns, "refresh": nr}},
    }

    if not args.no_gap:
        # time to a certified 1e-6 relative gap from x = 0 (float64 duality gap)
        p.set_x(np.zeros(A.n), k=0)
        out["time_to_gap"] = time_to_gap(p, 1e-6, args.gap_seconds, gap_check(args))
        print(f"[bench] {out['time_to_gap']}", file=sys.stderr, flush=True)
    p.close()
    del p

    if not args.no_cpu and host_thread is not None:
        out["cpu_baseline"] = big_cpu_baseline(cfg, args.dtype, host, tau, args.cpu_seconds)
    elif not args.no_cpu:
        import oracle
        ref = oracle.Solver(A, inst.b, inst.lam, tau=tau, seed=0)
        steps = 0
        t_c = time.perf_counter()
        while time.perf_counter() - t_c < args.cpu_seconds:
            ref.step(1)
            steps += 1
        tc = time.perf_counter() - t_c
        out["cpu_baseline"] = {"value": steps * tau / tc, "unit": "coord updates/s", "cores": 1,
                               "kind": "oracle", "cpu_model": cpu_model(), "host_threads_available": os.cpu_count(),
                               "sample": f"{steps} steps of tau={tau} from x=0 on the same matrix "
                                         f"({steps * tau} updates, {tc:.1f} s, float64, one thread)"}
        if A.nnz <= 2_000_000 and not args.no_gap:
            out["cpu_baseline"]["time_to_gap"] = oracle_time_to_gap(A, inst.b, inst.lam, tau, 1e-6,
                                                                    args.gap_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
