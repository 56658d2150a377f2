"""Python face of the C ABI: same operations, argument marshalling only.

Every step of the method runs in the HIP library; this module converts numpy
arrays or torch tensors into pointers and sizes, passes torch's current HIP
stream, and raises :class:`PCDMError` on a negative status.
"""

from __future__ import annotations

import ctypes
import math
from typing import Optional

import numpy as np

from ._lib import (PCDM_BF16, PCDM_F32, PCDM_F64, PCDMError, check, load, pcdm_csc, pcdm_model,  # noqa: F401
                   pcdm_info)

_NP_DTYPE = {np.dtype(np.float32): PCDM_F32, np.dtype(np.float64): PCDM_F64, np.dtype(np.uint16): PCDM_BF16}


def _torch():
    import torch
    return torch


def current_stream() -> Optional[int]:
    """Raw hipStream_t of torch's current stream (None when no GPU)."""
    try:
        torch = _torch()
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


def _ptr(a) -> int:
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


class Problem:
    """One LASSO problem held by the library (``pcdm_create`` .. ``pcdm_destroy``).

    ``A`` is a CSC with host numpy arrays (``workloads.CSC``: float64, float32
    or bf16 bits as uint16) or an object with attributes m, n, col_ptr,
    row_idx, values holding CUDA torch tensors (float64, float32 or bfloat16);
    ``b`` is float64 in the same place.
    """

    def __init__(self, A, b, lam: float, tau: int, seed: int = 0, model: Optional[dict] = None,
                 blocks=None):
        """``model`` (optional) selects another loss / regulariser
        (``pcdm_create_model``): keys loss ('square', 'logistic', 'sqhinge'),
        scale, l2, linear, lower, upper; ``lam`` is the l1 weight and ``b``
        the targets or +-1 labels.  ``blocks`` (optional, int64 [nblocks+1]
        column boundaries) makes a group LASSO (``pcdm_create_group``) whose
        tau counts blocks."""
        self._lib = load()
        self._h = ctypes.c_void_p()
        on_dev = not isinstance(A.values, np.ndarray)
        if on_dev:
            torch = _torch()
            tmap = {torch.float32: PCDM_F32, torch.float64: PCDM_F64, torch.bfloat16: PCDM_BF16}
            vals = A.values.contiguous()
            cp = A.col_ptr.to(torch.int64).contiguous()
            ri = A.row_idx.to(torch.int32).contiguous()
            bb = b.to(torch.float64).contiguous()
            dtype = tmap[vals.dtype]
            nnz = int(vals.numel())
        else:
            vals = np.ascontiguousarray(A.values)
            cp = np.ascontiguousarray(A.col_ptr, dtype=np.int64)
            ri = np.ascontiguousarray(A.row_idx, dtype=np.int32)
            bb = np.ascontiguousarray(b, dtype=np.float64)
            dtype = _NP_DTYPE[vals.dtype]
            nnz = int(vals.size)
        self._keep = (vals, cp, ri, bb)
        desc = pcdm_csc(int(A.m), int(A.n), nnz, _ptr(cp), _ptr(ri), _ptr(vals), dtype, int(on_dev))
        if on_dev:
            _torch().cuda.current_stream().synchronize()
        if blocks is not None:
            if model is not None:
                raise ValueError("a block problem is a group LASSO: no model")
            if on_dev:
                bpk = blocks.to(_torch().int64).contiguous()
                nblk = int(bpk.numel()) - 1
            else:
                bpk = np.ascontiguousarray(blocks, dtype=np.int64)
                nblk = int(bpk.size) - 1
            check(self._lib.pcdm_create_group(ctypes.byref(desc), _ptr(bb), float(lam), _ptr(bpk), nblk, int(tau),
                                              int(seed) & (2**64 - 1), ctypes.byref(self._h)))
        elif model is None:
            check(self._lib.pcdm_create(ctypes.byref(desc), _ptr(bb), float(lam), int(tau),
                                        int(seed) & (2**64 - 1), ctypes.byref(self._h)))
        else:
            unknown = set(model) - {"loss", "scale", "l2", "linear", "lower", "upper"}
            if unknown:
                raise ValueError(f"unknown model keys {sorted(unknown)}")
            mdl = pcdm_model(LOSSES[model.get("loss", "square")], 0, float(model.get("scale", 1.0)), float(lam),
                             float(model.get("l2", 0.0)), float(model.get("linear", 0.0)),
                             float(model.get("lower", -np.inf)), float(model.get("upper", np.inf)))
            check(self._lib.pcdm_create_model(ctypes.byref(desc), _ptr(bb), ctypes.byref(mdl), int(tau),
                                              int(seed) & (2**64 - 1), ctypes.byref(self._h)))
        self._keep = None
        self.m, self.n, self.dtype = int(A.m), int(A.n), dtype

    # -- lifetime -----------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            check(self._lib.pcdm_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- method ---------------------------------------------------------------
    def step(self, nsteps: int = 1, stream: Optional[int] = None) -> None:
        s = current_stream() if stream is None else stream
        check(self._lib.pcdm_step(self._h, int(nsteps), s))

    def objective(self, gap: bool = False, stream: Optional[int] = None):
        """(F, gap or None), both computed in float64 on the device."""
        s = current_stream() if stream is None else stream
        F = ctypes.c_double()
        G = ctypes.c_double()
        check(self._lib.pcdm_objective(self._h, ctypes.byref(F), ctypes.byref(G) if gap else None, s))
        return F.value, (G.value if gap else None)

    def set_option(self, key: str, value: float) -> None:
        check(self._lib.pcdm_set_option(self._h, key.encode(), float(value)))

    def step_async(self, epochs: int = 1, picks_per_epoch: Optional[int] = None) -> None:
        """Epochs of the asynchronous variant: each one launch of n picks
        (or ``picks_per_epoch``) followed by the float64 refresh."""
        picks = self.n if picks_per_epoch is None else int(picks_per_epoch)
        for _ in range(int(epochs)):
            check(self._lib.pcdm_step_async(self._h, picks, current_stream()))

    def set_sampling(self, sampling: str, pb: float = 1.0) -> None:
        """'nice', 'independent' or 'binomial' (availability pb); beta follows
        the sampling unless an explicit beta was set."""
        if sampling == "binomial":
            self.set_option("binomial_p", pb)
        self.set_option("sampling", SAMPLINGS[sampling])

    def set_slot_mask(self, mask) -> None:
        """Drop mask over slots (0 = processor down); None removes it."""
        if mask is None:
            check(self._lib.pcdm_set_slot_mask(self._h, None, 0, 0, current_stream()))
            return
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        check(self._lib.pcdm_set_slot_mask(self._h, m.ctypes.data_as(ctypes.c_void_p), int(m.size), 0,
                                           current_stream()))

    def info(self) -> dict:
        inf = pcdm_info()
        check(self._lib.pcdm_get_info(self._h, ctypes.byref(inf)))
        d = {f: getattr(inf, f) for f, _ in pcdm_info._fields_}
        d["lambda"] = d.pop("lambda_")
        return d

    def autotune(self, steps_per_candidate: int = 5) -> dict:
        """Time every supported schedule for a few real steps and keep the fastest."""
        check(self._lib.pcdm_autotune(self._h, int(steps_per_candidate), current_stream()))
        inf = self.info()
        return {"lanes_per_column": inf["lanes_per_column"], "chunks_per_lane": inf["chunks_per_lane"],
                "narrow_below": inf["narrow_below"]}

    def kernel_time(self, kernel: str):
        """(launches, total milliseconds) of one kernel kind while timing is on."""
        n = ctypes.c_int64()
        t = ctypes.c_double()
        check(self._lib.pcdm_kernel_time(self._h, kernel.encode(), ctypes.byref(n), ctypes.byref(t)))
        return n.value, t.value

    # -- state ------------------------------------------------------------------
    def get_x(self, dtype=np.float64) -> np.ndarray:
        out = np.empty(self.n, dtype=dtype)
        code = PCDM_F64 if np.dtype(dtype) == np.float64 else PCDM_F32
        check(self._lib.pcdm_get_x(self._h, out.ctypes.data, code, 0, current_stream()))
        return out

    def get_x_tensor(self, dtype=None):
        torch = _torch()
        dtype = dtype or torch.float64
        out = torch.empty(self.n, dtype=dtype, device="cuda")
        code = PCDM_F64 if dtype == torch.float64 else PCDM_F32
        check(self._lib.pcdm_get_x(self._h, out.data_ptr(), code, 1, current_stream()))
        return out

    def set_x(self, x, k: int = 0) -> None:
        if isinstance(x, np.ndarray):
            xx = np.ascontiguousarray(x)
            code = PCDM_F64 if xx.dtype == np.float64 else PCDM_F32
            if xx.dtype not in (np.float64, np.float32):
                xx = xx.astype(np.float64)
                code = PCDM_F64
            check(self._lib.pcdm_set_x(self._h, xx.ctypes.data, code, 0, int(k), current_stream()))
        else:
            torch = _torch()
            xx = x.contiguous()
            code = PCDM_F64 if xx.dtype == torch.float64 else PCDM_F32
            check(self._lib.pcdm_set_x(self._h, xx.data_ptr(), code, 1, int(k), current_stream()))

    def get_residual(self) -> np.ndarray:
        out = np.empty(self.m, dtype=np.float64)
        check(self._lib.pcdm_get_residual(self._h, out.ctypes.data, 0, current_stream()))
        return out

    def grad_backward(self, dL_dx):
        """(dL/db, dL/dlambda) through the current iterate, taken as the
        solution.  dL_dx: numpy array (result on the host) or CUDA tensor
        (result a CUDA tensor)."""
        dl = ctypes.c_double()
        if isinstance(dL_dx, np.ndarray):
            g = np.ascontiguousarray(dL_dx, dtype=np.float64)
            out = np.empty(self.m, dtype=np.float64)
            check(self._lib.pcdm_grad_backward(self._h, g.ctypes.data, out.ctypes.data, ctypes.byref(dl), 0,
                                               current_stream()))
        else:
            torch = _torch()
            g = dL_dx.to(torch.float64).contiguous()
            out = torch.empty(self.m, dtype=torch.float64, device=g.device)
            check(self._lib.pcdm_grad_backward(self._h, g.data_ptr(), out.data_ptr(), ctypes.byref(dl), 1,
                                               current_stream()))
        return out, dl.value

    def grad_backward_noalloc(self, dL_dx, out=None):
        """grad_backward through ``pcdm_grad_backward_noalloc``: dL_dx a CUDA
        tensor, dL/db written into ``out`` (a float64 CUDA tensor of m, or a
        new one) with no device allocation inside the library."""
        torch = _torch()
        g = dL_dx if dL_dx.dtype == torch.float64 and dL_dx.is_contiguous() else dL_dx.to(torch.float64).contiguous()
        if out is None:
            out = torch.empty(self.m, dtype=torch.float64, device=g.device)
        if out.dtype != torch.float64 or not out.is_contiguous() or out.numel() != self.m:
            raise ValueError("out must be a contiguous float64 tensor of m entries")
        dl = ctypes.c_double()
        check(self._lib.pcdm_grad_backward_noalloc(self._h, g.data_ptr(), out.data_ptr(), ctypes.byref(dl),
                                                   current_stream()))
        return out, dl.value

    def set_rhs(self, b) -> None:
        """Replace b (warm start: x and k are kept)."""
        if isinstance(b, np.ndarray):
            bb = np.ascontiguousarray(b, dtype=np.float64)
            check(self._lib.pcdm_set_rhs(self._h, bb.ctypes.data, 0, current_stream()))
        else:
            bb = b.to(_torch().float64).contiguous()
            check(self._lib.pcdm_set_rhs(self._h, bb.data_ptr(), 1, current_stream()))

    def solve(self, rel_gap: float = 1e-6, check_every="auto", max_epochs: int = 100000,
              max_seconds: Optional[float] = None) -> dict:
        """Step until the certified duality gap (F - D)/D <= rel_gap; returns
        {"epochs", "F", "gap", "rel_gap", "converged", "checks", "seconds",
        "evaluations": [(epochs, rel_gap, seconds of the evaluation), ...]}.

        ``check_every``: epochs between gap evaluations, or "auto" for
        :func:`next_check_interval` on the measured cost of the last
        evaluation and of the epochs before it.  ``max_seconds`` bounds the
        wall time (checked at evaluations)."""
        import time
        auto = isinstance(check_every, str) and check_every == "auto"
        interval = 1 if auto else int(check_every)
        if interval < 1:
            raise ValueError("check_every must be >= 1 or 'auto'")
        inf = self.info()
        spe = -(-(inf["nblocks"] or self.n) // inf["tau"])  # one epoch: every coordinate or block once
        sync = _torch().cuda.current_stream().synchronize if auto else (lambda: None)
        epochs = checks = 0
        F = gap = None
        rel = float("inf")
        last = None  # (epochs, rel_gap) of the previous evaluation
        evals = []
        sync()
        t0 = t_prev = time.perf_counter()
        while epochs < max_epochs:
            n_ep = min(interval, max_epochs - epochs)
            self.step(n_ep * spe)
            epochs += n_ep
            sync()
            t_mid = time.perf_counter()
            F, gap = self.objective(gap=True)
            checks += 1
            t_end = time.perf_counter()
            D = F - gap
            rel = gap / max(abs(D), 1e-300)
            evals.append((epochs, rel, t_end - t_mid))
            if rel <= rel_gap or (max_seconds is not None and t_end - t0 >= max_seconds):
                break
            if auto:
                trend = (last, (epochs, rel)) if last is not None else None
                interval = next_check_interval(t_end - t_mid, (t_mid - t_prev) / n_ep, epochs,
                                               trend=trend, target=rel_gap)
                last = (epochs, rel)
            t_prev = t_end
        return {"epochs": epochs, "F": F, "gap": gap, "rel_gap": rel, "converged": rel <= rel_gap,
                "checks": checks, "seconds": time.perf_counter() - t0, "evaluations": evals}

    def solve_path(self, lambdas, rel_gap: float = 1e-6, check_every: int = 1, max_epochs: int = 100000,
                   keep_x: bool = True) -> list:
        """Warm-started regularisation path: for each lambda in the given order
        (largest first is the usual order) set lambda and step on from the
        previous solution until the certified gap (F - D)/D <= rel_gap (no
        step when the warm start already meets it).  One dict per lambda:
        lambda, epochs, F, gap, rel_gap, converged and (keep_x) x."""
        out = []
        for lam in lambdas:
            self.set_option("lambda", float(lam))
            F, gap = self.objective(gap=True)
            rel = gap / max(abs(F - gap), 1e-300)
            st = {"epochs": 0, "F": F, "gap": gap, "rel_gap": rel, "converged": rel <= rel_gap}
            if not st["converged"]:
                st = self.solve(rel_gap, check_every, max_epochs)
            st["lambda"] = float(lam)
            if keep_x:
                st["x"] = self.get_x()
            out.append(st)
        return out


def next_check_interval(check_seconds: float, epoch_seconds: float, epochs_done: int = 0,
                        share: float = 0.1, cap: int = 16, trend=None, target: float = 0.0) -> int:
    """Epochs until the next duality-gap evaluation, between 1 and ``cap``.

    Checking every I epochs costs c/I per epoch (c: one evaluation, e: one
    epoch) and runs on average I/2 epochs past the first one that meets the
    target; with about as many epochs left as done (E), I = sqrt(2 E c / e)
    balances the two.  While E is small that rule would evaluate often, and an
    evaluation needs max_i |a_i^T r|: a pass over all of A costing about an
    epoch while many coordinates move, far less once the iterate settles (the
    bounded route).  So the interval is also at least what keeps the last
    evaluation near ``share`` of the stepping time: coarse early, every epoch
    near the solution when evaluations are cheap there.  ``trend`` =
    ((epochs, rel_gap) of the previous evaluation, (epochs, rel_gap) of the
    last): when the gap fell, the interval is at most 0.8 of the epochs its
    geometric rate needs to reach ``target``, so that a coarse interval does
    not run far past the target."""
    if not (epoch_seconds > 0.0) or not (check_seconds >= 0.0):
        return 1
    by_share = -(-check_seconds // (share * epoch_seconds))
    by_overshoot = round((2.0 * max(epochs_done, 0) * check_seconds / epoch_seconds) ** 0.5)
    interval = int(max(1, min(cap, max(by_share, by_overshoot))))
    if trend is not None and target > 0.0:
        (e0, g0), (e1, g1) = trend
        if e1 > e0 and 0.0 < g1 < g0 and g1 > target:
            rate = math.log(g1 / g0) / (e1 - e0)  # < 0: log-gap per epoch
            need = math.log(target / g1) / rate   # epochs to the target at that rate
            interval = max(1, min(interval, math.floor(0.8 * need)))
    return interval


def sample(seed: int, k: int, tau: int, n: int):
    """S_k of the tau-nice sampler as an int32 CUDA tensor (slot order)."""
    torch = _torch()
    out = torch.empty(max(int(tau), 1), dtype=torch.int32, device="cuda")
    check(load().pcdm_sample(int(seed) & (2**64 - 1), int(k), int(tau), int(n), out.data_ptr(),
                             current_stream()))
    return out[: int(tau)]


SAMPLINGS = {"nice": 0, "independent": 1, "binomial": 2}
LOSSES = {"square": 0, "logistic": 1, "sqhinge": 2}


def sample_draw(sampling: str, seed: int, k: int, tau: int, n: int, pb: float = 1.0):
    """Slot draws of a sampling as an int32 CUDA tensor: the tau-nice block, the
    raw independent pick (duplicates kept), or the binomial slot's block / -1
    when unavailable."""
    torch = _torch()
    out = torch.empty(max(int(tau), 1), dtype=torch.int32, device="cuda")
    check(load().pcdm_sample_draw(SAMPLINGS[sampling], float(pb), int(seed) & (2**64 - 1), int(k), int(tau),
                                  int(n), out.data_ptr(), current_stream()))
    return out[: int(tau)]


class Batch:
    """Many independent LASSO problems advanced together (``pcdm_batch_*``).

    ``problems``: a list of (A, b, lam, tau) with host numpy CSCs of one
    dtype.  Problem j samples with key (seed + j, k_j)."""

    def __init__(self, problems, seed: int = 0):
        self._lib = load()
        self._h = ctypes.c_void_p()
        cnt = len(problems)
        descs = (pcdm_csc * cnt)()
        keep = []
        bptr = (ctypes.c_void_p * cnt)()
        lams = (ctypes.c_double * cnt)()
        taus = (ctypes.c_int64 * cnt)()
        for j, (A, b, lam, tau) in enumerate(problems):
            vals = np.ascontiguousarray(A.values)
            cp = np.ascontiguousarray(A.col_ptr, dtype=np.int64)
            ri = np.ascontiguousarray(A.row_idx, dtype=np.int32)
            bb = np.ascontiguousarray(b, dtype=np.float64)
            keep += [vals, cp, ri, bb]
            descs[j] = pcdm_csc(int(A.m), int(A.n), int(vals.size), cp.ctypes.data, ri.ctypes.data,
                                vals.ctypes.data, _NP_DTYPE[vals.dtype], 0)
            bptr[j] = bb.ctypes.data
            lams[j] = float(lam)
            taus[j] = int(tau)
        check(self._lib.pcdm_batch_create(cnt, descs, bptr, lams, taus, int(seed) & (2**64 - 1),
                                          ctypes.byref(self._h)))
        self.count = cnt
        self.ns = [int(p[0].n) for p in problems]

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            check(self._lib.pcdm_batch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def step(self, nsteps: int = 1) -> None:
        check(self._lib.pcdm_batch_step(self._h, int(nsteps), current_stream()))

    def objective(self):
        F = (ctypes.c_double * self.count)()
        G = (ctypes.c_double * self.count)()
        check(self._lib.pcdm_batch_objective(self._h, F, G, current_stream()))
        return np.array(F[:]), np.array(G[:])

    def set_active(self, flags) -> None:
        arr = (ctypes.c_int32 * self.count)(*[1 if f else 0 for f in flags])
        check(self._lib.pcdm_batch_set_active(self._h, arr))

    def get_x(self, j: int) -> np.ndarray:
        out = np.empty(self.ns[j], dtype=np.float64)
        check(self._lib.pcdm_batch_get_x(self._h, int(j), out.ctypes.data, 0, current_stream()))
        return out

    def info(self, j: int) -> dict:
        inf = pcdm_info()
        check(self._lib.pcdm_batch_get_info(self._h, int(j), ctypes.byref(inf)))
        d = {f: getattr(inf, f) for f, _ in pcdm_info._fields_}
        d["lambda"] = d.pop("lambda_")
        return d

    def set_option(self, key: str, value: float) -> None:
        check(self._lib.pcdm_batch_set_option(self._h, key.encode(), float(value)))

    def autotune(self, steps_per_candidate: int = 3) -> dict:
        check(self._lib.pcdm_batch_autotune(self._h, int(steps_per_candidate), current_stream()))
        inf = self.info(0)
        return {"lanes_per_column": inf["lanes_per_column"], "chunks_per_lane": inf["chunks_per_lane"]}

    def solve(self, rel_gap: float = 1e-6, check_every_steps: int = 64, max_steps: int = 10**7) -> dict:
        """Step all problems, retiring each once its certified gap
        (F - D)/D <= rel_gap; returns per-problem steps and gaps."""
        active = [True] * self.count
        done_at = [None] * self.count
        steps = 0
        rel = np.full(self.count, np.inf)
        while any(active) and steps < max_steps:
            self.step(check_every_steps)
            steps += check_every_steps
            F, gap = self.objective()
            rel = gap / np.maximum(np.abs(F - gap), 1e-300)
            changed = False
            for j in range(self.count):
                if active[j] and rel[j] <= rel_gap:
                    active[j] = False
                    done_at[j] = steps
                    changed = True
            if changed:
                self.set_active(active)
        return {"steps": steps, "done_at": done_at, "rel_gap": rel.tolist(), "converged": not any(active)}
