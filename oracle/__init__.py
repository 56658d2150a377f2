"""Float64 CPU oracle for synchronous PCDM1 on the LASSO (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It is a plain serial implementation written from the
paper (Richtarik & Takac, "Parallel Coordinate Descent Methods for Big Data
Optimization"); the numbered facts each function follows are cited in
``pcdm_oracle.c``.  It shares no code with the HIP library.

Functions whose result has no independent pin say "parity unpinned" in their
docstring (none at present: every public function is pinned by a test under
``tests/test_oracle_*.py``).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcdm_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_handle = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_I64P = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_I32P = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_F64P = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_F32P = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_I32MP = np.ctypeslib.ndpointer(dtype=np.int32, flags=("C_CONTIGUOUS", "WRITEABLE"))
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_f64 = ctypes.c_double


def _lib():
    global _handle
    with _lock:
        if _handle is None:
            lib = ctypes.CDLL(build())
            sig = {
                "orc_beta_nice": (_f64, [_i64, _i64, _i64]),
                "orc_beta_uniform": (_f64, [_i64, _i64]),
                "orc_beta_binomial": (_f64, [_i64, _i64, _i64, _f64]),
                "orc_omega": (_i64, [_i64, _i64, _I64P, _I32P, _F64P]),
                "orc_lipschitz": (None, [_i64, _I64P, _F64P, _F64P]),
                "orc_splitmix64": (_u64, [_u64, _u64]),
                "orc_fmix32": (ctypes.c_uint32, [ctypes.c_uint32]),
                "orc_sample_nice": (ctypes.c_int, [_u64, _u64, _i64, _i64, _I64P]),
                "orc_soft": (_f64, [_f64, _f64]),
                "orc_residual": (None, [_i64, _i64, _I64P, _I32P, _F64P, _F64P, _F64P, _F64P]),
                "orc_objective": (_f64, [_i64, _i64, _F64P, _F64P, _f64]),
                "orc_gradient": (None, [_i64, _I64P, _I32P, _F64P, _F64P, _F64P]),
                "orc_dual_gap": (_f64, [_i64, _i64, _I64P, _I32P, _F64P, _F64P, _F64P, _F64P, _f64,
                                        ctypes.POINTER(_f64), ctypes.POINTER(_f64)]),
                "orc_step_with_set": (_i64, [_i64, _i64, _I64P, _I32P, _F64P, _F64P, _f64, _f64,
                                             _i64, _I64P, _F64P, _F64P]),
                "orc_pcdm_run": (_i64, [_i64, _i64, _I64P, _I32P, _F64P, _F64P, _f64, _f64,
                                        _i64, _u64, _i64, _i64, _F64P, _F64P]),
                "orc_draw_independent": (ctypes.c_int, [_u64, _u64, _i64, _i64, _I64P]),
                "orc_draw_binomial": (ctypes.c_int, [_u64, _u64, _i64, _i64, _f64, _I64P]),
                "orc_sample_set": (_i64, [ctypes.c_int, _f64, _u64, _u64, _i64, _i64, ctypes.c_void_p,
                                          _i64, _I64P]),
                "orc_independent_moments": (None, [_i64, _i64, ctypes.POINTER(_f64), ctypes.POINTER(_f64)]),
                "orc_beta_du": (_f64, [_i64, _i64, _f64, _f64]),
                "orc_async_serial_run": (_i64, [_i64, _i64, _I64P, _I32P, _F64P, _F64P, _f64, _f64, _u64,
                                                _u64, _i64, _F64P, _F64P]),
                "orc_loss_value": (_f64, [ctypes.c_int, _f64, _f64]),
                "orc_loss_deriv": (_f64, [ctypes.c_int, _f64, _f64]),
                "orc_loss_curvature_bound": (_f64, [ctypes.c_int]),
                "orc_model_prox": (_f64, [_f64, _f64, _f64, _f64, _f64, _f64, _f64]),
                "orc_model_omega": (_f64, [_i64, _F64P, _f64, _f64, _f64, _f64, _f64]),
                "orc_model_objective": (_f64, [_i64, _i64, _F64P, _F64P, _F64P, ctypes.c_int, _f64, _f64, _f64,
                                               _f64, _f64, _f64]),
                "orc_model_step_with_set": (_i64, [_i64, _i64, _I64P, _I32P, _F64P, _F64P, _F64P, ctypes.c_int,
                                                   _f64, _f64, _f64, _f64, _f64, _f64, _f64, _i64, _I64P, _F64P,
                                                   _F64P]),
                "orc_model_run": (_i64, [_i64, _i64, _I64P, _I32P, _F64P, _F64P, _F64P, ctypes.c_int, _f64, _f64,
                                         _f64, _f64, _f64, _f64, _f64, _i64, _u64, _i64, _i64, _F64P, _F64P]),
                "orc_column_stats_f32": (ctypes.c_int, [_i64, _I64P, _I32P, _F32P, _F64P, _i64, _I32MP,
                                                        ctypes.POINTER(_f64), ctypes.c_int]),
                "orc_pcdm_run_sampling": (_i64, [_i64, _i64, _I64P, _I32P, _F64P, _F64P, _f64, _f64,
                                                 _i64, _u64, _i64, _i64, ctypes.c_int, _f64,
                                                 ctypes.c_void_p, _i64, _F64P, _F64P]),
            }
            for name, (res, args) in sig.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _handle = lib
    return _handle


# --------------------------------------------------------------------------- #
# scalar rules
# --------------------------------------------------------------------------- #

def beta_nice(omega: int, tau: int, n: int) -> float:
    """beta for the tau-nice sampling (Table ESO; theorem ESO for nice samplings)."""
    return _lib().orc_beta_nice(int(omega), int(tau), int(n))


def beta_uniform(omega: int, tau: int) -> float:
    """Conservative beta = min(omega, tau) of any tau-uniform sampling (Table ESO)."""
    return _lib().orc_beta_uniform(int(omega), int(tau))


def beta_binomial(omega: int, tau: int, n: int, pb: float) -> float:
    """beta of the (tau, p_b)-binomial sampling (Table ESO)."""
    return _lib().orc_beta_binomial(int(omega), int(tau), int(n), float(pb))


def soft(u: float, c: float) -> float:
    """Soft threshold sign(u)*max(|u|-c, 0): the l1 block minimiser."""
    return _lib().orc_soft(float(u), float(c))


def splitmix64(state: int, t: int) -> int:
    """Output number t of SplitMix64 started at ``state``."""
    return int(_lib().orc_splitmix64(state & (2**64 - 1), t & (2**64 - 1)))


def fmix32(h: int) -> int:
    """MurmurHash3 32-bit finaliser."""
    return int(_lib().orc_fmix32(h & 0xFFFFFFFF))


def sample_nice(seed: int, k: int, tau: int, n: int) -> np.ndarray:
    """S_k of the tau-nice sampler, in slot order (int64 [tau])."""
    out = np.empty(max(int(tau), 1), dtype=np.int64)
    if _lib().orc_sample_nice(seed & (2**64 - 1), int(k), int(tau), int(n), out) != 0:
        raise ValueError("bad sampler arguments")
    return out[: int(tau)]


SAMPLINGS = {"nice": 0, "independent": 1, "binomial": 2}


def draw_independent(seed: int, k: int, tau: int, n: int) -> np.ndarray:
    """Raw picks of the tau processors of the tau-independent sampling at step
    k, slot order, duplicates kept (section Block Samplings, independent
    sampling)."""
    out = np.empty(max(int(tau), 1), dtype=np.int64)
    if _lib().orc_draw_independent(seed & (2**64 - 1), int(k), int(tau), int(n), out) != 0:
        raise ValueError("bad sampler arguments")
    return out[: int(tau)]


def draw_binomial(seed: int, k: int, tau: int, n: int, pb: float) -> np.ndarray:
    """Slot blocks of the (tau, p_b)-binomial sampling at step k: pi_k(j) of the
    tau-nice sampler, or -1 where slot j is unavailable (implicit selection)."""
    out = np.empty(max(int(tau), 1), dtype=np.int64)
    if _lib().orc_draw_binomial(seed & (2**64 - 1), int(k), int(tau), int(n), float(pb), out) != 0:
        raise ValueError("bad sampler arguments")
    return out[: int(tau)]


def _mask_arg(mask):
    if mask is None:
        return None, 0, None
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    return m.ctypes.data_as(ctypes.c_void_p), int(m.size), m


def sample_set(sampling: str, seed: int, k: int, tau: int, n: int, pb: float = 1.0, mask=None) -> np.ndarray:
    """S_k of a sampling with the drop mask applied, ascending, no duplicates."""
    out = np.empty(max(int(tau), 1), dtype=np.int64)
    mp, ml, _keep = _mask_arg(mask)
    c = _lib().orc_sample_set(SAMPLINGS[sampling], float(pb), seed & (2**64 - 1), int(k), int(tau), int(n),
                              mp, ml, out)
    if c < 0:
        raise ValueError("bad sampler arguments")
    return out[:c].copy()


def independent_moments(tau: int, n: int):
    """(E|S|, E|S|^2) of the tau-independent sampling (inclusion-exclusion)."""
    e1, e2 = _f64(), _f64()
    _lib().orc_independent_moments(int(tau), int(n), ctypes.byref(e1), ctypes.byref(e2))
    return e1.value, e2.value


def beta_du(omega: int, n: int, e1: float, e2: float) -> float:
    """beta of a doubly uniform sampling with E|S| = e1, E|S|^2 = e2 (Table ESO)."""
    return _lib().orc_beta_du(int(omega), int(n), float(e1), float(e2))


def beta_for(sampling: str, omega: int, tau: int, n: int, pb: float = 1.0) -> float:
    """The ESO beta (w = L) of the named sampling."""
    if sampling == "nice":
        return beta_nice(omega, tau, n)
    if sampling == "independent":
        return beta_du(omega, n, *independent_moments(tau, n))
    if sampling == "binomial":
        return beta_binomial(omega, tau, n, pb)
    raise ValueError(sampling)


# --------------------------------------------------------------------------- #
# matrix helpers (float64 upcast of the stored values)
# --------------------------------------------------------------------------- #

def _arrays(A):
    return (np.ascontiguousarray(A.col_ptr, dtype=np.int64),
            np.ascontiguousarray(A.row_idx, dtype=np.int32),
            np.ascontiguousarray(A.values_f64(), dtype=np.float64))


def omega(A) -> int:
    """Maximum number of nonzeros in a row of A."""
    cp, ri, v = _arrays(A)
    return int(_lib().orc_omega(A.m, A.n, cp, ri, v))


def lipschitz(A) -> np.ndarray:
    """L_i = ||a_i||^2 from the stored values."""
    cp, _, v = _arrays(A)
    L = np.empty(A.n)
    _lib().orc_lipschitz(A.n, cp, v, L)
    return L


def residual(A, x, b) -> np.ndarray:
    cp, ri, v = _arrays(A)
    r = np.empty(A.m)
    _lib().orc_residual(A.m, A.n, cp, ri, v, np.ascontiguousarray(x, np.float64),
                        np.ascontiguousarray(b, np.float64), r)
    return r


def objective(A, x, b, lam) -> float:
    r = residual(A, x, b)
    return _lib().orc_objective(A.m, A.n, r, np.ascontiguousarray(x, np.float64), float(lam))


def gradient(A, r) -> np.ndarray:
    cp, ri, v = _arrays(A)
    g = np.empty(A.n)
    _lib().orc_gradient(A.n, cp, ri, v, np.ascontiguousarray(r, np.float64), g)
    return g


def dual_gap(A, b, x, lam, r=None):
    """(gap, F, D) with theta = r*min(1, lam/||A^T r||_inf)."""
    cp, ri, v = _arrays(A)
    if r is None:
        r = residual(A, x, b)
    F, D = _f64(), _f64()
    gap = _lib().orc_dual_gap(A.m, A.n, cp, ri, v, np.ascontiguousarray(b, np.float64),
                              np.ascontiguousarray(x, np.float64), np.ascontiguousarray(r, np.float64),
                              float(lam), ctypes.byref(F), ctypes.byref(D))
    return gap, F.value, D.value


class Solver:
    """Serial float64 PCDM1 state: x, r = A x - b, step counter k.

    ``beta_rule``: 'nice' (the sampling's own ESO beta) or 'uniform'
    (min(omega, tau)).  ``sampling``: 'nice', 'independent' or 'binomial'
    (with availability ``pb``); ``mask``: optional drop mask over slots.
    """

    def __init__(self, A, b, lam, tau, seed=0, beta_rule="nice", beta=None, x0=None,
                 sampling="nice", pb=1.0, mask=None):
        self.A = A
        self.m, self.n = A.m, A.n
        self.cp, self.ri, self.v = _arrays(A)
        self.b = np.ascontiguousarray(b, np.float64)
        self.lam = float(lam)
        self.tau = int(tau)
        self.seed = int(seed)
        self.L = np.empty(self.n)
        _lib().orc_lipschitz(self.n, self.cp, self.v, self.L)
        self.omega = int(_lib().orc_omega(self.m, self.n, self.cp, self.ri, self.v))
        self.sampling = sampling
        self.pb = float(pb)
        self.mask = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        if beta is not None:
            self.beta = float(beta)
        elif beta_rule == "nice":
            self.beta = beta_for(sampling, self.omega, self.tau, self.n, self.pb)
        elif beta_rule == "uniform":
            self.beta = beta_uniform(self.omega, self.tau)
        else:
            raise ValueError(beta_rule)
        self.x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64)
        self.r = np.empty(self.m)
        self.refresh()
        self.k = 0
        self.changed = 0

    def refresh(self):
        _lib().orc_residual(self.m, self.n, self.cp, self.ri, self.v, self.x, self.b, self.r)

    def step(self, nsteps: int = 1) -> int:
        if self.sampling == "nice" and self.mask is None:
            c = _lib().orc_pcdm_run(self.m, self.n, self.cp, self.ri, self.v, self.L, self.lam,
                                    self.beta, self.tau, self.seed & (2**64 - 1), self.k, int(nsteps),
                                    self.x, self.r)
        else:
            mp, ml, _keep = _mask_arg(self.mask)
            c = _lib().orc_pcdm_run_sampling(self.m, self.n, self.cp, self.ri, self.v, self.L, self.lam,
                                             self.beta, self.tau, self.seed & (2**64 - 1), self.k,
                                             int(nsteps), SAMPLINGS[self.sampling], self.pb, mp, ml,
                                             self.x, self.r)
        if c < 0:
            raise RuntimeError("oracle step failed")
        self.k += int(nsteps)
        self.changed += int(c)
        return int(c)

    def step_with_set(self, S) -> int:
        S = np.ascontiguousarray(S, dtype=np.int64)
        c = _lib().orc_step_with_set(self.m, self.n, self.cp, self.ri, self.v, self.L, self.lam,
                                     self.beta, S.size, S, self.x, self.r)
        if c < 0:
            raise ValueError("bad set")
        return int(c)

    def objective(self, fresh: bool = True) -> float:
        r = residual(self.A, self.x, self.b) if fresh else self.r
        return _lib().orc_objective(self.m, self.n, np.ascontiguousarray(r), self.x, self.lam)

    def gap(self):
        return dual_gap(self.A, self.b, self.x, self.lam, r=residual(self.A, self.x, self.b))

    def steps_per_epoch(self) -> int:
        return -(-self.n // self.tau)

    def async_serial(self, launch: int, nupdates: int) -> int:
        """One processor of the asynchronous variant: nupdates serial updates
        over the pick stream of launch number ``launch`` (independent uniform
        picks), each applied at once."""
        c = _lib().orc_async_serial_run(self.m, self.n, self.cp, self.ri, self.v, self.L, self.lam, self.beta,
                                        self.seed & (2**64 - 1), int(launch), int(nupdates), self.x, self.r)
        if c < 0:
            raise RuntimeError("oracle async run failed")
        self.changed += int(c)
        return int(c)


# --------------------------------------------------------------------------- #
# adjoint through the LASSO solution (float64 support solve)
# --------------------------------------------------------------------------- #

def lasso_adjoint(A, x, g):
    """(dL/db, dL/dlambda) for L(x(b, lambda)) at a LASSO solution x.

    On the support S of x with signs s the optimality conditions read
    A_S^T (A_S x_S - b) + lambda s = 0, so x_S = (A_S^T A_S)^{-1}(A_S^T b - lambda s)
    while S and s stay fixed.  With v = (A_S^T A_S)^{-1} g_S (g = dL/dx):
    dL/db = A_S v and dL/dlambda = -s^T v.  The normal matrix is formed in
    float64 and solved directly (library Cholesky / LU)."""
    import scipy.linalg
    import scipy.sparse as sp
    x = np.asarray(x, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    S = np.nonzero(x)[0]
    if S.size == 0:
        return np.zeros(A.m), 0.0
    M = sp.csc_matrix((A.values_f64(), A.row_idx, A.col_ptr), shape=(A.m, A.n))[:, S]
    G = (M.T @ M).toarray()
    try:
        v = scipy.linalg.cho_solve(scipy.linalg.cho_factor(G), g[S])
    except np.linalg.LinAlgError:
        v = np.linalg.lstsq(G, g[S], rcond=None)[0]
    s = np.sign(x[S])
    return np.asarray(M @ v).ravel(), float(-(s @ v))


# --------------------------------------------------------------------------- #
# other losses and regularisers
# --------------------------------------------------------------------------- #

LOSSES = {"square": 0, "logistic": 1, "sqhinge": 2}


def loss_value(loss: str, z: float, y: float) -> float:
    return _lib().orc_loss_value(LOSSES[loss], float(z), float(y))


def loss_deriv(loss: str, z: float, y: float) -> float:
    return _lib().orc_loss_deriv(LOSSES[loss], float(z), float(y))


def loss_curvature_bound(loss: str) -> float:
    return _lib().orc_loss_curvature_bound(LOSSES[loss])


def model_prox(v, bl, l1=0.0, l2=0.0, c=0.0, lo=-np.inf, hi=np.inf) -> float:
    """argmin_u (bl/2)(u - v)^2 + l1|u| + (l2/2)u^2 + c u over lo <= u <= hi."""
    return _lib().orc_model_prox(float(v), float(bl), float(l1), float(l2), float(c), float(lo), float(hi))


class ModelSolver:
    """Serial float64 PCDM1 on F(x) = s sum_j phi(z_j, y_j) + sum_i Omega_i(x_i),
    z = A x, with the tau-nice sampler and beta of the tau-nice row.

    ``loss``: 'square' (y = targets), 'logistic' or 'sqhinge' (y = labels
    +-1); Omega_i(t) = l1|t| + (l2/2)t^2 + c t + indicator(lo <= t <= hi)."""

    def __init__(self, A, y, tau, seed=0, loss="square", scale=1.0, l1=0.0, l2=0.0, c=0.0,
                 lo=-np.inf, hi=np.inf, beta=None):
        self.A = A
        self.m, self.n = A.m, A.n
        self.cp, self.ri, self.v = _arrays(A)
        self.y = np.ascontiguousarray(y, np.float64)
        self.loss = loss
        self.s, self.l1, self.l2, self.c, self.lo, self.hi = (float(scale), float(l1), float(l2), float(c),
                                                              float(lo), float(hi))
        self.tau = int(tau)
        self.seed = int(seed)
        self.L = np.empty(self.n)
        _lib().orc_lipschitz(self.n, self.cp, self.v, self.L)
        self.L *= self.s * loss_curvature_bound(loss)
        self.omega = int(_lib().orc_omega(self.m, self.n, self.cp, self.ri, self.v))
        self.beta = beta_nice(self.omega, self.tau, self.n) if beta is None else float(beta)
        self.x = np.zeros(self.n)
        self.z = np.zeros(self.m)
        self.k = 0
        self.changed = 0

    def _margins(self):
        z = np.empty(self.m)
        _lib().orc_residual(self.m, self.n, self.cp, self.ri, self.v, self.x, np.zeros(self.m), z)
        return z

    def step(self, nsteps: int = 1) -> int:
        c = _lib().orc_model_run(self.m, self.n, self.cp, self.ri, self.v, self.L, self.y, LOSSES[self.loss],
                                 self.s, self.l1, self.l2, self.c, self.lo, self.hi, self.beta, self.tau,
                                 self.seed & (2**64 - 1), self.k, int(nsteps), self.x, self.z)
        if c < 0:
            raise RuntimeError("oracle model step failed")
        self.k += int(nsteps)
        self.changed += int(c)
        return int(c)

    def step_with_set(self, S) -> int:
        S = np.ascontiguousarray(S, dtype=np.int64)
        c = _lib().orc_model_step_with_set(self.m, self.n, self.cp, self.ri, self.v, self.L, self.y,
                                           LOSSES[self.loss], self.s, self.l1, self.l2, self.c, self.lo,
                                           self.hi, self.beta, S.size, S, self.x, self.z)
        if c < 0:
            raise ValueError("bad set")
        return int(c)

    def objective(self) -> float:
        return _lib().orc_model_objective(self.m, self.n, self._margins(), self.y, self.x, LOSSES[self.loss],
                                          self.s, self.l1, self.l2, self.c, self.lo, self.hi)

    def steps_per_epoch(self) -> int:
        return -(-self.n // self.tau)


# --------------------------------------------------------------------------- #
# instances too large to hold on the host as float64
# --------------------------------------------------------------------------- #

def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


class ColumnStats:
    """omega = max_j #{i : a_ji != 0} and ||A^T b||_inf of a matrix streamed
    in column slices with float32 stored values (introduction, partial
    separability; the lambda rule of the LASSO experiments).  Each slice is
    split over threads; the counts and the maximum equal those of one serial
    pass over the whole matrix."""

    def __init__(self, m: int, b):
        self.m = int(m)
        self.b = np.ascontiguousarray(b, dtype=np.float64)
        if self.b.size != self.m:
            raise ValueError("b has the wrong length")
        self.counts = np.zeros(self.m, dtype=np.int32)
        self.atb_inf = 0.0
        self.ncols = 0

    def add(self, col_ptr, row_idx, val_f32) -> None:
        """Columns whose entries are row_idx/val_f32[col_ptr[i] - col_ptr[0] ..]."""
        cp = np.ascontiguousarray(col_ptr, dtype=np.int64)
        cp = cp - cp[0]
        ri = np.ascontiguousarray(row_idx, dtype=np.int32)
        v = np.ascontiguousarray(val_f32, dtype=np.float32)
        if ri.size < cp[-1] or v.size < cp[-1]:
            raise ValueError("slice shorter than its column pointers")
        best = _f64()
        if _lib().orc_column_stats_f32(cp.size - 1, cp, ri, v, self.b, self.m, self.counts, ctypes.byref(best),
                                       _threads()) != 0:
            raise ValueError("row index out of range")
        self.atb_inf = max(self.atb_inf, best.value)
        self.ncols += cp.size - 1

    @property
    def omega(self) -> int:
        return int(self.counts.max()) if self.m else 0


class ColumnSetSolver:
    """Synchronous PCDM1 state for an instance whose columns do not fit on the
    host: x (float64 [n]) and r = A x - b (float64 [m], r = -b at x = 0) are
    held whole, and each step receives the columns of its set S_k from the
    caller (stored values, widened exactly).  The step is Algorithm PCDM1's,
    through the same C step as ``Solver`` (every g_i from r_k, then the
    updates in ascending coordinate order); lambda and beta are the caller's."""

    def __init__(self, m: int, n: int, b, lam: float, beta: float):
        self.m, self.n = int(m), int(n)
        self.lam, self.beta = float(lam), float(beta)
        self.r = -np.ascontiguousarray(b, dtype=np.float64)
        if self.r.size != self.m:
            raise ValueError("b has the wrong length")
        self.x = np.zeros(self.n)
        self.changed = 0

    @staticmethod
    def _sub(S, col_ptr, row_idx, val):
        S = np.ascontiguousarray(S, dtype=np.int64)
        if S.size > 1 and np.any(np.diff(S) <= 0):
            raise ValueError("S must be ascending and distinct")
        cp = np.ascontiguousarray(col_ptr, dtype=np.int64)
        cp = cp - cp[0]
        if cp.size != S.size + 1:
            raise ValueError("one column per element of S")
        ri = np.ascontiguousarray(row_idx, dtype=np.int32)
        v = np.ascontiguousarray(val, dtype=np.float64)
        return S, cp, ri, v

    def gradient(self, S, col_ptr, row_idx, val) -> np.ndarray:
        """g_i = a_i^T r at the current r for the given columns of S."""
        S, cp, ri, v = self._sub(S, col_ptr, row_idx, val)
        g = np.empty(S.size)
        _lib().orc_gradient(S.size, cp, ri, v, self.r, g)
        return g

    def step_with_columns(self, S, col_ptr, row_idx, val) -> int:
        """One step on the set S (ascending) whose columns are given in S's
        order; returns the number of coordinates that changed."""
        S, cp, ri, v = self._sub(S, col_ptr, row_idx, val)
        L = np.empty(S.size)
        _lib().orc_lipschitz(S.size, cp, v, L)
        xs = np.ascontiguousarray(self.x[S])
        local = np.arange(S.size, dtype=np.int64)
        c = _lib().orc_step_with_set(self.m, S.size, cp, ri, v, L, self.lam, self.beta, S.size, local, xs,
                                     self.r)
        if c < 0:
            raise ValueError("bad set")
        self.x[S] = xs
        self.changed += int(c)
        return int(c)

    def objective(self) -> float:
        """F(x) = 0.5*||r||^2 + lambda*||x||_1 on the maintained r."""
        return _lib().orc_objective(self.m, self.n, self.r, self.x, self.lam)
