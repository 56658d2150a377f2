"""Named LASSO workloads (synthetic stand-ins shaped like the paper's runs).

The paper's billion-variable LASSO (experiments section) uses a planted sparse
solution, 20 nonzeros per column and a small maximum row degree omega; its
generator is not given, so these recipes reproduce the shape, not the data.

Noise levels written N(0, s) are read as variances (std = sqrt(s)) except
where the recipe states a standard deviation.  Seeds: data seed 0 unless
given; instance j of the batched path uses ``seed + j``.
"""

from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

from .lasso import LassoInstance, planted_lasso, random_csc

# name -> recipe (all sizes at full scale; ``scale`` shrinks n and m together)
CONFIGS: Dict[str, dict] = {
    # small FP64 parity case: 2000 x 1000, 20 nnz/col uniform rows, unit columns
    "small_2000x1000": dict(m=2000, n=1000, d=20, balanced=False, normalize=True, xstar_nnz=50,
               noise_std=0.01, lam_factor=0.1, taus=(1, 8), epochs=200),
    # paper-shaped single instance: 1e6 x 1e7, 20 nnz/col from balanced slots
    "lasso_1e6x1e7": dict(m=1_000_000, n=10_000_000, d=20, balanced=True, normalize=True,
               xstar_nnz=10_000, noise_std=1e-2, lam_factor=0.05,
               taus=(1024, 65536, 1_000_000)),
    # same with more rows so that the balanced maximum row degree is ~60
    "lasso_3.33e6x1e7": dict(m=3_330_000, n=10_000_000, d=20, balanced=True, normalize=True,
                xstar_nnz=10_000, noise_std=1e-2, lam_factor=0.05,
                taus=(1024, 65536, 1_000_000)),
    # differentiable LASSO (train part): 1e5 x 1e6, 10 nnz/col, N(0,1) values
    "train_1e5x1e6": dict(m=100_000, n=1_000_000, d=10, balanced=False, normalize=False,
               xstar_nnz=2000, noise_std=0.1, lam_factor=0.1, taus=(4096,)),
    # big single-GPU instance: 2e8 x 5e8, 20 nnz/col, balanced slots
    # built on the device by the counter-based recipe of workloads/csrc/gen_common.h
    "lasso_2e8x5e8": dict(m=200_000_000, n=500_000_000, d=20, balanced=True, normalize=True,
               xstar_nnz=100_000, noise_std=1e-2, lam_factor=0.05,
               taus=(65536, 1 << 20), device_gen=True),
}


def make_config(name: str, seed: int = 0, scale: float = 1.0, dtype: str = "f32",
                tau: int | None = None) -> LassoInstance:
    """Build one named single-instance workload.  ``scale`` < 1 shrinks m, n
    and the planted support proportionally (d is kept)."""
    c = CONFIGS[name]
    m = max(int(round(c["m"] * scale)), c["d"])
    n = max(int(round(c["n"] * scale)), 1)
    rng = np.random.default_rng(seed)
    A = random_csc(m, n, c["d"], rng, balanced=c["balanced"], normalize=c["normalize"], dtype=dtype)
    k = max(1, int(round(c["xstar_nnz"] * scale))) if scale < 1 else c["xstar_nnz"]
    t = tau if tau is not None else c["taus"][-1]
    inst = planted_lasso(A, k, c["noise_std"], c["lam_factor"], rng, name=name, tau=min(t, n))
    return inst


def batched_path(count: int = 64, seed: int = 0, nmin: float = 1e3, nmax: float = 1e6,
                 dtype: str = "f32", tau_cap: int = 4096) -> List[LassoInstance]:
    """Many uneven LASSO instances for the batched solver.

    Instance j: n_j = round(10^U[log10 nmin, log10 nmax]), m_j = n_j / 5,
    10 nonzeros per column with N(0,1) values (not normalised), x* 1% dense
    with +/-U[1,2] entries, noise std 0.01, lambda_j on the geometric grid
    0.5 * 0.01^(j/(count-1)) * ||A_j^T b_j||_inf, tau_j = min(n_j, tau_cap).
    """
    out = []
    rng0 = np.random.default_rng(seed)
    ns = np.round(10 ** rng0.uniform(math.log10(nmin), math.log10(nmax), size=count)).astype(int)
    for j in range(count):
        rng = np.random.default_rng(seed + j + 1)
        n = int(ns[j])
        m = max(n // 5, 10)
        A = random_csc(m, n, 10, rng, balanced=False, normalize=False, dtype=dtype)
        frac = 0.5 * (0.01 ** (j / max(count - 1, 1)))
        inst = planted_lasso(A, max(1, n // 100), 0.01, frac, rng, name=f"path{j}",
                             tau=min(n, tau_cap))
        out.append(inst)
    return out
