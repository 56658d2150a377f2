"""Seeded synthetic sparse LASSO instances.

Every matrix is returned in canonical CSC form: column i holds coordinate i's
data (the paper stores A by columns and uses column norms as the block
Lipschitz constants), row indices are sorted and unique within a column, and no
explicit zeros are stored.  Randomness comes from ``numpy.random.Generator``
(PCG64) seeded by the caller, so every array is reproducible.

Shapes and value laws follow the LASSO workloads of the paper's experiments
section (a planted sparse solution, a fixed number of nonzeros per column, a
bounded maximum row degree); the exact recipes are stated per function.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


@dataclasses.dataclass
class CSC:
    """Compressed sparse column matrix (host arrays)."""

    m: int
    n: int
    col_ptr: np.ndarray  # int64 [n+1]
    row_idx: np.ndarray  # int32 [nnz]
    values: np.ndarray  # float64 / float32 / uint16 (bf16 bits) [nnz]

    @property
    def nnz(self) -> int:
        return int(self.col_ptr[-1])

    def values_f64(self) -> np.ndarray:
        """Stored values widened to float64 (bf16 bit patterns are decoded)."""
        v = self.values
        if v.dtype == np.uint16:
            return (v.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        return v.astype(np.float64)

    def astype(self, dtype: str) -> "CSC":
        """Copy with values rounded to ``dtype`` ('f64', 'f32' or 'bf16')."""
        v64 = self.values_f64()
        if dtype == "f64":
            vals = v64.copy()
        elif dtype == "f32":
            vals = v64.astype(np.float32)
        elif dtype == "bf16":
            vals = f32_to_bf16_bits(v64.astype(np.float32))
        else:
            raise ValueError(f"unknown dtype {dtype!r}")
        return CSC(self.m, self.n, self.col_ptr.copy(), self.row_idx.copy(), vals)


@dataclasses.dataclass
class LassoInstance:
    """min_x 0.5*||A x - b||^2 + lam*||x||_1 with a planted solution xstar."""

    A: CSC
    b: np.ndarray  # float64 [m]
    lam: float
    xstar: Optional[np.ndarray] = None  # float64 [n]
    name: str = ""
    tau: Optional[int] = None


def f32_to_bf16_bits(v: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 (round to nearest even), returned as uint16 bits."""
    u = np.ascontiguousarray(v, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    return ((u + rounding) >> 16).astype(np.uint16)


def _dedupe_rows(rows: np.ndarray, m: int, rng: np.random.Generator) -> np.ndarray:
    """Sort each column's rows and redraw duplicates uniformly until all are distinct."""
    rows.sort(axis=1)
    while True:
        dup = np.zeros(rows.shape, dtype=bool)
        dup[:, 1:] = rows[:, 1:] == rows[:, :-1]
        bad = np.nonzero(dup.any(axis=1))[0]
        if bad.size == 0:
            return rows
        sub = rows[bad]
        d = dup[bad]
        sub[d] = rng.integers(0, m, size=int(d.sum()), dtype=np.int64)
        sub.sort(axis=1)
        rows[bad] = sub


def random_csc(
    m: int,
    n: int,
    d: int,
    rng: np.random.Generator,
    balanced: bool = False,
    normalize: bool = True,
    dtype: str = "f64",
) -> CSC:
    """Exactly ``d`` nonzeros per column at distinct rows, values N(0,1).

    ``balanced=False``: rows uniform over [0, m).  ``balanced=True``: the n*d
    entry slots are dealt to rows by a random permutation of [0, n*d) taken
    modulo m, so every row receives floor or ceil of n*d/m entries (the
    maximum row degree omega is then close to its smallest possible value);
    the rare repeated row inside one column is redrawn uniformly.
    ``normalize``: columns scaled to unit Euclidean norm in float64 before the
    values are rounded to the storage type.
    """
    if not (1 <= d <= m):
        raise ValueError("need 1 <= d <= m")
    if n * d <= 4_000_000 and 4 * d > m:
        rows = np.empty((n, d), dtype=np.int64)
        for i in range(n):
            rows[i] = np.sort(rng.choice(m, size=d, replace=False))
    else:
        if balanced:
            rows = (rng.permutation(n * d) % m).reshape(n, d)
        else:
            rows = rng.integers(0, m, size=(n, d), dtype=np.int64)
        rows = _dedupe_rows(rows, m, rng)
    vals = rng.standard_normal((n, d))
    if normalize:
        vals /= np.sqrt(np.einsum("ij,ij->i", vals, vals))[:, None]
    col_ptr = np.arange(n + 1, dtype=np.int64) * d
    A = CSC(m, n, col_ptr, rows.reshape(-1).astype(np.int32), vals.reshape(-1))
    return A if dtype == "f64" else A.astype(dtype)


def _matvec(A: CSC, x: np.ndarray) -> np.ndarray:
    """y = A x for a sparse x (input construction only)."""
    v = A.values_f64()
    nzc = np.nonzero(x)[0]
    if nzc.size == 0:
        return np.zeros(A.m)
    starts, ends = A.col_ptr[nzc], A.col_ptr[nzc + 1]
    lens = ends - starts
    idx = np.repeat(starts - np.cumsum(lens) + lens, lens) + np.arange(int(lens.sum()))
    w = v[idx] * np.repeat(x[nzc], lens)
    return np.bincount(A.row_idx[idx], weights=w, minlength=A.m)


def _abs_rmatvec_max(A: CSC, y: np.ndarray) -> float:
    """max_i |a_i^T y| (input construction only: sets lambda relative to it)."""
    v = A.values_f64()
    prod = v * y[A.row_idx]
    lens = np.diff(A.col_ptr)
    if lens.size and np.all(lens == lens[0]) and lens[0] > 0:
        s = prod.reshape(A.n, int(lens[0])).sum(axis=1)
    else:
        s = np.zeros(A.n)
        nz = lens > 0
        s[nz] = np.add.reduceat(prod, A.col_ptr[:-1][nz])
    return float(np.max(np.abs(s)))


def planted_lasso(
    A: CSC,
    xstar_nnz: int,
    noise_std: float,
    lam_factor: float,
    rng: np.random.Generator,
    name: str = "",
    tau: Optional[int] = None,
) -> LassoInstance:
    """b = A x* + noise, x* with ``xstar_nnz`` entries +/-U[1,2] at distinct
    uniform positions (fair signs), lam = lam_factor * ||A^T b||_inf, all in
    float64 from the stored (possibly rounded) values of A."""
    n = A.n
    xstar = np.zeros(n)
    k = min(int(xstar_nnz), n)
    if k > 0:
        pos = rng.choice(n, size=k, replace=False)
        signs = np.where(rng.random(k) < 0.5, -1.0, 1.0)
        xstar[pos] = signs * rng.uniform(1.0, 2.0, size=k)
    b = _matvec(A, xstar) + noise_std * rng.standard_normal(A.m)
    lam = lam_factor * _abs_rmatvec_max(A, b)
    return LassoInstance(A=A, b=b, lam=float(lam), xstar=xstar, name=name, tau=tau)


def dense_to_csc(M: np.ndarray) -> CSC:
    """Canonical CSC of a dense matrix (explicit zeros dropped)."""
    M = np.asarray(M, dtype=np.float64)
    m, n = M.shape
    rows, vals, ptr = [], [], [0]
    for i in range(n):
        nz = np.nonzero(M[:, i])[0]
        rows.append(nz)
        vals.append(M[nz, i])
        ptr.append(ptr[-1] + nz.size)
    return CSC(
        m,
        n,
        np.asarray(ptr, dtype=np.int64),
        np.concatenate(rows).astype(np.int32) if rows else np.zeros(0, np.int32),
        np.concatenate(vals) if vals else np.zeros(0),
    )


def csc_to_dense(A: CSC) -> np.ndarray:
    M = np.zeros((A.m, A.n))
    v = A.values_f64()
    for i in range(A.n):
        s, e = A.col_ptr[i], A.col_ptr[i + 1]
        M[A.row_idx[s:e], i] = v[s:e]
    return M


def tightness_matrix(n: int, omega: int, k: int, row_values: Optional[np.ndarray] = None) -> CSC:
    """0-1 matrix with exactly ``omega`` nonzeros per row and ``k`` per column.

    Row j holds ones at columns (j*omega + t) mod n, t = 0..omega-1, so the
    m*omega = n*k entries sweep the columns cyclically and every column is hit
    exactly k times (the construction of the tightness remark after the DSO
    theorem).  ``row_values`` replaces the ones of row j by row_values[j] (the
    remark's generalisation: equal nonzeros within a row).
    """
    if (n * k) % omega:
        raise ValueError("n*k must be divisible by omega")
    if omega > n:
        raise ValueError("omega <= n")
    m = n * k // omega
    M = np.zeros((m, n))
    for j in range(m):
        cols = (j * omega + np.arange(omega)) % n
        M[j, cols] = 1.0 if row_values is None else row_values[j]
    return dense_to_csc(M)


def biregular_matrix(m: int, n: int, omega: int, rng: np.random.Generator) -> CSC:
    """Random 0-1 matrix with exactly ``omega`` ones in every row and
    m*omega/n in every column (a random biregular pattern: the column slots,
    each column repeated m*omega/n times, are shuffled and dealt to the rows
    omega at a time; a column repeated within a row is swapped with a slot of
    another row until no row repeats one).  The matrix of the tightness
    remark after the DSO theorem with its pattern drawn at random instead of
    cyclically."""
    if (m * omega) % n or omega > n:
        raise ValueError("m*omega must be a multiple of n and omega <= n")
    k = m * omega // n
    slots = rng.permutation(np.repeat(np.arange(n, dtype=np.int64), k)).reshape(m, omega)
    for _ in range(10000):
        srt = np.sort(slots, axis=1)
        bad = np.nonzero(np.any(srt[:, 1:] == srt[:, :-1], axis=1))[0]
        if bad.size == 0:
            break
        for j in bad:
            row = slots[j]
            _, first = np.unique(row, return_index=True)
            for t in np.setdiff1d(np.arange(omega), first):
                j2, t2 = int(rng.integers(m)), int(rng.integers(omega))
                slots[j, t], slots[j2, t2] = slots[j2, t2], slots[j, t]
    else:
        raise RuntimeError("could not remove repeated columns")
    rows = np.repeat(np.arange(m, dtype=np.int64), omega)
    cols = slots.ravel()
    order = np.lexsort((rows, cols))
    col_ptr = np.zeros(n + 1, dtype=np.int64)
    col_ptr[1:] = np.cumsum(np.bincount(cols, minlength=n))
    return CSC(m, n, col_ptr, rows[order].astype(np.int32), np.ones(m * omega))


def separable_matrix(n: int, rows_per_col: int, rng: np.random.Generator) -> CSC:
    """Disjoint row supports: column i owns rows [i*r, (i+1)*r); omega = 1."""
    r = rows_per_col
    vals = rng.standard_normal(n * r)
    rows = np.arange(n * r, dtype=np.int32)
    return CSC(n * r, n, np.arange(n + 1, dtype=np.int64) * r, rows, vals)


def _sylvester_hadamard(b: int) -> np.ndarray:
    H = np.ones((1, 1))
    while H.shape[0] < b:
        H = np.block([[H, H], [H, -H]])
    if H.shape[0] != b:
        raise ValueError("block size must be a power of two")
    return H


def orthonormal_block_hadamard(nblocks: int, bsize: int, rng: Optional[np.random.Generator] = None) -> CSC:
    """A^T A = I: block diagonal of Sylvester-Hadamard blocks scaled by
    1/sqrt(bsize), rows and columns randomly permuted when ``rng`` is given.
    Every row has ``bsize`` nonzeros, so omega = bsize."""
    H = _sylvester_hadamard(bsize) / np.sqrt(bsize)
    n = nblocks * bsize
    M = np.zeros((n, n))
    for t in range(nblocks):
        M[t * bsize:(t + 1) * bsize, t * bsize:(t + 1) * bsize] = H
    if rng is not None:
        M = M[rng.permutation(n)][:, rng.permutation(n)]
    return dense_to_csc(M)


def random_csc_ragged(m: int, n: int, dmin: int, dmax: int, rng: np.random.Generator,
                      normalize: bool = False, dtype: str = "f64", shuffle_rows: bool = True) -> CSC:
    """Column degrees uniform in [dmin, dmax] (distinct rows, N(0,1) values).
    ``shuffle_rows`` stores each column's rows in random order (CSC allows any
    order within a column)."""
    degs = rng.integers(dmin, dmax + 1, size=n)
    col_ptr = np.zeros(n + 1, dtype=np.int64)
    col_ptr[1:] = np.cumsum(degs)
    rows = np.empty(int(col_ptr[-1]), dtype=np.int32)
    vals = rng.standard_normal(int(col_ptr[-1]))
    for i in range(n):
        s, e = col_ptr[i], col_ptr[i + 1]
        r = rng.choice(m, size=int(degs[i]), replace=False)
        rows[s:e] = r if shuffle_rows else np.sort(r)
        if normalize:
            vals[s:e] /= np.linalg.norm(vals[s:e])
    A = CSC(m, n, col_ptr, rows, vals)
    return A if dtype == "f64" else A.astype(dtype)
