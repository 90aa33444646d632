"""Seeded synthetic inputs for the quantum-walk path.

This module only draws random numbers and assembles plain CSC arrays and
right-hand sides.  It holds none of the walk's arithmetic (no rescaling, no
padding, no sparsity rounding, no amplitudes): the oracle and the HIP path each
do their own preprocessing of what is produced here.

The paper's own matrices (random positive symmetric band matrices, Sec. V.B
"Numerical results") are not published, so every workload is synthetic:

* ``tridiagonal(n, seed)``: non-cyclic tridiagonal, off-diagonals U[-1,1]
  mirrored, diagonal U[-1,1]+2.
* ``offset_matrix(n, c, seed)``: exactly ``c`` stored entries per column,
  symmetric: the diagonal, ``(c-1)//2`` distinct cyclic offsets ``d`` in
  ``[1, n/2)`` placed at ``(j, j+d mod n)`` and mirrored, plus the
  self-mirrored offset ``n/2`` when ``c-1`` is odd.  Off-diagonal values are
  U[-1,1], one value per unordered pair; the diagonal is U[-1,1] + (c-1).
* ``band_matrix(n, bandwidth, seed)``: the paper's matrix family, positive
  symmetric band matrix with entries U[0,1).
* ``laplacian_2d(m, shift)``: 5-point Dirichlet Laplacian on an m x m grid
  plus ``shift`` * I.

All functions return ``Csc(n, colptr int32, rowidx int32, vals float64)``
with row indices sorted inside each column.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Csc:
    n: int
    colptr: np.ndarray  # int32, n+1
    rowidx: np.ndarray  # int32, nnz, sorted inside each column
    vals: np.ndarray  # float64 (or complex128 for a Hermitian matrix), nnz

    @property
    def nnz(self) -> int:
        return int(self.rowidx.shape[0])

    def dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n), dtype=self.vals.dtype)
        for c in range(self.n):
            for p in range(self.colptr[c], self.colptr[c + 1]):
                a[self.rowidx[p], c] = self.vals[p]
        return a


def _from_triplets(n: int, rows, cols, vals) -> Csc:
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals)
    vals = vals.astype(np.complex128 if np.iscomplexobj(vals) else np.float64)
    order = np.lexsort((rows, cols))
    rows, cols, vals = rows[order], cols[order], vals[order]
    key = cols * n + rows
    if key.size and np.any(np.diff(key) == 0):
        raise ValueError("duplicate entry in generated matrix")
    counts = np.bincount(cols, minlength=n)
    colptr = np.zeros(n + 1, dtype=np.int32)
    colptr[1:] = np.cumsum(counts)
    return Csc(n, colptr, rows.astype(np.int32), vals)


def from_dense(a: np.ndarray) -> Csc:
    """CSC of the nonzero pattern of a dense square matrix."""
    a = np.asarray(a)
    a = a.astype(np.complex128 if np.iscomplexobj(a) else np.float64)
    r, c = np.nonzero(a)
    return _from_triplets(a.shape[0], r, c, a[r, c])


def tridiagonal(n: int = 16, seed: int = 1) -> Csc:
    rng = np.random.default_rng(seed)
    off = rng.uniform(-1.0, 1.0, n - 1)
    diag = rng.uniform(-1.0, 1.0, n) + 2.0
    rows, cols, vals = [], [], []
    for j in range(n):
        rows.append(j), cols.append(j), vals.append(diag[j])
    for j in range(n - 1):
        rows += [j, j + 1]
        cols += [j + 1, j]
        vals += [off[j], off[j]]
    return _from_triplets(n, rows, cols, vals)


def offset_matrix(n: int, c: int, seed=None, rng: np.random.Generator | None = None) -> Csc:
    """Symmetric matrix with exactly ``c`` entries per column (see module doc)."""
    if rng is None:
        rng = np.random.default_rng(seed)
    if c < 1 or c > n:
        raise ValueError("need 1 <= c <= n")
    p = (c - 1) // 2
    half = (c - 1) % 2 == 1
    if p > max(0, n // 2 - 1):
        raise ValueError("too many offsets for this n")
    offsets = rng.choice(np.arange(1, n // 2), size=p, replace=False) if p else np.zeros(0, np.int64)
    j = np.arange(n)
    rows = [j]
    cols = [j]
    pieces = []
    for d in offsets:
        v = rng.uniform(-1.0, 1.0, n)
        k = (j + int(d)) % n
        rows += [j, k]
        cols += [k, j]
        pieces += [v, v]
    if half:
        h = n // 2
        v = rng.uniform(-1.0, 1.0, h)
        lo = np.arange(h)
        rows += [lo, lo + h]
        cols += [lo + h, lo]
        pieces += [v, v]
    diag = rng.uniform(-1.0, 1.0, n) + (c - 1)
    vals = [diag] + pieces
    return _from_triplets(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def hermitian_offset_matrix(n: int, c: int, seed=None, rng: np.random.Generator | None = None) -> Csc:
    """Complex Hermitian counterpart of ``offset_matrix``: the same pattern of
    exactly ``c`` entries per column; the pair at offset d holds v at (j, j+d)
    and conj(v) at (j+d, j) with v = U[-1,1] + i U[-1,1], except the first
    offset, which keeps real values U[-1,1] (negative ones included) so that
    the real axis is exercised as well; the diagonal is real, U[-1,1] + (c-1)."""
    if rng is None:
        rng = np.random.default_rng(seed)
    if c < 1 or c > n:
        raise ValueError("need 1 <= c <= n")
    p = (c - 1) // 2
    half = (c - 1) % 2 == 1
    if p > max(0, n // 2 - 1):
        raise ValueError("too many offsets for this n")
    offsets = rng.choice(np.arange(1, n // 2), size=p, replace=False) if p else np.zeros(0, np.int64)
    j = np.arange(n)
    rows, cols, vals = [j], [j], [rng.uniform(-1.0, 1.0, n) + (c - 1) + 0j]
    for i, d in enumerate(offsets):
        v = rng.uniform(-1.0, 1.0, n) + (0.0 if i == 0 else 1j * rng.uniform(-1.0, 1.0, n))
        k = (j + int(d)) % n
        rows += [j, k]
        cols += [k, j]
        vals += [v, np.conj(v)]
    if half:
        h = n // 2
        v = rng.uniform(-1.0, 1.0, h) + 1j * rng.uniform(-1.0, 1.0, h)
        lo = np.arange(h)
        rows += [lo, lo + h]
        cols += [lo + h, lo]
        vals += [v, np.conj(v)]
    r, cc, vv = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    order = np.lexsort((r, cc))
    r, cc, vv = r[order], cc[order], vv[order]
    if np.any(np.diff(cc * n + r) == 0):
        raise ValueError("duplicate entry in generated matrix")
    colptr = np.zeros(n + 1, dtype=np.int32)
    colptr[1:] = np.cumsum(np.bincount(cc, minlength=n))
    return Csc(n, colptr, r.astype(np.int32), vv.astype(np.complex128))


def band_matrix(n: int, bandwidth: int, seed: int = 0) -> Csc:
    """Positive symmetric band matrix, entries U[0,1) (the paper's family)."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for d in range(0, bandwidth + 1):
        v = rng.uniform(0.0, 1.0, n - d)
        j = np.arange(n - d)
        rows.append(j), cols.append(j + d), vals.append(v)
        if d:
            rows.append(j + d), cols.append(j), vals.append(v)
    return _from_triplets(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def fixed_point_band(n: int, bandwidth: int, word: int, seed: int = 0, negative: float = 0.0) -> Csc:
    """Symmetric band matrix whose entries are fixed-point numbers of `word`
    fraction bits in (0, 1): q / 2^word with q uniform on 1 ... 2^word - 1 (the
    paper's matrices, Sec. V.B).  `negative`: probability that an
    off-diagonal pair is negated (the paper's matrices are positive)."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for d in range(0, bandwidth + 1):
        v = rng.integers(1, 1 << word, n - d).astype(np.float64) / float(1 << word)
        if d and negative:
            v = np.where(rng.uniform(size=n - d) < negative, -v, v)
        j = np.arange(n - d)
        rows.append(j), cols.append(j + d), vals.append(v)
        if d:
            rows.append(j + d), cols.append(j), vals.append(v)
    return _from_triplets(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def laplacian_2d(m: int = 32, shift: float = 0.1) -> Csc:
    n = m * m
    rows, cols, vals = [], [], []
    for y in range(m):
        for x in range(m):
            i = y * m + x
            rows.append(i), cols.append(i), vals.append(4.0 + shift)
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                xx, yy = x + dx, y + dy
                if 0 <= xx < m and 0 <= yy < m:
                    rows.append(yy * m + xx), cols.append(i), vals.append(-1.0)
    return _from_triplets(n, rows, cols, vals)


def uniform_b(n: int) -> np.ndarray:
    return np.full(n, 1.0 / np.sqrt(n))


def gaussian_b(n: int, seed: int = 0) -> np.ndarray:
    b = np.random.default_rng(seed).normal(size=n)
    return b / np.linalg.norm(b)


def basis_b(n: int, j: int) -> np.ndarray:
    b = np.zeros(n)
    b[j] = 1.0
    return b


# ---- the named workloads ----------------------------------------------------

def tiny_tridiagonal():
    """16x16 tridiagonal (seed 1), start column j=0."""
    return tridiagonal(16, seed=1), basis_b(16, 0)


def paper_scale(n: int = 16384, c: int = 8, seed: int = 2):
    """G(16384, 8), uniform superposition over all columns."""
    return offset_matrix(n, c, seed=seed), uniform_b(n)


# The shapes of the paper's five experimental matrices (its table of
# experimental settings): positive symmetric band matrices of n rows and
# bandwidth w, so 2w + 1 entries per interior column and s = 2^ceil(log2(2w+1)).
# The paper's values are not published; these are seeded stand-ins.
TABLE1_SHAPES = {
    "A": (16, 3, 11),      # s = 8
    "B": (128, 7, 12),     # s = 16
    "C": (1024, 15, 13),   # s = 32
    "D": (8192, 15, 14),   # s = 32
    "E": (16384, 31, 7),   # s = 64
}
# The word length of each shape's fixed-point entries in the same table.
TABLE1_WORD = {"A": 8, "B": 8, "C": 8, "D": 16, "E": 32}
# The paper's single-core time per walk step for each shape (context only).
TABLE1_PAPER_SECONDS_PER_STEP = {"A": 1.1e-3, "B": 12e-3, "C": 1.2, "D": 14.0, "E": 66.0}


def table1_band(name: str):
    """Band matrix of the given shape of the paper's table, uniform b."""
    n, w, seed = TABLE1_SHAPES[name]
    return band_matrix(n, w, seed=seed), uniform_b(n)


def table1_fixed_point_band(name: str):
    """The shape's band matrix with fixed-point entries of the table's word
    length, uniform b; returns (matrix, b, word length)."""
    n, w, seed = TABLE1_SHAPES[name]
    word = TABLE1_WORD[name]
    return fixed_point_band(n, w, word, seed=seed), uniform_b(n), word


def paper_band():
    """Shape E: 16384 rows, bandwidth 31 (s = 64), the paper's largest
    single-core walk-step measurement."""
    return table1_band("E")


def batched_instances(count: int = 256, seed: int = 3, emin: int = 6, emax: int = 12,
                      cmin: int = 4, cmax: int = 16):
    """``count`` instances: instance i draws from default_rng([seed, i]):
    n_i = 2**e with e ~ U{emin..emax}, c_i ~ U{cmin..cmax}, the offset matrix
    G(n_i, c_i) from the same generator, then a start column j_i ~ U[0, n_i)."""
    out = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        e = int(rng.integers(emin, emax + 1))
        n = 1 << e
        c = int(rng.integers(cmin, cmax + 1))
        a = offset_matrix(n, c, rng=rng)
        j = int(rng.integers(0, n))
        out.append((a, basis_b(n, j)))
    return out


def adjoint_problem(n: int = 1024, c: int = 8, seed: int = 4, n_obs: int = 32,
                    obs_seed: int = 5):
    """G(1024, 8) with uniform b; the observable is the total probability of
    ``n_obs`` distinct column-register outcomes drawn from default_rng(obs_seed)."""
    a = offset_matrix(n, c, seed=seed)
    obs = np.sort(np.random.default_rng(obs_seed).choice(n, size=n_obs, replace=False))
    w = np.zeros(n)
    w[obs] = 1.0
    return a, uniform_b(n), w


def fd_sample(vals_scaled: np.ndarray, count: int = 16, seed: int = 6,
              lo: float = 1e-4, hi: float = 1.0 - 1e-4) -> np.ndarray:
    """Indices of ``count`` stored entries whose (already scaled) magnitude lies
    strictly inside (lo, hi), drawn from default_rng(seed)."""
    ok = np.nonzero((np.abs(vals_scaled) > lo) & (np.abs(vals_scaled) < hi))[0]
    return np.sort(np.random.default_rng(seed).choice(ok, size=count, replace=False))


def solver_problem(m: int = 32, shift: float = 0.1, seed: int = 0):
    """5-point Laplacian on an m x m grid + shift*I, b = normalised Gaussian."""
    return laplacian_2d(m, shift), gaussian_b(m * m, seed)
