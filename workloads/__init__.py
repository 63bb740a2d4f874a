"""Seeded synthetic lower-triangular systems ``L x = b`` in CSR form.

This module only *generates inputs*.  It holds none of the solver's
arithmetic (no levels, no elimination, no substitution): it draws a
sparsity pattern, fills it with values, and draws right-hand sides.  Both
the CPU oracle (``oracle/``) and the GPU library are fed from here, and
neither of them is imported by this module.

CSR convention used everywhere: ``row_ptr`` int32[n+1], ``col_idx`` int32[nnz],
``val`` float64[nnz]; within a row the columns are strictly increasing and the
diagonal entry is the last one of the row.

Value rule (the same for every family):
  * numpy ``default_rng(seed)`` (PCG64); draw order is structure, then
    values, then right-hand sides;
  * off-diagonal entries ``uniform(-0.25, 0.0)`` drawn in CSR order;
  * diagonal ``1 + sum(|off-diagonals of the row|)``, accumulated in column
    order, which makes ``L`` a diagonally dominant M-matrix (so ``|x| <= 1``
    for ``|b| <= 1``);
  * right-hand sides ``uniform(-1, 1)``.

Structural families (sizes of the large workload in brackets):
  * ``stencil2d(g)``  lower triangle of the 5-point stencil on a g x g grid
    [g=100 small workload];
  * ``stencil3d(g)``  lower triangle of the 7-point stencil on g^3 [g=128];
  * ``banded(n, bw, lo, hi)``  each row holds U{lo..hi} entries including the
    diagonal, the off-diagonals a uniform subset of the previous ``bw``
    columns [n=1e6, bw=200, 8..24];
  * ``powerlaw(n, tail)``  Zipf(1.8) row lengths capped at 64, uniform
    predecessors for the bulk, then a serial tail of ``tail`` rows grouped in
    chained levels of width U{1..4} [n=4e6, tail=2e4].
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "System", "assemble", "stencil2d", "stencil3d", "banded", "powerlaw",
    "random_lower", "bidiagonal", "diagonal", "from_pairs", "transpose", "batch_corpus", "config",
    "CONFIGS", "rhs", "fp32_valued",
]


@dataclasses.dataclass
class System:
    """A CSR lower-triangular matrix and one or more right-hand sides."""
    name: str
    row_ptr: np.ndarray  # int32[n+1]
    col_idx: np.ndarray  # int32[nnz]
    val: np.ndarray      # float64[nnz]
    b: np.ndarray        # float64[n] or float64[n, k] (row-major)

    @property
    def n(self) -> int:
        return int(self.row_ptr.size - 1)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.size)


def _csr_from_sorted_pairs(n: int, rows: np.ndarray, cols: np.ndarray):
    """Insert the diagonal after the (row-major, column-sorted) off-diagonal
    pairs and return ``row_ptr``, ``col_idx`` and the position of each
    off-diagonal and each diagonal entry in the CSR arrays."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    counts = np.bincount(rows, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts + 1, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    if nnz > np.iinfo(np.int32).max:
        raise ValueError("matrix too large for int32 CSR")
    off_pos = np.arange(rows.size, dtype=np.int64) + rows
    diag_pos = row_ptr[1:] - 1
    col_idx = np.empty(nnz, dtype=np.int32)
    col_idx[off_pos] = cols
    col_idx[diag_pos] = np.arange(n, dtype=np.int32)
    return row_ptr.astype(np.int32), col_idx, off_pos, diag_pos, rows


def assemble(name: str, n: int, rows, cols, rng: np.random.Generator,
             k: int = 1) -> System:
    """Build a :class:`System` from a row-major, column-sorted list of strictly
    lower off-diagonal positions, drawing values and ``k`` right-hand sides
    from ``rng`` according to the value rule of this module."""
    row_ptr, col_idx, off_pos, diag_pos, rows64 = _csr_from_sorted_pairs(n, rows, cols)
    val = np.empty(col_idx.size, dtype=np.float64)
    off = rng.uniform(-0.25, 0.0, size=off_pos.size)
    val[off_pos] = off
    # bincount accumulates in input order, i.e. in column order within a row.
    val[diag_pos] = 1.0 + np.bincount(rows64, weights=np.abs(off), minlength=n)
    b = rhs(n, rng, k)
    return System(name, row_ptr, col_idx, val, b)


def rhs(n: int, rng: np.random.Generator, k: int = 1) -> np.ndarray:
    """``k`` right-hand sides, uniform in [-1, 1); shape (n,) for k == 1,
    else (n, k) row-major."""
    if k == 1:
        return rng.uniform(-1.0, 1.0, size=n)
    return rng.uniform(-1.0, 1.0, size=(n, k))


# --------------------------------------------------------------- families --

def stencil2d(g: int, seed: int = 0, k: int = 1) -> System:
    """Lower triangle of the 5-point stencil on a g x g grid, row
    ``i = r*g + c`` coupled to ``i-g`` (r > 0) and ``i-1`` (c > 0)."""
    rng = np.random.default_rng(seed)
    n = g * g
    i = np.arange(n, dtype=np.int64)
    r, c = i // g, i % g
    up = np.where(r > 0, i - g, -1)
    left = np.where(c > 0, i - 1, -1)
    pairs = np.stack([up, left], axis=1)  # per row: ascending columns
    mask = pairs >= 0
    rows = np.broadcast_to(i[:, None], pairs.shape)[mask]
    cols = pairs[mask]
    return assemble(f"stencil2d_{g}", n, rows, cols, rng, k)


def stencil3d(g: int, seed: int = 1, k: int = 1) -> System:
    """Lower triangle of the 7-point stencil on a g^3 grid, row
    ``i = (z*g + y)*g + x`` coupled to ``i-g*g``, ``i-g`` and ``i-1``."""
    rng = np.random.default_rng(seed)
    n = g * g * g
    i = np.arange(n, dtype=np.int64)
    x = i % g
    y = (i // g) % g
    z = i // (g * g)
    pairs = np.stack([np.where(z > 0, i - g * g, -1),
                      np.where(y > 0, i - g, -1),
                      np.where(x > 0, i - 1, -1)], axis=1)
    mask = pairs >= 0
    rows = np.broadcast_to(i[:, None], pairs.shape)[mask]
    cols = pairs[mask]
    return assemble(f"stencil3d_{g}", n, rows, cols, rng, k)


def banded(n: int, bw: int = 200, lo: int = 8, hi: int = 24, seed: int = 2,
           k: int = 1) -> System:
    """Random banded lower triangle.  Row ``i`` holds ``r_i ~ U{lo..hi}``
    entries including the diagonal; its ``min(r_i - 1, i)`` off-diagonals are
    a uniformly random subset of the columns ``[max(0, i-bw), i)``.

    The subset is drawn by sequential selection sampling (select candidate
    column ``c`` with probability needed/remaining), candidate columns
    visited in ascending order, vectorised over rows, one uniform per
    (row, candidate slot)."""
    rng = np.random.default_rng(seed)
    r = rng.integers(lo, hi + 1, size=n)
    i = np.arange(n, dtype=np.int64)
    need = np.minimum(r - 1, i).astype(np.int64)
    chosen = np.zeros((n, bw), dtype=bool)
    for t in range(bw):  # slot t <-> column i - bw + t
        u = rng.random(n)
        valid = t >= (bw - i)
        remaining = bw - t
        take = valid & (u * remaining < need)
        chosen[:, t] = take
        need -= take
    rows, slots = np.nonzero(chosen)
    cols = rows - bw + slots
    del chosen
    return assemble(f"banded_{n}_{bw}", n, rows, cols, rng, k)


def powerlaw(n: int, tail: int = 20_000, cap: int = 64, a: float = 1.8,
             seed: int = 3, k: int = 1) -> System:
    """Power-law DAG with a serial tail.

    * ``l_i = min(zipf(a), cap)`` is the length of row ``i`` including the
      diagonal.
    * Bulk rows ``i < n - tail`` draw ``min(l_i - 1, i)`` predecessors
      uniformly from ``[0, i)`` with replacement; duplicates collapse.
    * The tail rows are cut into consecutive groups of width U{1..4}.  Each
      tail row takes one predecessor uniformly from the previous group (the
      first group hangs off the last bulk row), plus ``max(l_i - 2, 0)``
      predecessors drawn uniformly from the bulk with replacement.
    """
    if tail >= n:
        raise ValueError("tail must be shorter than n")
    rng = np.random.default_rng(seed)
    ell = np.minimum(rng.zipf(a, size=n), cap).astype(np.int64)
    nb = n - tail
    # bulk
    ib = np.arange(nb, dtype=np.int64)
    kb = np.minimum(ell[:nb] - 1, ib)
    rows_b = np.repeat(ib, kb)
    u = rng.random(rows_b.size)
    cols_b = np.minimum((u * rows_b).astype(np.int64), rows_b - 1)
    # tail groups
    widths = rng.integers(1, 5, size=tail)
    ends = np.cumsum(widths)
    ngroups = int(np.searchsorted(ends, tail)) + 1
    starts = np.concatenate([[0], ends[:ngroups - 1]])
    starts = nb + starts
    it = np.arange(nb, n, dtype=np.int64)
    gid = np.searchsorted(starts, it, side="right") - 1
    prev_start = np.where(gid > 0, starts[np.maximum(gid - 1, 0)], nb - 1)
    prev_width = np.where(gid > 0, starts[np.maximum(gid, 0)] - prev_start, 1)
    u = rng.random(tail)
    chain = prev_start + np.minimum((u * prev_width).astype(np.int64), prev_width - 1)
    kt = np.maximum(ell[nb:] - 2, 0)
    rows_t = np.repeat(it, kt)
    u = rng.random(rows_t.size)
    cols_t = np.minimum((u * nb).astype(np.int64), nb - 1)
    rows = np.concatenate([rows_b, it, rows_t])
    cols = np.concatenate([cols_b, chain, cols_t])
    key = np.unique(rows * n + cols)  # sorts row-major and drops duplicates
    rows, cols = key // n, key % n
    return assemble(f"powerlaw_{n}_{tail}", n, rows, cols, rng, k)


# ---------------------------------------------------------- small helpers --

def from_pairs(n: int, pairs, seed: int = 0, k: int = 1, name: str = "pairs") -> System:
    """Matrix with the given strictly-lower (row, col) positions (any order,
    duplicates ignored) and values by the module's value rule."""
    rng = np.random.default_rng(seed)
    pairs = np.asarray(list(pairs), dtype=np.int64).reshape(-1, 2)
    if pairs.size and (np.any(pairs[:, 1] >= pairs[:, 0]) or np.any(pairs[:, 1] < 0)):
        raise ValueError("pairs must be strictly lower triangular")
    key = np.unique(pairs[:, 0] * max(n, 1) + pairs[:, 1]) if pairs.size else np.zeros(0, np.int64)
    return assemble(name, n, key // max(n, 1), key % max(n, 1), rng, k)


def random_lower(n: int, density: float, seed: int = 0, k: int = 1) -> System:
    """Each strictly-lower position present independently with probability
    ``density`` (drawn row by row)."""
    rng = np.random.default_rng(seed)
    ii, jj = np.tril_indices(n, -1)
    keep = rng.random(ii.size) < density
    order = np.lexsort((jj[keep], ii[keep]))
    return assemble(f"random_{n}_{density}", n, ii[keep][order], jj[keep][order], rng, k)


def bidiagonal(n: int, seed: int = 0) -> System:
    """Chain: row i depends on row i-1 only."""
    i = np.arange(1, n, dtype=np.int64)
    return assemble(f"bidiagonal_{n}", n, i, i - 1, np.random.default_rng(seed))


def diagonal(n: int, seed: int = 0) -> System:
    """No off-diagonal entries at all."""
    e = np.zeros(0, dtype=np.int64)
    return assemble(f"diagonal_{n}", n, e, e, np.random.default_rng(seed))


def transpose(s: System, name: str | None = None) -> System:
    """The upper-triangular transpose U = L^T of a lower system (CSR with the
    diagonal first in each row), keeping its right-hand sides."""
    n = s.n
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(s.row_ptr))
    order = np.lexsort((rows, s.col_idx.astype(np.int64)))  # by column, then row
    t_rows = s.col_idx[order].astype(np.int64)
    t_cols = rows[order].astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(t_rows, minlength=n), out=row_ptr[1:])
    return System(name or s.name + "_T", row_ptr.astype(np.int32), t_cols, s.val[order], s.b)


def batch_corpus(count: int = 64, nmin: int = 1_000, nmax: int = 200_000, ks=(1, 4, 8, 32),
                 seed: int = 4) -> list:
    """Many systems of uneven size: n log-uniform in [nmin, nmax], family
    uniform over {2D stencil, 3D stencil, banded, power-law}, and k drawn
    from ``ks`` right-hand sides (row-major n x k).  System j is drawn from
    seed 40000 + j (the family, size and k of all systems from ``seed``)."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        n = int(np.exp(rng.uniform(np.log(nmin), np.log(nmax))))
        fam = int(rng.integers(0, 4))
        k = int(rng.choice(ks))
        sd = 40000 + j
        if fam == 0:
            s = stencil2d(max(2, int(round(n ** 0.5))), seed=sd, k=k)
        elif fam == 1:
            s = stencil3d(max(2, int(round(n ** (1 / 3)))), seed=sd, k=k)
        elif fam == 2:
            s = banded(n, min(200, max(1, n // 2)), 8, 24, seed=sd, k=k)
        else:
            s = powerlaw(n, max(1, n // 200), seed=sd, k=k)
        if k == 1:
            s.b = s.b.reshape(-1, 1)
        out.append(s)
    return out


# ------------------------------------------------------ named workloads --

def fp32_valued(s: System, k: int = 1, b_seed: int | None = None) -> System:
    """The same structure with every value rounded to the nearest FP32 (ties
    to even) and held in FP64: that FP32-valued matrix is the problem, so an
    FP32 copy of it is exact.  With ``b_seed``, ``k`` new right-hand sides
    are drawn from ``default_rng(b_seed)``; else ``s.b`` is kept."""
    val = s.val.astype(np.float32).astype(np.float64)
    b = s.b if b_seed is None else rhs(s.n, np.random.default_rng(b_seed), k)
    return System(s.name + "_fp32", s.row_ptr, s.col_idx, val, b)


CONFIGS = {
    # small workload: the oracle finishes it in milliseconds
    "stencil2d_100": lambda: stencil2d(100, seed=0),
    # large workload: three matrices solved in one step
    "stencil3d_128": lambda: stencil3d(128, seed=1),
    "banded_1m": lambda: banded(1_000_000, 200, 8, 24, seed=2),
    "powerlaw_4m": lambda: powerlaw(4_000_000, 20_000, seed=3),
    # precision workload: the power-law matrix with FP32 values, 8 right-hand sides
    "powerlaw_4m_fp32_k8": lambda: fp32_valued(powerlaw(4_000_000, 20_000, seed=3), k=8, b_seed=5),
}


def config(name: str) -> System:
    """One of the named workloads in :data:`CONFIGS`."""
    return CONFIGS[name]()
