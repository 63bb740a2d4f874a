"""Exact rational arithmetic used to pin the oracle (tests only).

Everything here works on dense ``fractions.Fraction`` matrices built from the
exact binary values of the FP64 inputs, and uses *different* algorithms from
the oracle: Gauss-Jordan elimination on the full augmented matrix instead of
row-oriented forward substitution, a linear-system characterisation of a
rewritten row instead of the descending substitution worklist, and path
enumeration instead of the one-pass level recurrence.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def dense(row_ptr, col_idx, val):
    n = len(row_ptr) - 1
    A = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        for p in range(row_ptr[i], row_ptr[i + 1]):
            A[i][int(col_idx[p])] = Fraction(float(val[p]))
    return A


def gauss_jordan_solve(A, rhs):
    """Solve A y = rhs exactly (A square, non-singular) by Gauss-Jordan
    elimination with row pivoting on the first nonzero."""
    n = len(A)
    M = [list(A[i]) + [Fraction(rhs[i])] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        pv = M[c][c]
        M[c] = [e / pv for e in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    return [M[i][n] for i in range(n)]


def exact_solve(row_ptr, col_idx, val, b):
    A = dense(row_ptr, col_idx, val)
    return gauss_jordan_solve(A, [Fraction(float(v)) for v in b])


def longest_path_levels(row_ptr, col_idx):
    """Level of each row = number of edges on the longest dependency path that
    ends at it, found by enumerating every path (no memoisation)."""
    n = len(row_ptr) - 1
    preds = [[int(col_idx[p]) for p in range(row_ptr[i], row_ptr[i + 1]) if col_idx[p] < i]
             for i in range(n)]

    def longest(i):
        best = 0
        for j in preds[i]:
            best = max(best, 1 + longest(j))
        return best

    return [longest(i) for i in range(n)]


def exact_rewritten_row(A, i, in_stage):
    """Exact rewritten equation of row i when every row j < i with
    ``in_stage[j]`` is eliminated.

    The rewritten equation is row_i + sum_j m_j row_j (j over the in-stage
    rows before i) whose coefficient on each in-stage x_k is zero.  That is a
    triangular linear system for the m_j, solved here by Gauss-Jordan.
    Returns ({k: coeff of x_k, k out of stage, k < i}, {j: m_j}) keeping only
    nonzero entries."""
    T = [j for j in range(i) if in_stage[j]]
    if T:
        # unknowns m_j (j in T); equations: for k in T, A[i][k] + sum_j m_j A[j][k] = 0
        sys = [[A[j][k] for j in T] for k in T]
        m = gauss_jordan_solve(sys, [-A[i][k] for k in T])
    else:
        m = []
    mm = {j: mj for j, mj in zip(T, m) if mj != 0}
    coeffs = {}
    for k in range(i):
        if in_stage[k]:
            continue
        c = A[i][k] + sum(mj * A[j][k] for j, mj in mm.items())
        if c != 0:
            coeffs[k] = c
    return coeffs, mm


def all_lower_patterns(n):
    """Every strictly-lower sparsity pattern of an n x n matrix, as lists of
    (row, col) pairs."""
    slots = [(i, j) for i in range(n) for j in range(i)]
    for mask in range(1 << len(slots)):
        yield [slots[t] for t in range(len(slots)) if mask >> t & 1]


def rel_close(x: float, exact: Fraction, rel: float) -> bool:
    if exact == 0:
        return x == 0
    return abs(Fraction(float(x)) - exact) <= abs(exact) * Fraction(rel)


def ulp_diff(a: np.ndarray, b: np.ndarray) -> int:
    """Largest distance in units in the last place between two FP64 arrays
    of finite, same-sign values."""
    ia = np.asarray(a, dtype=np.float64).view(np.int64)
    ib = np.asarray(b, dtype=np.float64).view(np.int64)
    return int(np.max(np.abs(ia - ib))) if ia.size else 0
