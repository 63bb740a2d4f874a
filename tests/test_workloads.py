"""The seeded generators produce valid CSR lower-triangular systems with the
advertised shapes and value rule.  No GPU."""
import numpy as np
import pytest

import workloads as wl


def _check_csr(s):
    rp, ci, v = s.row_ptr, s.col_idx, s.val
    assert rp.dtype == np.int32 and ci.dtype == np.int32 and v.dtype == np.float64
    assert rp[0] == 0 and np.all(np.diff(rp) >= 1)
    rows = np.repeat(np.arange(s.n), np.diff(rp))
    assert np.all(ci <= rows)
    assert np.array_equal(ci[rp[1:] - 1], np.arange(s.n))  # diagonal last
    inner = np.ones(ci.size, bool)
    inner[rp[1:] - 1] = False
    starts = np.zeros(ci.size, bool)
    starts[rp[:-1]] = True
    asc = np.diff(ci) > 0
    assert np.all(asc | starts[1:])  # strictly increasing inside each row
    off = v[inner]
    assert np.all((off >= -0.25) & (off < 0))
    sums = np.bincount(rows[inner], weights=np.abs(off), minlength=s.n)
    assert np.array_equal(v[rp[1:] - 1], 1.0 + sums)
    assert np.all(np.abs(s.b) <= 1)


@pytest.mark.parametrize("make", [
    lambda: wl.stencil2d(17, seed=0), lambda: wl.stencil3d(9, seed=1),
    lambda: wl.banded(3000, 200, 8, 24, seed=2), lambda: wl.powerlaw(20000, 300, seed=3),
    lambda: wl.random_lower(50, 0.3, seed=4), lambda: wl.bidiagonal(10), lambda: wl.diagonal(10),
])
def test_valid_and_deterministic(make):
    s1, s2 = make(), make()
    _check_csr(s1)
    for a in ("row_ptr", "col_idx", "val", "b"):
        assert np.array_equal(getattr(s1, a), getattr(s2, a))


def test_family_shapes():
    s = wl.stencil2d(100, seed=0)
    assert s.n == 10000 and s.nnz == 29800
    s = wl.stencil3d(8, seed=0)
    assert s.nnz == 8 ** 3 + 3 * 8 * 8 * 7
    s = wl.banded(5000, 200, 8, 24, seed=2)
    rl = np.diff(s.row_ptr)
    assert rl[200:].min() >= 8 and rl.max() <= 24
    assert np.array_equal(rl[:8], np.arange(1, 9))  # row i < 8 keeps all i predecessors
    rows = np.repeat(np.arange(s.n), rl)
    assert np.all(rows - s.col_idx <= 200)
    s = wl.powerlaw(50000, 1000, seed=3)
    rl = np.diff(s.row_ptr)
    assert rl.max() <= 64 and 0.4 < (rl == 1).mean() < 0.65
    s = wl.stencil2d(5, seed=0, k=4)
    assert s.b.shape == (25, 4)
