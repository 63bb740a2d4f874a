"""GPU: plans stored in FP32 and mixed-precision refinement, through the C ABI.

* The FP32 solve is checked against the FP64 oracle solve of the same
  FP32-valued system with a componentwise bound derived from the rounding
  error analysis of substitution (Higham, Accuracy and Stability of Numerical
  Algorithms, Thm. 8.5, applied to the rewritten system): the computed x^
  solves a system whose every coefficient is perturbed by at most
  gamma_m = m u / (1 - m u) relatively, m the terms of a row plus two (the
  rounding of the coefficient to FP32, the division), so
  |x^ - x| <= gamma_m L'^{-1} (|L'| |x^| + |b| + |M| |b|).  L' has a positive
  diagonal and non-positive off-diagonals for the M-matrices generated here
  (rewriting adds non-positive multiples of non-positive entries), so
  L'^{-1} >= 0 and the bound is one more oracle solve.  The test allows
  twice the bound (first order in u: x stands in for x^).
* The refined solve must reach 1e-12 componentwise, floored at 1e-3 max|x|,
  against the long-double oracle rounded to FP64 (the FP64 oracle's own
  rounding error is ~1e-11 at these sizes, so it cannot be the reference at
  that level; the strict FP64-oracle error is printed beside it).
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from gate import errors

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
REFINED_TOL = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def sp():
    import paper_2103_11445_amd as m
    m.load()
    return m


POLICIES = [
    ("none", {}),
    ("threshold", {}),
    ("threshold", {"max_width": 10**9, "max_depth": 4, "max_fill": 10.0}),
    ("threshold", {"max_width": 10**9, "max_depth": 16, "max_fill": 12.0}),
]


def _row_ids(ptr):
    ptr = np.asarray(ptr, dtype=np.int64)
    return np.repeat(np.arange(ptr.size - 1), np.diff(ptr))


def fp32_bound(s, b, x, pol):
    """Componentwise bound on |x^ - x| for the FP32 solve of L x = b under
    policy ``pol`` (x the exact solution, approximated by the oracle)."""
    o = oracle.plan(s.row_ptr, s.col_idx, s.val, pol)
    (lp_ptr, lp_col, lp_val), (m_ptr, m_col, m_val) = o["lp"], o["m"]
    n = s.n
    rows = _row_ids(lp_ptr)
    diag = np.zeros(lp_val.size, dtype=bool)
    diag[np.asarray(lp_ptr[1:]) - 1] = True
    assert np.all(lp_val[~diag] <= 0) and np.all(lp_val[diag] > 0) and np.all(m_val >= 0)
    v = np.bincount(rows, weights=np.abs(lp_val) * np.abs(x)[lp_col], minlength=n)
    v += np.abs(b) + np.bincount(_row_ids(m_ptr), weights=m_val * np.abs(b)[m_col], minlength=n)
    empty = (np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float64))
    y = oracle.solve_rewritten(o["lp"], empty, v)
    terms = np.diff(lp_ptr) + np.diff(m_ptr) + 2
    m = int(terms.max())
    gamma = m * U32 / (1 - m * U32)
    return 2.0 * gamma * y


@pytest.mark.parametrize("make", [
    lambda: wl.stencil2d(60, seed=21),
    lambda: wl.stencil3d(20, seed=22),
    lambda: wl.banded(9001, 200, 8, 24, seed=23),
    lambda: wl.powerlaw(60000, 1500, seed=24),
    lambda: wl.random_lower(500, 0.5, seed=25),
    lambda: wl.bidiagonal(3000, seed=26),
])
@pytest.mark.parametrize("kind,kw", POLICIES)
def test_fp32_solve_within_rounding_bound(torch, sp, make, kind, kw):
    s = wl.fp32_valued(make())
    b32 = s.b.astype(np.float32)
    b = b32.astype(np.float64)            # the problem's right-hand side
    x = oracle.solve(s.row_ptr, s.col_idx, s.val, b)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val).set_precision(32).rewrite(kind, **kw).upload()
    bd = torch.from_numpy(b32).cuda()
    xd = torch.full_like(bd, float("nan"))
    plan.solve_fp32(bd, xd)
    assert plan.check() == 0
    xh = xd.cpu().numpy().astype(np.float64)
    bound = fp32_bound(s, b, x, {"kind": kind, **kw})
    err = np.abs(xh - x)
    ratio = float(np.max(err / np.maximum(bound, 1e-300)))
    print(s.name, kind, kw, "fp32 err/bound", ratio, "max rel", errors(xh, x)[1], flush=True)
    assert np.all(np.isfinite(xh)) and ratio <= 1.0


@pytest.mark.parametrize("tpl", [8, 16])
def test_fp32_solve_eight_register_chunks(torch, sp, tpl):
    """The kernel instance holding 8 chunks of a wide tile in registers (rows
    of 5..8 chunks, and longer ones streamed 8 chunks at a time), in FP32."""
    s = wl.fp32_valued(wl.banded(9001, 200, 8, 24, seed=27))
    b32 = s.b.astype(np.float32)
    b = b32.astype(np.float64)
    x = oracle.solve(s.row_ptr, s.col_idx, s.val, b)
    kw = {"max_width": 10**9, "max_depth": 16, "max_fill": 12.0}
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val).set_precision(32).rewrite("threshold", **kw)
    plan.set_tiling(tpl).upload()
    assert plan.info()["reg_chunks"] == 8
    bd = torch.from_numpy(b32).cuda()
    xd = torch.full_like(bd, float("nan"))
    plan.solve_fp32(bd, xd)
    assert plan.check() == 0
    xh = xd.cpu().numpy().astype(np.float64)
    ratio = float(np.max(np.abs(xh - x) / np.maximum(fp32_bound(s, b, x, {"kind": "threshold", **kw}), 1e-300)))
    print(s.name, tpl, "fp32 err/bound", ratio, flush=True)
    assert np.all(np.isfinite(xh)) and ratio <= 1.0


def _refine(torch, sp, plan, b, iterations=10, tol=1e-14):
    bd = torch.from_numpy(np.ascontiguousarray(b).reshape(-1)).cuda()
    xd = torch.full_like(bd, float("nan"))
    plan.solve_refined(bd, xd, iterations=iterations, tol=tol)
    assert plan.check() == 0
    return xd.cpu().numpy(), plan.refine_stats()


@pytest.mark.parametrize("kind,kw", POLICIES)
def test_refined_batch_k8(torch, sp, kind, kw):
    """One FP32-valued power-law matrix with 8 right-hand sides (a batched
    plan of 8 copies) refined to FP64 accuracy."""
    s = wl.fp32_valued(wl.powerlaw(60000, 1500, seed=27), k=8, b_seed=5)
    ref = oracle.solve_ld(s.row_ptr, s.col_idx, s.val, s.b)
    ref64 = oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
    plan = sp.Plan.batch([(s.row_ptr, s.col_idx, s.val)], [8]).set_precision(32).rewrite(kind, **kw).upload()
    x, (it, corr) = _refine(torch, sp, plan, s.b)
    x = x.reshape(s.n, 8)
    strict, floored = errors(x, ref)
    print(s.name, kind, kw, "iterations", it, "correction", corr, "vs long double", floored,
          "strict", strict, "vs FP64 oracle", errors(x, ref64), flush=True)
    assert 2 <= it <= 10
    assert floored <= REFINED_TOL


@pytest.mark.parametrize("upper", [False, True])
def test_refined_single_system(torch, sp, upper):
    s = wl.fp32_valued(wl.stencil3d(24, seed=28))
    if upper:
        s = wl.transpose(s)
        ref = oracle.solve_upper(s.row_ptr, s.col_idx, s.val, s.b)
    else:
        ref = oracle.solve_ld(s.row_ptr, s.col_idx, s.val, s.b)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val, upper=upper).set_precision(32)
    plan.rewrite("threshold", max_width=10**9, max_depth=4, max_fill=10.0).upload()
    x, (it, corr) = _refine(torch, sp, plan, s.b)
    print(s.name, "upper" if upper else "lower", it, corr, errors(x, ref), flush=True)
    assert it >= 2
    # the backward-substitution reference is the FP64 oracle (no long-double
    # variant); its rounding error is far below 1e-10 at this size
    assert errors(x, ref)[1] <= (1e-10 if upper else REFINED_TOL)


def test_refined_uneven_batch(torch, sp):
    """Systems of different sizes and right-hand-side counts in one plan:
    the residual finds each entry's system and column."""
    corp = [wl.fp32_valued(s) for s in wl.batch_corpus(6, nmin=200, nmax=20000, ks=(1, 3, 8), seed=29)]
    ks = [1 if s.b.ndim == 1 else s.b.shape[1] for s in corp]
    plan = sp.Plan.batch([(s.row_ptr, s.col_idx, s.val) for s in corp], ks).set_precision(32)
    plan.rewrite("threshold", max_width=10**9, max_depth=8, max_fill=12.0).upload()
    b = np.concatenate([s.b.reshape(-1) for s in corp])
    x, (it, corr) = _refine(torch, sp, plan, b)
    off = 0
    for s, k in zip(corp, ks):
        ref = oracle.solve_ld(s.row_ptr, s.col_idx, s.val, s.b).reshape(-1)
        part = x[off:off + s.n * k]
        off += s.n * k
        print(s.name, k, errors(part, ref), flush=True)
        assert errors(part, ref)[1] <= REFINED_TOL
    assert it >= 2


def test_refined_single_step_is_the_fp32_solve(torch, sp):
    """One step: x is the FP32 solve of b rounded to FP32, widened."""
    s = wl.fp32_valued(wl.powerlaw(30000, 800, seed=30))
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val).set_precision(32)
    plan.rewrite("threshold", max_width=10**9, max_depth=4, max_fill=10.0).upload()
    x, (it, corr) = _refine(torch, sp, plan, s.b, iterations=1)
    b32 = torch.from_numpy(s.b.astype(np.float32)).cuda()
    x32 = plan.solve_fp32(b32).cpu().numpy()
    assert it == 1 and corr == float("inf")
    assert np.array_equal(x, x32.astype(np.float64))


def test_refined_timeout_then_recover(torch, sp):
    """A wait limit of zero makes the waits give up: the status word says so
    and the steps never count as converged; with the default limit the next
    call is correct again."""
    s = wl.fp32_valued(wl.stencil3d(24, seed=31))
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val).set_precision(32).upload()
    plan.set_wait_limit(0)
    bd = torch.from_numpy(s.b).cuda()
    xd = torch.empty_like(bd)
    plan.solve_refined(bd, xd, iterations=3)
    it, corr = plan.refine_stats()
    assert plan.check() == 8  # SPTRSV_ERR_TIMEOUT
    assert corr > 1e-13
    plan.set_wait_limit(200_000_000)
    x, (it, corr) = _refine(torch, sp, plan, s.b)
    ref = oracle.solve_ld(s.row_ptr, s.col_idx, s.val, s.b)
    assert errors(x, ref)[1] <= REFINED_TOL
