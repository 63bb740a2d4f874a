"""GPU parity of the two right-hand-side steps (b' = b + M b by a pass over
M, or by solves of the stages' diagonal blocks of L): every plan solved both
ways against the FP64 oracle, lower, upper, batched and FP32-refined."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gate import TOL, errors

pytestmark = pytest.mark.gpu

INF = 10**9
POLICIES = [
    ("threshold", {}),
    ("threshold", {"max_width": INF, "max_depth": 4, "max_fill": 10.0}),
    ("threshold", {"max_width": INF, "max_depth": 64, "max_fill": 40.0}),
]


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


@pytest.mark.parametrize("mode", ["mpass", "stage"])
@pytest.mark.parametrize("make", [
    lambda: wl.stencil3d(24, seed=51),
    lambda: wl.banded(20011, 200, 8, 24, seed=52),
    lambda: wl.powerlaw(100003, 1501, seed=53),
    lambda: wl.random_lower(700, 0.6, seed=54),
    lambda: wl.bidiagonal(4099, seed=55),
])
@pytest.mark.parametrize("kind,kw", POLICIES)
def test_modes_match_oracle(torch, sp, make, kind, kw, mode):
    s = make()
    ref = oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite(kind, **kw).set_rhs_mode(mode).upload()
    b = torch.from_numpy(s.b).cuda()
    x = plan.solve(b)
    assert plan.check() == 0
    info = plan.info()
    err = errors(x.cpu().numpy(), ref)
    print(s.name, kind, kw, mode, info["rhs_mode"], info["levels_rw"], err, flush=True)
    assert info["rhs_mode"] in ((1 if mode == "mpass" else 2), 0)
    assert err[1] <= TOL


@pytest.mark.parametrize("mode", ["mpass", "stage"])
def test_modes_upper_batched_graph(torch, sp, mode):
    """Backward substitution and a batched plan through a captured graph."""
    U = wl.transpose(wl.banded(9001, 200, 8, 24, seed=56))
    plan = sp.Plan(U.row_ptr, U.col_idx, U.val, upper=True)
    plan.rewrite("threshold", max_width=INF, max_depth=16, max_fill=12.0).set_rhs_mode(mode).upload()
    x = plan.solve(torch.from_numpy(U.b).cuda())
    assert plan.check() == 0
    assert errors(x.cpu().numpy(), oracle.solve_upper(U.row_ptr, U.col_idx, U.val, U.b))[1] <= TOL
    corp = wl.batch_corpus(5, nmin=300, nmax=20000, ks=(1, 3, 8), seed=57)
    ks = [1 if c.b.ndim == 1 else c.b.shape[1] for c in corp]
    bp = sp.Plan.batch([(c.row_ptr, c.col_idx, c.val) for c in corp], ks)
    bp.rewrite("threshold", max_width=INF, max_depth=16, max_fill=12.0).set_rhs_mode(mode).upload()
    bcat = torch.from_numpy(np.concatenate([c.b.reshape(-1) for c in corp])).cuda()
    xg = torch.empty_like(bcat)
    for _ in range(3):
        bp.solve_graph(bcat, xg)
        torch.cuda.synchronize()
    assert bp.check() == 0
    got, off = xg.cpu().numpy(), 0
    for c, k in zip(corp, ks):
        ref = oracle.solve(c.row_ptr, c.col_idx, c.val, c.b).reshape(-1)
        assert errors(got[off:off + c.n * k], ref)[1] <= TOL
        off += c.n * k


@pytest.mark.parametrize("mode", ["mpass", "stage"])
def test_modes_refined(torch, sp, mode):
    s = wl.fp32_valued(wl.powerlaw(60000, 1500, seed=58), k=8, b_seed=5)
    ref = oracle.solve_ld(s.row_ptr, s.col_idx, s.val, s.b)
    plan = sp.Plan.batch([(s.row_ptr, s.col_idx, s.val)], [8]).set_precision(32)
    plan.rewrite("threshold", max_width=INF, max_depth=16, max_fill=12.0).set_rhs_mode(mode).upload()
    b = torch.from_numpy(np.ascontiguousarray(s.b).reshape(-1)).cuda()
    x = plan.solve_refined(b, iterations=10, tol=1e-14)
    assert plan.check() == 0
    it, _ = plan.refine_stats()
    err = errors(x.cpu().numpy().reshape(s.n, 8), ref)
    print(mode, plan.info()["rhs_mode"], it, err, flush=True)
    assert err[1] <= 1e-12


def test_stage_mode_timeout_reported(torch, sp):
    """A wait that gives up inside the stage system's solve is reported by
    the plan's status word like one in the main solve."""
    s = wl.stencil3d(24, seed=59)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite("threshold", max_width=INF, max_depth=8, max_fill=12.0)
    plan.set_rhs_mode("stage").upload()
    plan.set_wait_limit(0)
    b = torch.from_numpy(s.b).cuda()
    plan.solve(b)
    assert plan.check() == 8
    plan.set_wait_limit(200_000_000)
    x = plan.solve(b)
    assert plan.check() == 0
    assert errors(x.cpu().numpy(), oracle.solve(s.row_ptr, s.col_idx, s.val, s.b))[1] <= TOL


@pytest.mark.parametrize("tpl", [1, 2, 8, 16])
@pytest.mark.parametrize("make", [
    lambda: wl.stencil3d(24, seed=61),
    lambda: wl.banded(20011, 200, 8, 24, seed=62),
    lambda: wl.powerlaw(100003, 1501, seed=63),
    lambda: wl.random_lower(700, 0.6, seed=64),
])
def test_tilings_match_oracle(torch, sp, make, tpl):
    """Every row-to-wavefront tiling solves to the gate (rows over 1..64
    lanes, up to 16 chunks a row)."""
    s = make()
    ref = oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite("threshold", max_width=INF, max_depth=8, max_fill=12.0)
    plan.set_tiling(tpl).upload()
    x = plan.solve(torch.from_numpy(s.b).cuda())
    assert plan.check() == 0
    err = errors(x.cpu().numpy(), ref)
    print(s.name, tpl, plan.info()["tiles"], plan.info()["reg_chunks"], err, flush=True)
    assert err[1] <= TOL


@pytest.mark.parametrize("tpl", [1, 4, 16])
@pytest.mark.parametrize("kind,kw", [
    ("none", {}),
    ("threshold", {"max_width": 10**9, "max_depth": 4, "max_fill": 10.0}),
    ("threshold", {"max_width": 10**9, "max_depth": 64, "max_fill": 40.0}),
], ids=["plain", "depth4", "depth64"])
def test_shared_copy_terms(torch, sp, tpl, kind, kw):
    """Batched systems with 2, 5, 16 and 64 right-hand sides: the copies of a
    row (power-of-two k) share copy 0's terms in the tiles, whether a row's
    copies share a tile (k below the rows per tile) or one row's copies span
    several tiles (k above it); k = 5 keeps a copy of the terms per row.
    Every column against the oracle."""
    corp = wl.batch_corpus(8, nmin=300, nmax=15000, ks=(2, 5, 16, 64), seed=60)
    ks = [c.b.shape[1] for c in corp]
    assert {2, 5, 16, 64} <= set(ks)
    plan = sp.Plan.batch([(c.row_ptr, c.col_idx, c.val) for c in corp], ks)
    plan.rewrite(kind, **kw).set_tiling(tpl).upload()
    b = torch.from_numpy(np.concatenate([c.b.reshape(-1) for c in corp])).cuda()
    x = torch.full_like(b, float("nan"))
    plan.solve(b, x)
    assert plan.check() == 0
    got, off = x.cpu().numpy(), 0
    for c in corp:
        k = c.b.shape[1]
        ref = oracle.solve(c.row_ptr, c.col_idx, c.val, c.b)
        err = errors(got[off:off + c.n * k].reshape(c.n, k), ref)
        print(c.name, k, tpl, kind, kw.get("max_depth"), plan.info()["rhs_mode"], err, flush=True)
        assert err[1] <= TOL, (c.name, k)
        off += c.n * k
    plan.close()
