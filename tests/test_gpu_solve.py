"""GPU parity: the HIP solve (through the C ABI) against the CPU oracle, on
the same seeded inputs, elementwise, max componentwise relative error
<= 1e-10 against the FP64 serial substitution."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

from gate import TOL, errors


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


def relerr(x, ref):
    """Floored componentwise relative error (see tests/gate.py)."""
    return errors(x, ref)[1]


def gpu_solve(torch, sp, s, kind="none", reps=1, **kw):
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite(kind, **kw).upload()
    b = torch.from_numpy(np.ascontiguousarray(s.b)).cuda()
    outs = []
    for _ in range(reps):
        x = torch.full_like(b, float("nan"))
        plan.solve(b, x)
        outs.append(x.cpu().numpy())
    assert plan.check() == 0
    return outs, plan


POLICIES = [
    ("none", {}),
    ("threshold", {}),
    ("threshold", {"max_width": 16, "max_depth": 64, "max_fill": 1.0}),
    ("threshold", {"max_width": 10**9, "max_depth": 4, "max_fill": 10.0}),
]


@pytest.mark.parametrize("kind,kw", POLICIES)
def test_stencil2d_small(torch, sp, kind, kw):
    s = wl.stencil2d(100, seed=0)
    ref = oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
    (x,), plan = gpu_solve(torch, sp, s, kind, **kw)
    print(s.name, kind, kw, plan.info()["levels_rw"], relerr(x, ref), flush=True)
    assert relerr(x, ref) <= TOL


@pytest.mark.parametrize("make", [
    lambda: wl.stencil3d(24, seed=11),
    lambda: wl.banded(20011, 200, 8, 24, seed=12),
    lambda: wl.powerlaw(100003, 1501, seed=13),
    lambda: wl.random_lower(700, 0.6, seed=14),   # rows of hundreds of terms
    lambda: wl.bidiagonal(4099, seed=15),          # one long chain
    lambda: wl.diagonal(1000, seed=16),
    lambda: wl.from_pairs(1, [], seed=17),
    lambda: wl.from_pairs(65, [(64, j) for j in range(64)], seed=18),
])
@pytest.mark.parametrize("kind,kw", POLICIES)
def test_families(torch, sp, make, kind, kw):
    s = make()
    ref = oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
    (x,), plan = gpu_solve(torch, sp, s, kind, **kw)
    print(s.name, kind, kw, plan.info()["levels_rw"], relerr(x, ref), flush=True)
    assert relerr(x, ref) <= TOL


def test_rewritten_matches_oracle_rewritten_solve(torch, sp):
    """The GPU solve of L' x = b + M b agrees with the oracle's serial solve of
    the oracle's own rewritten system."""
    s = wl.powerlaw(60000, 3000, seed=21)
    pol = {"kind": "threshold", "max_width": 4, "max_depth": 64, "max_fill": 0.25}
    o = oracle.plan(s.row_ptr, s.col_idx, s.val, pol)
    ref = oracle.solve_rewritten(o["lp"], o["m"], s.b)
    (x,), plan = gpu_solve(torch, sp, s, "threshold", max_width=4, max_depth=64, max_fill=0.25)
    assert plan.info()["levels_rw"] == o["nlev_rw"]
    assert relerr(x, ref) <= TOL


def test_deterministic_and_no_sentinel(torch, sp):
    """Each row's reduction order is fixed by the packing, so repeated solves
    are bitwise identical; no output keeps the not-ready pattern."""
    s = wl.powerlaw(50000, 2000, seed=22)
    outs, _ = gpu_solve(torch, sp, s, "threshold", reps=20)
    for o in outs[1:]:
        assert np.array_equal(o.view(np.int64), outs[0].view(np.int64))
    assert np.all(np.isfinite(outs[0]))


def test_empty_system(torch, sp):
    s = wl.from_pairs(0, [], seed=0)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val)
    plan.upload()
    b = torch.zeros(0, dtype=torch.float64, device="cuda")
    x = plan.solve(b)
    assert x.numel() == 0


def test_wait_limit_reports_timeout_and_recovers(torch, sp):
    """A wait limit of 0 ticks makes every cross-wave wait that is not
    satisfied on its first poll give up: the kernel still drains, the status
    word reports a timeout, and the next solve with a normal limit is
    correct.  (Wide levels, so that rows wait on other waves.)"""
    s = wl.stencil3d(24, seed=23)
    ref = oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val).upload()
    b = torch.from_numpy(s.b).cuda()
    plan.set_wait_limit(0)
    plan.solve(b)
    assert plan.check() == 8  # SPTRSV_ERR_TIMEOUT
    plan.set_wait_limit(200_000_000)
    x = plan.solve(b)
    assert plan.check() == 0
    assert relerr(x.cpu().numpy(), ref) <= TOL


def test_solve_state_errors(torch, sp):
    s = wl.stencil2d(10, seed=1)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val)
    b = torch.from_numpy(s.b).cuda()
    with pytest.raises(sp.SptrsvError) as e:
        plan.solve(b)
    assert e.value.status == "ERR_STATE"
    plan.upload()
    with pytest.raises(sp.SptrsvError) as e:
        plan.solve(b, b)
    assert e.value.status == "ERR_ARG"
    plan.rewrite("threshold")
    with pytest.raises(sp.SptrsvError) as e:
        plan.solve(b)
    assert e.value.status == "ERR_STATE"


@pytest.mark.parametrize("make", [lambda: wl.stencil3d(20, seed=31), lambda: wl.banded(8000, 200, 8, 24, seed=32),
                                  lambda: wl.powerlaw(60000, 1500, seed=33)])
@pytest.mark.parametrize("kind,kw", POLICIES)
def test_upper_backward_substitution(torch, sp, make, kind, kw):
    """U x = b with U = L^T (backward substitution) against the oracle's
    backward substitution."""
    U = wl.transpose(make())
    ref = oracle.solve_upper(U.row_ptr, U.col_idx, U.val, U.b)
    plan = sp.Plan(U.row_ptr, U.col_idx, U.val, upper=True).rewrite(kind, **kw).upload()
    b = torch.from_numpy(U.b).cuda()
    x = plan.solve(b)
    assert plan.check() == 0
    assert relerr(x.cpu().numpy(), ref) <= TOL


# -------------------------------------------------------------- batches --

def _batch_rhs(corp):
    return np.concatenate([s.b.reshape(-1) for s in corp])


def _batch_refs(corp):
    return [oracle.solve(s.row_ptr, s.col_idx, s.val, s.b) for s in corp]


def _check_batch(corp, xall):
    off = 0
    for s, ref in zip(corp, _batch_refs(corp)):
        k = s.b.shape[1]
        got = xall[off:off + s.n * k].reshape(s.n, k)
        off += s.n * k
        assert relerr(got, ref.reshape(s.n, k)) <= TOL, s.name


@pytest.mark.parametrize("kind,kw", POLICIES)
def test_batch_parity(torch, sp, kind, kw):
    """Many uneven systems with 1..32 right-hand sides, one launch."""
    corp = wl.batch_corpus(16, nmin=500, nmax=20000, seed=41)
    plan = sp.Plan.batch([(s.row_ptr, s.col_idx, s.val) for s in corp], [s.b.shape[1] for s in corp])
    plan.rewrite(kind, **kw).upload()
    b = torch.from_numpy(_batch_rhs(corp)).cuda()
    x = plan.solve(b)
    assert plan.check() == 0
    _check_batch(corp, x.cpu().numpy())


def test_graph_replays_match_eager(torch, sp):
    """The captured solve, replayed several times with eager work and
    synchronisations in between, gives the eager result every time."""
    corp = wl.batch_corpus(10, nmin=500, nmax=10000, seed=42)
    plan = sp.Plan.batch([(s.row_ptr, s.col_idx, s.val) for s in corp], [s.b.shape[1] for s in corp])
    plan.rewrite("threshold", max_width=10**9, max_depth=4, max_fill=10.0).upload()
    b = torch.from_numpy(_batch_rhs(corp)).cuda()
    eager = plan.solve(b).cpu().numpy()
    x = torch.empty_like(b)
    for rep in range(5):
        x.fill_(float("nan"))
        y = torch.randn(1000, device="cuda").sum()  # unrelated eager work
        plan.solve_graph(b, x)
        torch.cuda.synchronize()
        assert float(y) == float(y)
        got = x.cpu().numpy()
        assert np.array_equal(got.view(np.int64), eager.view(np.int64)), rep
    assert plan.check() == 0
    _check_batch(corp, eager)


def test_hop_probe(torch, sp):
    """The hop probe returns a plausible latency for both placements: above
    the 10 ns clock tick, below a millisecond, and the same-XCD hop is not
    several times slower than the cross-XCD one."""
    cross = sp.probe_hop(4000, same_xcd=False)
    same = sp.probe_hop(4000, same_xcd=True)
    print("hop ns: cross-XCD", cross, "same-XCD", same, flush=True)
    for v in (cross, same):
        assert 10.0 < v < 1e6
    assert same < 4 * cross


@pytest.mark.parametrize("make,pol", [
    (lambda: wl.stencil3d(40, seed=1), {"max_width": 10**9, "max_depth": 4, "max_fill": 12.0}),
    (lambda: wl.banded(60000, 200, 8, 24, seed=2), {"max_width": 10**9, "max_depth": 64, "max_fill": 40.0}),
    (lambda: wl.powerlaw(300000, 3000, seed=3), {"max_width": 4, "max_depth": 256, "max_fill": 1.0}),
], ids=["stencil3d", "banded", "powerlaw"])
def test_chain_waves_sweep_bitwise(torch, sp, make, pol):
    """Chain and sink queues on separate waves: any split of the waves, and
    one queue of every row in level order, give the oracle's solution to the
    gate and the same bits (each row's summation order is fixed by its
    length and the tiling, whichever tile and wave run it)."""
    s = make()
    ref = oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite("threshold", **pol).upload()
    info = plan.info()
    assert 0 < info["chain_items"] < info["tiles"]
    b = torch.from_numpy(s.b).cuda()
    first = None
    for q, cw in ((2, 0), (2, 1), (2, 125), (2, 500), (2, 875), (2, 1000), (1, 0)):
        if q == 1:
            plan.set_queues(1)
            plan._buf = None
            plan.upload()
        plan.set_chain_share(cw)
        x = torch.full_like(b, float("nan"))
        plan.solve(b, x)
        assert plan.check() == 0
        got = x.cpu().numpy()
        print(s.name, "queues", q, "chain share", cw, plan.launch_shape(), relerr(got, ref), flush=True)
        assert relerr(got, ref) <= TOL
        if first is None:
            first = got
        assert np.array_equal(got, first), cw
    plan.close()


@pytest.mark.parametrize("make,pol,tpl", [
    (lambda: wl.banded(60000, 200, 8, 24, seed=2), {"max_width": 10**9, "max_depth": 64, "max_fill": 40.0}, 8),
    (lambda: wl.banded(20000, 200, 8, 24, seed=7), {"max_width": 10**9, "max_depth": 512, "max_fill": 140.0}, 4),
    (lambda: wl.stencil2d(150, seed=5), {"max_width": 10**9, "max_depth": 4, "max_fill": 12.0}, 2),
    (lambda: wl.random_lower(3000, 0.01, seed=9), {"max_width": 10**9, "max_depth": 8, "max_fill": 12.0}, 4),
], ids=["banded-64", "banded-512", "stencil2d", "random"])
def test_compact_columns_bitwise(torch, sp, monkeypatch, make, pol, tpl):
    """Wide tiles that store each column as a 16-bit distance back from the
    tile's first slot give the same bits as 32-bit columns, in the plain and
    in the instrumented solve, and the oracle's solution to the gate."""
    s = make()
    ref = oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
    b = torch.from_numpy(s.b).cuda()
    got = {}
    for env in ("", "0"):
        monkeypatch.setenv("SPTRSV_COMPACT_COLS", env)
        plan = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite("threshold", **pol).set_tiling(tpl).upload()
        info = plan.info()
        assert info["compact_cols"] == (0 if env == "0" else 1), (env, info["compact_cols"])
        x = torch.full_like(b, float("nan"))
        plan.solve(b, x)
        assert plan.check() == 0
        xs = torch.full_like(b, float("nan"))
        stamps = torch.empty(info["tiles"] + info["seg_tiles"] + 1, dtype=torch.int64, device="cuda")
        plan.solve_stamped(b, xs, stamps)
        assert plan.check() == 0
        got[env] = (x.cpu().numpy(), xs.cpu().numpy())
        print(s.name, "compact" if info["compact_cols"] else "32-bit", info["compact_terms"],
              relerr(got[env][0], ref), flush=True)
        assert relerr(got[env][0], ref) <= TOL
        assert np.array_equal(got[env][0], got[env][1])
        plan.close()
    assert np.array_equal(got[""][0], got["0"][0])


def _csr_from_rows(rows):
    """CSR (diagonal last in each row) from a list of [(col, val), ...]."""
    ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([c for r in rows for c, _ in r], dtype=np.int32)
    val = np.array([v for r in rows for _, v in r], dtype=np.float64)
    return ptr, col, val


def test_row_arithmetic_bits_match_ieee(torch, sp):
    """A row ends with x_i = (b_i + sum_k -L_ik x_k) / L_ii.  Where the sum's
    order is fixed, the kernel's result must carry the bits of the same
    operations done one by one in IEEE FP64: a diagonal system (wide tiles,
    one ragged; x_i = (b_i + 0) / d_i), with signed zeros, subnormals,
    overflow and extreme diagonals, and a bidiagonal chain run as ring-only
    segments (x_i = (b_i + RN(-l_i x_{i-1})) / d_i)."""
    rng = np.random.default_rng(17)
    n = 100_003
    d = rng.uniform(0.5, 2.0, n) * np.exp2(rng.integers(-40, 41, n)) * rng.choice([-1.0, 1.0], n)
    b = rng.uniform(0.5, 2.0, n) * np.exp2(rng.integers(-40, 41, n)) * rng.choice([-1.0, 1.0], n)
    edge = [(0.0, 3.0), (-0.0, 3.0), (1e-310, 1.5), (-4e-320, 0.75), (1e308, 1e-10), (3.0, 1e-300),
            (3.0, 1e300), (-2.5, 7e-145), (2.5, 5e144), (1.0, 3.0), (-7.0, 3.0)]
    for k, (bv, dv) in enumerate(edge):
        b[1000 * k + 7], d[1000 * k + 7] = bv, dv
    ptr, col, val = _csr_from_rows([[(i, d[i])] for i in range(n)])
    plan = sp.Plan(ptr, col, val).upload()
    x = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    with np.errstate(over="ignore"):
        want = (b + 0.0) / d
    plan.solve(torch.from_numpy(b).cuda(), x)
    got = x.cpu().numpy()
    assert plan.check() == 0
    assert np.array_equal(got.view(np.int64), want.view(np.int64))

    m = 6_000
    dd = rng.uniform(0.5, 2.0, m) * rng.choice([-1.0, 1.0], m)
    ll = rng.uniform(-1.0, 1.0, m)
    bb = rng.uniform(-1.0, 1.0, m)
    rows = [[(0, dd[0])]] + [[(i - 1, ll[i]), (i, dd[i])] for i in range(1, m)]
    ptr, col, val = _csr_from_rows(rows)
    plan = sp.Plan(ptr, col, val).upload()
    assert plan.info()["seg_tiles"] > 0
    want = np.empty(m)
    want[0] = (bb[0] + 0.0) / dd[0]
    for i in range(1, m):
        want[i] = (bb[i] + (-ll[i]) * want[i - 1]) / dd[i]
    x = torch.full((m,), float("nan"), dtype=torch.float64, device="cuda")
    plan.solve(torch.from_numpy(bb).cuda(), x)
    got = x.cpu().numpy()
    assert plan.check() == 0
    assert np.array_equal(got.view(np.int64), want.view(np.int64))
