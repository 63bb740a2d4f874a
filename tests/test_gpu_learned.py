"""GPU: the learned rewrite policy's pieces through the C ABI.

* cost-model kernels (forward, mean-squared-error gradient, Adam) against
  the float64 CPU oracle (oracle/mlp.py, itself pinned by finite differences
  and closed forms).  Tolerances: FP32 kernels against FP64 -- each output
  sums at most 64 products of magnitude <= a few units, so the error is a
  few hundred FP32 ulps of the largest partial sum; the tests allow 1e-4
  relative to the largest magnitude involved;
* the instrumented solve: the same x as the plain solve, and clock stamps
  that split into non-negative level times summing to the solve's span;
* the LEARNED policy with the committed model: its plans are the oracle's
  plans for the same stage choice (bit-exact) and solve to the gate, and on
  held-out matrices the judged choice is never slower than the threshold
  heuristic while the learned plans gain on it (printed and asserted).
"""
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from gate import TOL, errors
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


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


def _params(seed):
    p = omlp.init(seed)
    rng = np.random.default_rng(seed + 100)
    p[omlp.N_PARAMS - 1 - 64:] += rng.normal(scale=0.1, size=65)  # non-zero output layer biases
    p[64 * 6:64 * 7] = rng.normal(scale=0.3, size=64)             # b1
    return p


def _data(m, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1.5, (m, omlp.N_IN)), rng.normal(size=m)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("m", [1, 2, 255, 1000, 4097])
def test_mlp_forward_matches_oracle(torch, sp, m):
    p = _params(1)
    X, _ = _data(m, 2)
    p32 = p.astype(np.float32).astype(np.float64)
    X32 = X.astype(np.float32).astype(np.float64)
    y = sp.mlp_forward(_dev(torch, p), _dev(torch, X)).cpu().numpy()
    ref = omlp.forward(p32, X32)
    err = np.max(np.abs(y - ref)) / max(1.0, np.max(np.abs(ref)))
    print("forward", m, err, flush=True)
    assert err <= 1e-4


@pytest.mark.parametrize("m", [1, 33, 256, 257, 3000])
def test_mlp_grad_matches_oracle(torch, sp, m):
    p = _params(3)
    X, t = _data(m, 4)
    p32 = p.astype(np.float32).astype(np.float64)
    X32 = X.astype(np.float32).astype(np.float64)
    t32 = t.astype(np.float32).astype(np.float64)
    g, loss = sp.mlp_grad(_dev(torch, p), _dev(torch, X), _dev(torch, t))
    g = g.cpu().numpy()
    lref, gref = omlp.loss_grad(p32, X32, t32)
    err = np.max(np.abs(g - gref)) / np.max(np.abs(gref))
    print("grad", m, err, float(loss.item()), lref, flush=True)
    assert err <= 1e-4
    assert abs(float(loss.item()) - lref) <= 1e-4 * lref
    # deterministic: the same call gives the same bits
    g2, _ = sp.mlp_grad(_dev(torch, p), _dev(torch, X), _dev(torch, t))
    assert np.array_equal(g, g2.cpu().numpy())


def test_mlp_adam_matches_oracle(torch, sp):
    rng = np.random.default_rng(5)
    p = rng.normal(size=omlp.N_PARAMS)
    g = rng.normal(size=omlp.N_PARAMS)
    m1 = rng.normal(scale=0.1, size=omlp.N_PARAMS)
    m2 = rng.uniform(0.01, 1.0, size=omlp.N_PARAMS)
    f = lambda a: a.astype(np.float32).astype(np.float64)  # noqa: E731
    want, wm1, wm2 = omlp.adam_step(f(p), f(g), f(m1), f(m2), 7, lr=1e-2)
    pd, m1d, m2d = _dev(torch, p), _dev(torch, m1), _dev(torch, m2)
    sp.mlp_adam(pd, _dev(torch, g), m1d, m2d, 7, 1e-2)
    assert np.allclose(pd.cpu().numpy(), want, rtol=2e-6, atol=1e-6)
    assert np.allclose(m1d.cpu().numpy(), wm1, rtol=2e-6, atol=1e-7)
    assert np.allclose(m2d.cpu().numpy(), wm2, rtol=2e-6, atol=1e-7)


def test_training_follows_oracle(torch, sp):
    """Thirty Adam steps on one batch: the GPU parameters stay with the
    oracle's and the loss falls the same way."""
    X, _ = _data(512, 6)
    t = np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2]
    p = _params(7).astype(np.float32).astype(np.float64)
    X32 = X.astype(np.float32).astype(np.float64)
    t32 = t.astype(np.float32).astype(np.float64)
    q, m1, m2 = p.copy(), np.zeros_like(p), np.zeros_like(p)
    pd, m1d, m2d = _dev(torch, p), torch.zeros(omlp.N_PARAMS, device="cuda"), torch.zeros(omlp.N_PARAMS, device="cuda")
    Xd, td = _dev(torch, X32), _dev(torch, t32)
    losses = []
    for k in range(1, 31):
        l, g = omlp.loss_grad(q, X32, t32)
        q, m1, m2 = omlp.adam_step(q, g, m1, m2, k, lr=3e-3)
        gd, ld = sp.mlp_grad(pd, Xd, td)
        sp.mlp_adam(pd, gd, m1d, m2d, k, 3e-3)
        losses.append((l, float(ld.item())))
    diff = np.max(np.abs(pd.cpu().numpy() - q))
    print("training", losses[0], losses[-1], diff, flush=True)
    assert diff <= 1e-3
    assert abs(losses[-1][1] - losses[-1][0]) <= 1e-3 * losses[0][0]
    assert losses[-1][0] < 0.7 * losses[0][0]


@pytest.mark.parametrize("make", [lambda: wl.stencil3d(20, seed=41), lambda: wl.powerlaw(50000, 3000, seed=42),
                                  lambda: wl.bidiagonal(5000, seed=43)])
def test_stamped_solve(torch, sp, make):
    s = make()
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite("threshold", max_width=10**9, max_depth=4,
                                                        max_fill=10.0).upload()
    b = torch.from_numpy(s.b).cuda()
    x1, x2 = torch.empty_like(b), torch.empty_like(b)
    plan.solve(b, x1)
    info = plan.info()
    stamps = torch.zeros(info["tiles"] + info["seg_tiles"] + 1, dtype=torch.int64, device="cuda")
    plan.solve_stamped(b, x2, stamps)
    assert plan.check() == 0
    # the instrumented solve runs the general segment loop: on the chain,
    # whose segment is ring-only, it must agree bit for bit with the lighter one
    assert torch.equal(x1, x2)
    st = stamps.cpu().numpy()
    lv = plan.stamp_levels()
    from paper_2103_11445_amd.learn import level_times
    t = level_times(st, lv, info["levels_rw"])
    span = (st[:-1][lv >= 0].max() - st[-1]) / 100.0
    assert np.all(t >= 0) and abs(t.sum() - span) <= 1e-9 * max(span, 1.0)
    assert np.all(st[:-1][lv >= 0] >= st[-1])
    print(s.name, info["levels_rw"], "span us", span, flush=True)


MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_2103_11445_amd", "cost_model.npz")


@pytest.fixture(scope="module")
def model(torch):
    if not os.path.exists(MODEL):
        pytest.skip("no trained cost model committed")
    from paper_2103_11445_amd.learn import load_model
    params, meta = load_model(MODEL)
    return torch.from_numpy(params).cuda(), meta


@pytest.mark.parametrize("make", [lambda: wl.stencil2d(100, seed=0), lambda: wl.banded(20000, 200, 8, 24, seed=44),
                                  lambda: wl.powerlaw(40000, 2000, seed=45)])
def test_learned_plan_is_the_oracle_plan(torch, sp, model, make):
    """The library's rewrite under the learned stage choice equals the
    oracle's rewrite under the same choice given as an explicit mask, and
    the learned plan solves to the gate."""
    s = make()
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite("learned", model=model[0], max_depth=64, max_fill=12.0)
    sol, _ = plan.stages()
    absorb = np.zeros(sol.size, np.uint8)
    absorb[1:] = sol[1:] == sol[:-1]
    o = oracle.plan(s.row_ptr, s.col_idx, s.val, {"kind": "explicit", "absorb": absorb})
    assert np.array_equal(sol, o["stage_of_level"])
    lp, m = plan.export()
    for a, b in zip(lp + m, o["lp"] + o["m"]):
        assert np.array_equal(a, b)
    plan.upload()
    b = torch.from_numpy(s.b).cuda()
    x = plan.solve(b)
    assert plan.check() == 0
    ref = oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
    print(s.name, "levels", plan.info()["levels"], "->", plan.info()["levels_rw"], errors(x.cpu().numpy(), ref),
          flush=True)
    assert errors(x.cpu().numpy(), ref)[1] <= TOL


def test_learned_gain_on_heldout(torch, sp, model):
    """Held-out matrices (seeds never trained on): re-timed on fresh samples
    after the choice, the judged plan is not slower than the threshold
    heuristic's beyond timing noise (10%) on any matrix and not slower in
    geometric mean, and the learned plans are faster than the heuristic's in
    geometric mean."""
    from paper_2103_11445_amd.learn import HELDOUT_SEED, evaluate
    params = model[0].cpu().numpy()
    seeds = [HELDOUT_SEED + 100 + m for m in range(8)]
    summary, rows = evaluate(torch, params, seeds, reps=5, nmax=2e5)
    print(summary, flush=True)
    for r in rows:
        print(r["matrix"], r["threshold_ms"], r["learned_ms"], r["chosen"], r["judged_ms"],
              r["threshold_fresh_ms"], flush=True)
        assert r["judged_ms"] <= r["threshold_fresh_ms"] * 1.10
    assert summary["geomean_speedup_judged_vs_threshold"] >= 1.0
    assert summary["geomean_speedup_learned_vs_threshold"] > 1.0
