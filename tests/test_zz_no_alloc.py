"""The allocation-free gradient entry point (sptrsv_mlp_grad_noalloc) against
the workspace one (sptrsv_mlp_grad) through the C ABI: bit-identical
gradients and losses on two calls in a row, the second with fewer samples
(it runs over what the first left in the shared static workspace), and
against the cost model's CPU oracle; sizes above the static maximum are
refused."""
import numpy as np
import pytest

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


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_noalloc_grad_equals_workspace_grad(torch, sp):
    rng = np.random.default_rng(21)
    p = omlp.init(7)
    p[64 * 6:64 * 7] = rng.normal(scale=0.3, size=64)
    pd = _dev(torch, p)
    for m, seed in ((sp.MLP_NOALLOC_MAX_SAMPLES, 1), (3001, 2), (1, 3)):
        r = np.random.default_rng(seed)
        X, t = r.uniform(-1, 1.5, (m, omlp.N_IN)), r.normal(size=m)
        Xd, td = _dev(torch, X), _dev(torch, t)
        g_ws, l_ws = sp.mlp_grad(pd, Xd, td)
        g_na, l_na = sp.mlp_grad_noalloc(pd, Xd, td)
        torch.cuda.synchronize()
        print("noalloc", m, float(l_na.item()), float(l_ws.item()), flush=True)
        assert torch.equal(g_na, g_ws), m
        assert torch.equal(l_na, l_ws), m
        # and the shared result against the CPU oracle (the workspace path's bar)
        f = lambda a: a.astype(np.float32).astype(np.float64)  # noqa: E731
        lref, gref = omlp.loss_grad(f(p), f(X), f(t))
        g = g_na.cpu().numpy()
        assert np.max(np.abs(g - gref)) / np.max(np.abs(gref)) <= 1e-4
        assert abs(float(l_na.item()) - lref) <= 1e-4 * lref


def test_noalloc_refuses_oversize(torch, sp):
    m = sp.MLP_NOALLOC_MAX_SAMPLES + 1
    X = torch.zeros((m, 6), dtype=torch.float32, device="cuda")
    t = torch.zeros(m, dtype=torch.float32, device="cuda")
    p = torch.zeros(sp.MLP_PARAMS, dtype=torch.float32, device="cuda")
    with pytest.raises(sp.SptrsvError) as e:
        sp.mlp_grad_noalloc(p, X, t)
    assert e.value.status == "ERR_ARG"
