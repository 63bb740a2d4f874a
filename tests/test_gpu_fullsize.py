"""GPU parity at the benchmark's full sizes and launch configuration: the
three large systems (3D stencil 128^3, banded n=1e6, power-law n=4e6) with the
recorded policies, tilings, queues, waves and chain shares bench.py times,
every component against the FP64 oracle (floored componentwise error <= 1e-10,
and <= 1e-12, the rounding-level sentinel), plus the plain schedule."""
import importlib.util
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from gate import SENTINEL, TOL, errors, report

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


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


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name", ["stencil3d_128", "banded_1m", "powerlaw_4m"])
def test_large_tuned(torch, sp, bench, name):
    s = wl.config(name)
    ref = oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
    kind, kw = bench.CANDIDATES[bench.TUNED[name]]
    b = torch.from_numpy(s.b).cuda()
    for label, policy in (("tuned", (kind, kw)), ("plain", ("none", {}))):
        plan = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite(policy[0], **policy[1])
        if label == "tuned":
            # the launch configuration the benchmark times
            plan.set_tiling(bench.TUNED_TILING[name]).set_queues(bench.TUNED_QUEUES[name])
        plan.upload()
        if label == "tuned":
            plan.set_launch(bench.TUNED_WAVES[name]).set_chain_share(bench.TUNED_CHAIN[name])
        x = plan.solve(b)
        assert plan.check() == 0
        err = errors(x.cpu().numpy(), ref)
        info = plan.info()
        print(name, label, info["levels_rw"], info["rhs_mode"], report(x.cpu().numpy(), ref), flush=True)
        assert np.all(np.isfinite(x.cpu().numpy()))
        assert err[1] <= TOL
        assert err[1] <= SENTINEL, err
        plan.close()
        del x
