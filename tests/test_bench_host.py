"""Host checks of the benchmark script's contract (no GPU): the multi-GPU
request is refused with a message, and the recorded tuning refers to
candidates the tuning leg can build."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_recorded_tuning_is_buildable():
    b = _bench()
    for name in b.LARGE:
        assert b.TUNED[name] in b.CANDIDATES
        assert b.TUNED_TILING[name] in (2, 4, 8, 16)
        assert b.TUNED_WAVES[name] in (0, 2, 4, 8)
        assert b.TUNED_CHAIN[name] in (0,) + b.CHAIN_CANDIDATES
        assert b.TUNED_QUEUES[name] in (1, 2)
    # the batched and precision workloads' recorded choices (used by the
    # default run's summaries of those workloads)
    assert b.TUNED_BATCH["policy"] in b.BATCH_CANDIDATES
    for t in (b.TUNED_BATCH, b.TUNED_BATCH_PLAIN):
        assert t["tiling"] in (2, 4, 8, 16) and t["waves"] in (0, 2, 4, 8)
        assert t["queues"] in (1, 2) and t["chain"] in (0, 250, 500, 750)
    assert b.TUNED_PREC["policy"] in b.prec_candidates_for(8)
    assert b.TUNED_PREC["tiling"] in (2, 4, 8) and b.TUNED_PREC["queues"] in (1, 2)
    for shallow, deep in b.DEEPER.items():
        assert shallow in b.CANDIDATES and deep in b.CANDIDATES
        assert b.CANDIDATES[deep][1]["max_depth"] > b.CANDIDATES[shallow][1]["max_depth"]


def test_kernel_hash_is_deterministic():
    b = _bench()
    assert b.kernel_sources_hash() == b.kernel_sources_hash()
