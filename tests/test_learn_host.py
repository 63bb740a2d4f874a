"""Host pieces of the learned policy's driver (no GPU): the split of an
instrumented solve's clock stamps into level times, and the share of the
right-hand-side step per executed level."""
import numpy as np
import pytest

import workloads as wl


@pytest.fixture(scope="module")
def learn():
    import paper_2103_11445_amd as sp
    sp.load()
    from paper_2103_11445_amd import learn as m
    return m


def test_level_times_frontier(learn):
    # start 100; level 0 ends at 130 and 120, level 1 at 125 (inside level 0's
    # span: adds nothing), level 2 at 200; a -1 unit is ignored
    stamps = np.array([130, 120, 125, 999, 200, 100], dtype=np.int64)
    level = np.array([0, 0, 1, -1, 2], dtype=np.int32)
    t = learn.level_times(stamps, level, 3)
    assert np.allclose(t, [0.30, 0.0, 0.70])
    assert np.isclose(t.sum(), (200 - 100) / learn.TICKS_PER_US)


def test_level_times_sum_to_span_random(learn):
    rng = np.random.default_rng(0)
    for _ in range(50):
        nl = int(rng.integers(1, 20))
        units = int(rng.integers(nl, 100))
        level = np.concatenate([np.arange(nl), rng.integers(-1, nl, units - nl)]).astype(np.int32)
        start = 1000
        stamps = np.concatenate([start + rng.integers(0, 5000, units), [start]]).astype(np.int64)
        t = learn.level_times(stamps, level, nl)
        span = (stamps[:-1][level >= 0].max() - start) / learn.TICKS_PER_US
        assert np.all(t >= 0) and np.isclose(t.sum(), span)


def test_rhs_share(learn):
    import paper_2103_11445_amd as sp
    s = wl.banded(3000, 200, 8, 24, seed=3)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val)
    assert np.all(learn.rhs_share(plan, s.row_ptr, s.col_idx) == 0)       # no b-terms
    plan.rewrite("threshold", max_width=10**9, max_depth=8, max_fill=12.0)
    for mode in ("mpass", "stage"):
        plan.set_rhs_mode(mode)
        w = learn.rhs_share(plan, s.row_ptr, s.col_idx)
        assert w.shape == (plan.info()["levels_rw"],) and np.isclose(w.sum(), 1.0) and np.all(w >= 0)
    # M pass: each level's share is its rows' b-terms over all of them
    plan.set_rhs_mode("mpass")
    _, (m_ptr, _, _) = plan.export()
    lev = plan.levels(1)
    per = np.bincount(lev, weights=np.diff(m_ptr), minlength=plan.info()["levels_rw"])
    assert np.allclose(learn.rhs_share(plan, s.row_ptr, s.col_idx), per / per.sum())


def test_corpus_is_seeded(learn):
    a, b = learn.corpus_matrix(10007, nmax=3e4), learn.corpus_matrix(10007, nmax=3e4)
    assert a.name == b.name and np.array_equal(a.col_idx, b.col_idx) and np.array_equal(a.val, b.val)
    pols = learn.label_policies(10007)
    assert pols[0] == ("none", {}) and len(pols) == 10
    # the deep stage depths the benchmark's tuning picks are among the labels
    assert max(kw.get("max_depth", 0) for _, kw in pols) == 512
    assert pols == learn.label_policies(10007)


def test_label_parts_merge(learn, tmp_path, capsys):
    """Labels collected in parts (each its own seed range, saved as npz) are
    read back and trained on together; with no new matrices and no training
    steps nothing touches the GPU."""
    rng = np.random.default_rng(1)
    paths = []
    for first, used, rows in ((254, 3, 40), (257, 2, 25)):
        X = rng.random((rows, 6)).astype(np.float32)
        y = rng.random(rows).astype(np.float32)
        p = tmp_path / f"labels_{first}.npz"
        np.savez_compressed(p, X=X, y=y, first=first, used=used, collect_s=1.5)
        paths.append(str(p))
    learn.main(["train", "--train", "0", "--heldout", "0", "--steps", "0", "--labels-in", *paths])
    with np.load(paths[0], allow_pickle=False) as z:
        assert z["X"].shape == (40, 6) and int(z["used"]) == 3
