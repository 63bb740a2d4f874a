"""Host side of the C ABI (no GPU): the library loads and exports every
declared entry point, rejects malformed input with the documented status,
and its plans (levels, stages, rewritten structure and values, schedule)
are bit-exact with the CPU oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sp():
    import paper_2103_11445_amd as m
    m.load()
    return m


def declared_functions():
    with open(os.path.join(ROOT, "include", "sptrsv.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sptrsv_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(sp):
    names = declared_functions()
    assert "sptrsv_solve" in names and "sptrsv_analyse" in names and len(names) >= 15
    assert "sptrsv_solve_fp32" in names and "sptrsv_solve_refined" in names
    lib = ctypes.CDLL(sp.library_path())
    for name in names:
        assert hasattr(lib, name), name


def _policy(kind, **kw):
    return {"kind": kind, **kw}


def compare_with_oracle(sp, s, pol):
    kw = {k: v for k, v in pol.items() if k != "kind"}
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite(pol["kind"], **kw)
    o = oracle.plan(s.row_ptr, s.col_idx, s.val, pol)
    info = plan.info()
    assert np.array_equal(plan.levels(0), o["level"])
    assert info["levels"] == o["nlev"]
    sol, dol = plan.stages()
    assert np.array_equal(sol, o["stage_of_level"])
    assert np.array_equal(dol, o["delta_of_level"])
    assert info["stages"] == o["nstages"]
    # M's entries are held only when the M pass reads them; export builds
    # them (same values) without touching the device image
    assert info["m_stored"] == (0 if info["rhs_mode"] == 2 else 1), info
    lp, m = plan.export()
    after = plan.info()
    assert after["m_stored"] == 1
    assert (after["rhs_mode"], after["nnz_rhs"], after["device_bytes"], after["stages"]) == \
        (info["rhs_mode"], info["nnz_rhs"], info["device_bytes"], info["stages"])
    for a, b in zip(lp, o["lp"]):
        assert np.array_equal(a, b)
    for a, b in zip(m, o["m"]):
        assert np.array_equal(a, b)
    assert np.array_equal(plan.levels(1), o["level_rw"])
    ptr, rows = plan.schedule()
    assert np.array_equal(ptr, o["sched_ptr"]) and np.array_equal(rows, o["sched_rows"])
    assert info["levels_rw"] == o["nlev_rw"]
    assert info["nnz_rw"] == o["lp"][0][-1] and info["nnz_m"] == o["m"][0][-1]
    assert info["flops"] == oracle.flops(s.row_ptr)
    assert info["flops_rw"] == oracle.flops(o["lp"][0], o["m"][0])
    assert info["bytes"] == 12 * s.nnz + 24 * s.n
    extra = {0: 0, 1: 16 * s.n, 2: 24 * s.n}[info["rhs_mode"]]
    assert info["bytes_rw"] == 12 * (info["nnz_rw"] + info["nnz_rhs"]) + 24 * s.n + extra - 2 * info["compact_terms"]
    # compact columns: every wide-tile term (the off-diagonal entries not in segments) at 16 bits
    assert info["compact_terms"] == 0 or info["compact_cols"] == 1
    assert info["nnz_rhs"] == (0 if info["nnz_m"] == 0 else info["nnz_rhs"])
    return plan, o


POLICIES = [
    _policy("none"),
    _policy("threshold"),
    _policy("threshold", max_width=16, max_depth=64, max_fill=1.0),
    _policy("threshold", max_width=10**9, max_depth=4, max_fill=10.0),
    _policy("threshold", max_width=10**9, max_depth=10**9, max_fill=0.05, max_entries=40000),
]


@pytest.mark.parametrize("pol", POLICIES, ids=lambda p: str(p))
@pytest.mark.parametrize("make", [
    lambda: wl.stencil2d(100, seed=0),
    lambda: wl.stencil3d(20, seed=1),
    lambda: wl.banded(6000, 200, 8, 24, seed=2),
    lambda: wl.powerlaw(50000, 1200, seed=3),
    lambda: wl.random_lower(300, 0.05, seed=4),
    lambda: wl.bidiagonal(500, seed=5),
    lambda: wl.diagonal(77, seed=6),
], ids=["2d", "3d", "banded", "powerlaw", "random", "chain", "diag"])
def test_plan_bit_exact(sp, make, pol):
    compare_with_oracle(sp, make(), pol)


# Every policy the benchmark's tuning leg can pick, on reduced instances of
# the large workload's three families (sized so that the oracle's sorted-list
# rewrite finishes in seconds): levels, stages, entries per level, L' and M
# structure and values, levels of L' and the schedule, bit for bit.
def _bench_policy(cand):
    import bench
    kind, kw = bench.CANDIDATES[cand]
    return {"kind": kind, **kw}


BENCH_CASES = [
    # the thin-level rule: budget binding (long tail) and not binding (short tail)
    ("powerlaw 2e5 tail 2e4", lambda: wl.powerlaw(200000, 20000, seed=3), ["paper", "paper256"]),
    ("powerlaw 2e5 tail 1e3", lambda: wl.powerlaw(200000, 1000, seed=3), ["paper", "paper256"]),
    ("powerlaw 2e4 tail 2e3", lambda: wl.powerlaw(20000, 2000, seed=3),
     ["depth2", "depth16", "depth64", "depth128", "depth256", "depth512"]),
    ("banded 2e4 bw 200", lambda: wl.banded(20000, 200, 8, 24, seed=2), ["depth2", "depth16", "depth64", "depth128"]),
    ("banded 1e4 bw 200", lambda: wl.banded(10000, 200, 8, 24, seed=2), ["depth256", "depth512"]),
    ("stencil3d 32", lambda: wl.stencil3d(32, seed=1),
     ["paper", "paper256", "depth2", "depth16", "depth64", "depth128", "depth256", "depth512"]),
]


@pytest.mark.parametrize("name,make,cands", BENCH_CASES, ids=[c[0] for c in BENCH_CASES])
def test_bench_policies_bit_exact(sp, name, make, cands):
    s = make()
    for cand in cands:
        plan, o = compare_with_oracle(sp, s, _bench_policy(cand))
        assert o["nlev_rw"] < o["nlev"] or cand == "plain", (name, cand)
        plan.close()


def _plan_arrays(plan):
    sol, dol = plan.stages()
    lp, m = plan.export()
    ptr, rows = plan.schedule()
    return [sol, dol, *lp, *m, plan.levels(1), ptr, rows]


@pytest.mark.parametrize("make,cand", [
    (lambda: wl.banded(10000, 200, 8, 24, seed=2), "depth512"),
    (lambda: wl.banded(20000, 200, 8, 24, seed=4), "depth64"),
    (lambda: wl.powerlaw(20000, 2000, seed=3), "depth256"),
    (lambda: wl.powerlaw(200000, 20000, seed=3), "paper256"),
    (lambda: wl.stencil3d(24, seed=1), "depth16"),
    (lambda: wl.random_lower(400, 0.03, seed=7), "depth64"),
], ids=["banded-512", "banded-64", "powerlaw-256", "powerlaw-paper256", "3d-16", "random-64"])
def test_stage_representations_agree(sp, monkeypatch, make, cand):
    """A stage's rewritten rows are built from bit sets over the stage's
    local index space while it is small, else from sorted lists, and a stage
    that outgrows the limit switches from one to the other; every limit
    (0: lists only; 64 and 300: switches inside stages) gives the same plan
    bit for bit, and the default one matches the oracle."""
    s = make()
    pol = _bench_policy(cand)
    kw = {k: v for k, v in pol.items() if k != "kind"}
    ref = None
    for bits in ("0", "64", "300", ""):
        monkeypatch.setenv("SPTRSV_DENSE_STAGE_BITS", bits)
        plan = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite(pol["kind"], **kw)
        arrays = _plan_arrays(plan)
        plan.close()
        if ref is None:
            ref = arrays
            continue
        for a, b in zip(arrays, ref):
            assert np.array_equal(a, b), bits
    monkeypatch.delenv("SPTRSV_DENSE_STAGE_BITS")
    compare_with_oracle(sp, s, pol)[0].close()


def test_explicit_masks_bit_exact(sp):
    rng = np.random.default_rng(3)
    s = wl.powerlaw(20000, 800, seed=9)
    nlev = oracle.levels(s.row_ptr, s.col_idx)[1]
    for t in range(5):
        mask = (rng.random(nlev) < rng.uniform(0.2, 0.9)).astype(np.uint8)
        compare_with_oracle(sp, s, {"kind": "explicit", "absorb": mask, "max_entries": 2**40})


@pytest.mark.parametrize("name", ["stencil3d_128", "banded_1m", "powerlaw_4m"])
def test_full_size_default_policy_bit_exact(sp, name):
    """The large workload, at full size, under the default threshold rule."""
    compare_with_oracle(sp, wl.config(name), _policy("threshold"))


def test_rewrite_restarts_from_analysed_matrix(sp):
    s = wl.powerlaw(30000, 900, seed=4)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val)
    plan.rewrite("threshold", max_width=4, max_depth=16, max_fill=0.5)
    first = plan.export()
    plan.rewrite("threshold", max_width=10**9, max_depth=3, max_fill=9.0)
    plan.rewrite("threshold", max_width=4, max_depth=16, max_fill=0.5)
    again = plan.export()
    for a, b in zip(first[0] + first[1], again[0] + again[1]):
        assert np.array_equal(a, b)


def test_empty_system(sp):
    plan = sp.Plan(np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    i = plan.info()
    assert i["n"] == 0 and i["levels"] == 0 and i["levels_rw"] == 0 and i["tiles"] == 0


def test_policy_default(sp):
    pol = sp.Policy()
    sp.load().sptrsv_policy_default(ctypes.byref(pol))
    assert (pol.kind, pol.max_width, pol.max_depth, pol.max_fill, pol.max_entries) == \
        (1, 4, 64, 0.25, 2**31 - 1)


# ------------------------------------------------------------- errors --

def _analyse_status(sp, n, rp, ci, v):
    lib = sp.load()
    h = ctypes.c_void_p(123)
    rp = None if rp is None else np.ascontiguousarray(rp, np.int32)
    ci = None if ci is None else np.ascontiguousarray(ci, np.int32)
    v = None if v is None else np.ascontiguousarray(v, np.float64)
    p = lambda a: None if a is None else a.ctypes.data
    st = lib.sptrsv_analyse(n, p(rp), p(ci), p(v), ctypes.byref(h))
    if st == 0:
        lib.sptrsv_plan_destroy(h)
    else:
        assert h.value is None  # *out = NULL on error
        assert lib.sptrsv_last_error().decode() != ""
    return sp.STATUS[st]


def test_csr_errors(sp):
    good_rp, good_ci, good_v = [0, 1, 3], [0, 0, 1], [2.0, -1.0, 3.0]
    assert _analyse_status(sp, 2, good_rp, good_ci, good_v) == "OK"
    cases = {
        "ERR_ARG": [(-1, good_rp, good_ci, good_v), (2, None, good_ci, good_v),
                    (2, good_rp, None, good_v), (2, good_rp, good_ci, None)],
        "ERR_CSR": [(2, [1, 1, 3], good_ci, good_v),             # row_ptr[0] != 0
                    (2, [0, 2, 1], [0, 0, 1], good_v),           # decreasing row_ptr
                    (2, [0, 1, 3], [0, 5, 1], good_v),           # column out of range
                    (2, [0, 1, 3], [0, -1, 1], good_v),          # negative column
                    (3, [0, 1, 2, 5], [0, 1, 1, 0, 2], [1.0] * 5),  # unsorted
                    (3, [0, 1, 2, 5], [0, 1, 0, 0, 2], [1.0] * 5),  # duplicate
                    (2, [0, 2, 4], [0, 1, 0, 1], [1.0] * 4)],       # entry above diagonal
        "ERR_DIAG": [(2, [0, 1, 2], [0, 0], [1.0, -1.0]),         # row 1 has no diagonal
                     (2, [0, 1, 1], [0], [1.0]),                  # empty row
                     (2, [0, 1, 3], [0, 0, 1], [2.0, -1.0, 0.0])],  # zero diagonal
    }
    for want, lst in cases.items():
        for args in lst:
            assert _analyse_status(sp, *args) == want, (want, args)
    lib = sp.load()
    assert sp.STATUS[lib.sptrsv_analyse(2, None, None, None, None)] == "ERR_ARG"


def test_policy_errors(sp):
    s = wl.stencil2d(5, seed=0)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val)
    bad = [dict(kind="threshold", max_width=-1), dict(kind="threshold", max_depth=0),
           dict(kind="threshold", max_fill=-0.5), dict(kind="threshold", max_fill=float("nan")),
           dict(kind="threshold", max_entries=-1)]
    for kw in bad:
        kind = kw.pop("kind")
        with pytest.raises(sp.SptrsvError) as e:
            plan.rewrite(kind, **kw)
        assert e.value.status == "ERR_ARG"
    pol, _ = sp.make_policy("explicit")
    pol.absorb_len = 3  # no mask pointer
    assert sp.STATUS[sp.load().sptrsv_rewrite(plan._h, ctypes.byref(pol))] == "ERR_ARG"
    pol.kind = 7
    assert sp.STATUS[sp.load().sptrsv_rewrite(plan._h, ctypes.byref(pol))] == "ERR_ARG"
    # a failed rewrite leaves a usable (plain) plan behind
    info = plan.info()
    assert info["levels_rw"] == info["levels"]


def test_null_and_state_errors_without_gpu(sp):
    lib = sp.load()
    st = ctypes.c_int32()
    for call in (lambda: lib.sptrsv_rewrite(None, None),
                 lambda: lib.sptrsv_device_bytes(None, None),
                 lambda: lib.sptrsv_plan_info(None, None),
                 lambda: lib.sptrsv_solve(None, None, None, None),
                 lambda: lib.sptrsv_check(None, None, ctypes.byref(st))):
        assert sp.STATUS[call()] == "ERR_ARG"
    s = wl.stencil2d(4, seed=0)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val)
    assert sp.STATUS[lib.sptrsv_solve(plan._h, None, None, None)] == "ERR_STATE"
    assert sp.STATUS[lib.sptrsv_check(plan._h, None, ctypes.byref(st))] == "ERR_STATE"
    assert sp.STATUS[lib.sptrsv_upload(plan._h, None, 0, None)] == "ERR_ARG"
    lib.sptrsv_plan_destroy(None)  # ignored


# ------------------------------------------ upper-triangular input (U x = b) --

def _reversed_lower(s):
    """The lower-triangular matrix obtained by reversing the index order of an
    upper-triangular system, built independently of the library."""
    n = s.n
    rows = []
    for r in range(n):
        i = n - 1 - r
        seg = slice(s.row_ptr[i], s.row_ptr[i + 1])
        rows.append((n - 1 - s.col_idx[seg][::-1], s.val[seg][::-1]))
    rp = np.concatenate([[0], np.cumsum([len(c) for c, _ in rows])]).astype(np.int32)
    ci = np.concatenate([c for c, _ in rows]).astype(np.int32)
    v = np.concatenate([x for _, x in rows])
    return rp, ci, v


@pytest.mark.parametrize("make", [lambda: wl.stencil2d(40, seed=2), lambda: wl.powerlaw(30000, 700, seed=5),
                                  lambda: wl.banded(3000, 200, 8, 24, seed=4)])
def test_upper_plan_is_the_reversed_lower_plan(sp, make):
    U = wl.transpose(make())
    rp, ci, v = _reversed_lower(U)
    pol = {"kind": "threshold", "max_width": 10**9, "max_depth": 4, "max_fill": 10.0}
    plan = sp.Plan(U.row_ptr, U.col_idx, U.val, upper=True)
    plan.rewrite("threshold", max_width=10**9, max_depth=4, max_fill=10.0)
    o = oracle.plan(rp, ci, v, pol)
    assert np.array_equal(plan.levels(0), o["level"])
    lp, m = plan.export()
    for a, b in zip(lp + m, o["lp"] + o["m"]):
        assert np.array_equal(a, b)


def test_upper_errors(sp):
    lib = sp.load()
    h = ctypes.c_void_p()

    def st(n, rp, ci, v):
        rp = np.ascontiguousarray(rp, np.int32)
        ci = np.ascontiguousarray(ci, np.int32)
        v = np.ascontiguousarray(v, np.float64)
        r = lib.sptrsv_analyse_upper(n, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, ctypes.byref(h))
        if r == 0:
            lib.sptrsv_plan_destroy(h)
        return sp.STATUS[r]

    assert st(2, [0, 2, 3], [0, 1, 1], [2.0, -1.0, 3.0]) == "OK"
    assert st(2, [0, 2, 3], [0, 1, 0], [2.0, -1.0, 3.0]) == "ERR_CSR"   # below the diagonal
    assert st(2, [0, 1, 2], [1, 1], [2.0, 3.0]) == "ERR_DIAG"           # row 0 has no diagonal
    assert st(2, [0, 2, 3], [0, 1, 1], [0.0, -1.0, 3.0]) == "ERR_DIAG"  # zero diagonal


# -------------------------------------------------------------- batches --

def test_batch_plan_is_the_union_plan(sp):
    """A batched plan equals the oracle plan of the block-diagonal union
    (k copies of each system), built here independently."""
    corp = wl.batch_corpus(7, nmin=50, nmax=3000, ks=(1, 2, 3), seed=8)
    ks = [s.b.shape[1] for s in corp]
    rows, cols, vals, base = [], [], [], 0
    rp = [0]
    for s, k in zip(corp, ks):
        # copy c of row i is union row base + i*k + c
        for i in range(s.n):
            for c in range(k):
                seg = slice(s.row_ptr[i], s.row_ptr[i + 1])
                cols.append(base + s.col_idx[seg] * k + c)
                vals.append(s.val[seg])
                rp.append(rp[-1] + (s.row_ptr[i + 1] - s.row_ptr[i]))
        base += s.n * k
    rp = np.array(rp, np.int32)
    ci = np.concatenate(cols).astype(np.int32)
    v = np.concatenate(vals)
    pol = {"kind": "threshold", "max_width": 10**9, "max_depth": 3, "max_fill": 10.0}
    plan = sp.Plan.batch([(s.row_ptr, s.col_idx, s.val) for s in corp], ks)
    plan.rewrite("threshold", max_width=10**9, max_depth=3, max_fill=10.0)
    o = oracle.plan(rp, ci, v, pol)
    assert plan.info()["n"] == rp.size - 1
    assert np.array_equal(plan.levels(0), o["level"])
    lp, m = plan.export()
    for a, b in zip(lp + m, o["lp"] + o["m"]):
        assert np.array_equal(a, b)


def test_batch_errors(sp):
    s = wl.stencil2d(4, seed=0)
    with pytest.raises(sp.SptrsvError) as e:
        sp.Plan.batch([(s.row_ptr, s.col_idx, s.val)], [0])
    assert e.value.status == "ERR_ARG"
    bad = s.val.copy()
    bad[s.row_ptr[3] - 1] = 0.0
    with pytest.raises(sp.SptrsvError) as e:
        sp.Plan.batch([(s.row_ptr, s.col_idx, s.val), (s.row_ptr, s.col_idx, bad)])
    assert e.value.status == "ERR_DIAG" and "system 1" in str(e.value)
    empty = sp.Plan.batch([])
    assert empty.info()["n"] == 0


# ------------------------------------------------------- FP32 storage --

def test_fp32_plan_keeps_the_schedule(sp):
    """Storing the device image in FP32 changes the value type only: levels,
    stages, rewritten structure and values (FP64 on the host) are those of
    the FP64 plan, the precision survives a rewrite, and the byte counts
    follow the value size."""
    s = wl.powerlaw(20000, 600, seed=6)
    p64 = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite("threshold", max_depth=8)
    p32 = sp.Plan(s.row_ptr, s.col_idx, s.val).set_precision(32).rewrite("threshold", max_depth=8)
    i64, i32 = p64.info(), p32.info()
    assert i64["precision"] == 64 and i32["precision"] == 32
    for k in ("n", "levels", "stages", "levels_rw", "nnz", "nnz_rw", "nnz_m", "flops", "flops_rw", "tiles"):
        assert i64[k] == i32[k], k
    n = i64["n"]
    assert i32["bytes"] == 8 * i32["nnz"] + 16 * n
    extra = {0: 0, 1: 8 * n, 2: 16 * n}[i32["rhs_mode"]]
    assert i32["bytes_rw"] == 8 * (i32["nnz_rw"] + i32["nnz_rhs"]) + 16 * n + extra - 2 * i32["compact_terms"]
    assert i64["bytes"] == 12 * i64["nnz"] + 24 * n
    assert np.array_equal(p64.levels(1), p32.levels(1))
    for a, b in zip(p64.export()[0] + p64.export()[1], p32.export()[0] + p32.export()[1]):
        assert np.array_equal(a, b)
    # the FP32 image carries the FP64 residual matrix and two FP32 vectors
    assert i32["device_bytes"] > 12 * i32["nnz"] + 8 * n
    p32.set_precision(64)
    assert p32.info()["device_bytes"] == i64["device_bytes"]


def test_fp32_errors_without_gpu(sp):
    lib = sp.load()
    s = wl.stencil2d(4, seed=0)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val)
    assert sp.STATUS[lib.sptrsv_set_precision(plan._h, 16)] == "ERR_ARG"
    assert sp.STATUS[lib.sptrsv_set_precision(None, 32)] == "ERR_ARG"
    assert sp.STATUS[lib.sptrsv_solve_fp32(plan._h, None, None, None)] == "ERR_STATE"
    assert sp.STATUS[lib.sptrsv_solve_refined(plan._h, None, None, 0, 0.0, None)] == "ERR_ARG"
    assert sp.STATUS[lib.sptrsv_solve_refined(plan._h, None, None, 17, 0.0, None)] == "ERR_ARG"
    assert sp.STATUS[lib.sptrsv_solve_refined(plan._h, None, None, 4, float("nan"), None)] == "ERR_ARG"
    assert sp.STATUS[lib.sptrsv_solve_refined(plan._h, None, None, 4, 1e-13, None)] == "ERR_STATE"
    it, corr = ctypes.c_int32(), ctypes.c_double()
    assert sp.STATUS[lib.sptrsv_refine_stats(plan._h, None, ctypes.byref(it), ctypes.byref(corr))] == "ERR_STATE"
    plan.set_precision(32)
    assert sp.STATUS[lib.sptrsv_solve(plan._h, None, None, None)] == "ERR_STATE"


def test_fp32_batch_plan_packs(sp):
    """FP32 packing of batched plans (systems of different sizes and
    right-hand-side counts) and of upper plans: the residual matrix the
    packer rebuilds has exactly the callers' entries (the packer checks its
    counts and fails with ERR_STATE otherwise)."""
    corp = wl.batch_corpus(6, nmin=200, nmax=20000, ks=(1, 3, 8), seed=29)
    ks = [1 if s.b.ndim == 1 else s.b.shape[1] for s in corp]
    plan = sp.Plan.batch([(s.row_ptr, s.col_idx, s.val) for s in corp], ks)
    b64 = plan.info()["device_bytes"]
    plan.set_precision(32).rewrite("threshold", max_width=10**9, max_depth=8, max_fill=12.0)
    assert plan.info()["precision"] == 32
    nnz = sum(s.nnz for s in corp)
    rows = sum(s.n * k for s, k in zip(corp, ks))
    assert plan.info()["device_bytes"] >= 12 * nnz + 8 * rows
    U = wl.transpose(wl.powerlaw(5000, 300, seed=3))
    sp.Plan(U.row_ptr, U.col_idx, U.val, upper=True).set_precision(32)
    assert b64 > 0


# -------------------------------------------- learned-policy host pieces --

def _group_features(rows, terms, orig, maxlen, span):
    """The documented feature formula, written out independently."""
    return np.array([np.log2(1 + rows) / 16, np.log2(1 + terms) / 24,
                     min(16.0, max(terms - orig, 0) / max(orig, 1)) / 4, np.log2(1 + maxlen) / 8,
                     min(256.0, terms / max(rows, 1)) / 16, np.log2(max(span, 1)) / 8], dtype=np.float32)


def test_level_features_plain_and_rewritten(sp):
    """Features of the executed levels, recomputed here from the exported
    rewritten system and the levels of L."""
    s = wl.powerlaw(3000, 200, seed=11)
    for kind, kw in [("none", {}), ("threshold", {"max_width": INF, "max_depth": 4, "max_fill": 10.0})]:
        plan = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite(kind, **kw)
        f = plan.level_features()
        (lp_ptr, _, _), (m_ptr, _, _) = plan.export()
        lev0 = plan.levels(0)
        ptr, rows = plan.schedule()
        assert f.shape == (plan.info()["levels_rw"], 6)
        for l in range(0, f.shape[0], max(1, f.shape[0] // 25)):
            r = rows[ptr[l]:ptr[l + 1]]
            lens = (lp_ptr[r + 1] - lp_ptr[r]) + (m_ptr[r + 1] - m_ptr[r])
            orig = int(np.sum(s.row_ptr[r + 1] - s.row_ptr[r]))
            want = _group_features(r.size, int(lens.sum()), orig, int(lens.max()),
                                   int(lev0[r].max() - lev0[r].min() + 1))
            assert np.allclose(f[l], want, rtol=1e-6, atol=1e-7), (kind, l)


INF = 10**9


def test_stamp_levels_cover_every_level(sp):
    """Every executed level is finished by at least one stamp unit, and the
    map only names existing levels (or -1)."""
    for make in (lambda: wl.bidiagonal(3000, seed=1), lambda: wl.stencil3d(16, seed=2),
                 lambda: wl.powerlaw(20000, 2000, seed=3)):
        s = make()
        plan = sp.Plan(s.row_ptr, s.col_idx, s.val)
        lv = plan.stamp_levels()
        info = plan.info()
        assert lv.size == info["tiles"] + info["seg_tiles"]
        assert lv.min() >= -1 and lv.max() < info["levels_rw"]
        assert np.array_equal(np.unique(lv[lv >= 0]), np.arange(info["levels_rw"]))


def test_learned_policy_needs_a_model(sp):
    s = wl.stencil2d(8, seed=0)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val)
    with pytest.raises(sp.SptrsvError) as e:
        plan.rewrite("learned", max_depth=8)
    assert e.value.status == "ERR_ARG"
    lib = sp.load()
    assert sp.STATUS[lib.sptrsv_mlp_grad_workspace(0, None)] == "ERR_ARG"
    assert sp.STATUS[lib.sptrsv_mlp_forward(None, None, None, 0, None)] == "OK"   # nothing to do
    assert sp.STATUS[lib.sptrsv_mlp_forward(None, None, None, 4, None)] == "ERR_ARG"
    assert sp.STATUS[lib.sptrsv_mlp_adam(None, None, None, None, 1, 0.1, 0.9, 0.999, 1e-8, None)] == "ERR_ARG"


# ------------------------------------------------ right-hand-side modes --

def test_rhs_modes(sp):
    """The two ways of applying b' = b + M b: the M pass reads nnz(M)
    entries, the stage solve the entries of L inside the stages (counted
    here from the stage of every level); the rewrite itself is unchanged."""
    s = wl.banded(4000, 200, 8, 24, seed=9)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite("threshold", max_width=INF, max_depth=16, max_fill=12.0)
    # the stage solve does not read M: only its row counts are kept ...
    assert plan.info()["m_stored"] == 0 and plan.info()["nnz_m"] > 0
    # ... and the M pass builds its entries (compared below with export's)
    plan.set_rhs_mode("mpass")
    assert plan.info()["m_stored"] == 1 and plan.info()["rhs_mode"] == 1
    lp_mp, m_mp = plan.export()
    plan.set_rhs_mode("auto").rewrite("threshold", max_width=INF, max_depth=16, max_fill=12.0)
    assert plan.info()["m_stored"] == 0
    lp0, m0 = plan.export()
    for a, b in zip(lp_mp + m_mp, lp0 + m0):
        assert np.array_equal(a, b)
    sol, _ = plan.stages()
    lev = plan.levels(0)
    st = sol[lev]
    rows = np.repeat(np.arange(s.n), np.diff(s.row_ptr))
    nnz_b = int(np.sum(st[rows] == st[s.col_idx]))
    assert plan.info()["rhs_mode"] == 2 and plan.info()["nnz_rhs"] == nnz_b   # auto: M is large here
    plan.set_rhs_mode("mpass")
    i = plan.info()
    assert i["rhs_mode"] == 1 and i["nnz_rhs"] == i["nnz_m"]
    plan.set_rhs_mode("stage")
    assert plan.info()["rhs_mode"] == 2
    for a, b in zip(plan.export()[0] + plan.export()[1], lp0 + m0):
        assert np.array_equal(a, b)
    plain = sp.Plan(s.row_ptr, s.col_idx, s.val)
    assert plain.info()["rhs_mode"] == 0 and plain.info()["nnz_rhs"] == 0
    lib = sp.load()
    assert sp.STATUS[lib.sptrsv_set_rhs_mode(plan._h, 7)] == "ERR_ARG"
    # the mode survives a rewrite, and FP32 packing carries the stage system too
    plan.set_precision(32).rewrite("threshold", max_width=INF, max_depth=8, max_fill=12.0)
    assert plan.info()["rhs_mode"] == 2


def _stage_segments_expected(s, stage_of_row):
    """Stages of L_B that the packer should run whole on one wave: at least
    two levels of L_B and at most 4 segment tiles (4 terms a lane, 64 lanes)
    per level on average."""
    n, rp, ci = s.n, s.row_ptr, s.col_idx
    lev = np.zeros(n, dtype=np.int64)
    xt = np.zeros(n, dtype=np.int64)
    for i in range(n):
        cols = ci[rp[i]:rp[i + 1]]
        same = cols[(cols != i) & (stage_of_row[cols] == stage_of_row[i])]
        xt[i] = len(same)
        lev[i] = 1 + lev[same].max() if len(same) else 0
    count = 0
    for st in np.unique(stage_of_row):
        rows = np.nonzero(stage_of_row == st)[0]
        tiles, depth = 0, 0
        for l in np.unique(lev[rows]):
            r = rows[lev[rows] == l]
            mx = xt[r].max()
            lg = next(g for g in range(7) if mx <= 4 << g)
            tiles += -(-len(r) // (64 >> lg))
            depth += 1
        count += depth >= 2 and tiles <= 4 * depth
    return count


@pytest.mark.parametrize("make,depth", [
    (lambda: wl.banded(4000, 200, 8, 24, seed=9), 16),
    (lambda: wl.banded(6007, 100, 2, 6, seed=10), 64),
    (lambda: wl.stencil3d(20, seed=11), 2),
    (lambda: wl.powerlaw(20011, 500, seed=12), 8),
])
def test_stage_segments(sp, make, depth):
    """In the stage solve, narrow stages run whole on one wave each (their
    count recomputed here from the stage of every level and the levels of
    L_B), and only in that solve."""
    s = make()
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val)
    plan.rewrite("threshold", max_width=INF, max_depth=depth, max_fill=40.0).set_rhs_mode("stage")
    sol, _ = plan.stages()
    want = _stage_segments_expected(s, sol[plan.levels(0)])
    i = plan.info()
    print(s.name, i["stages"], want, i["rhs_segments"])
    assert i["rhs_mode"] == 2 and i["rhs_segments"] == want
    assert plan.set_rhs_mode("mpass").info()["rhs_segments"] == 0


def test_register_chunks_choice(sp):
    """The solve holds 8 chunks of a wide tile in registers when most tiles
    need more than 4 (8 terms per lane give rows 4 < len / lanes <= 8), else
    4; the choice follows the tiling and never changes the rewrite."""
    s = wl.banded(4000, 200, 8, 24, seed=9)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite("threshold", max_width=INF, max_depth=16, max_fill=12.0)
    assert plan.info()["reg_chunks"] == 4
    assert plan.set_tiling(8).info()["reg_chunks"] == 8
    assert plan.set_tiling(2).info()["reg_chunks"] == 4
    st = wl.stencil3d(16, seed=3)
    assert sp.Plan(st.row_ptr, st.col_idx, st.val).set_tiling(8).info()["reg_chunks"] == 4


def test_stage_segments_random(sp):
    """The same count on seeded random matrices of every family and a range
    of stage depths and fill budgets (stage mode forced)."""
    rng = np.random.default_rng(2024)
    makers = [lambda q: wl.banded(int(q.integers(500, 3000)), int(q.integers(20, 200)), 2, 12,
                                  seed=int(q.integers(1 << 30))),
              lambda q: wl.powerlaw(int(q.integers(2000, 8000)), int(q.integers(50, 400)),
                                    seed=int(q.integers(1 << 30))),
              lambda q: wl.stencil2d(int(q.integers(10, 40)), seed=int(q.integers(1 << 30))),
              lambda q: wl.random_lower(int(q.integers(50, 300)), float(q.uniform(0.05, 0.5)),
                                        seed=int(q.integers(1 << 30)))]
    for trial in range(12):
        s = makers[trial % len(makers)](rng)
        depth = int(rng.choice([2, 3, 8, 32, 128]))
        plan = sp.Plan(s.row_ptr, s.col_idx, s.val)
        plan.rewrite("threshold", max_width=INF, max_depth=depth, max_fill=float(rng.choice([2.0, 12.0, 60.0])))
        if plan.info()["nnz_m"] == 0:
            continue
        plan.set_rhs_mode("stage")
        sol, _ = plan.stages()
        assert plan.info()["rhs_segments"] == _stage_segments_expected(s, sol[plan.levels(0)]), (s.name, depth)


def test_ring_only_segments(sp):
    """A segment whose every term comes from the LDS ring is counted (and
    run by the lighter loop when all segments are such): a chain keeps each
    dependency in the ring, the power-law tail reaches back past its segment."""
    ch = wl.bidiagonal(5000, seed=43)
    i = sp.Plan(ch.row_ptr, ch.col_idx, ch.val).info()
    assert i["segments"] == i["ring_segments"] == 1 and i["seg_tiles"] == 5000
    pl = wl.powerlaw(50000, 3000, seed=42)
    i = sp.Plan(pl.row_ptr, pl.col_idx, pl.val).info()
    assert i["segments"] >= 1 and i["ring_segments"] == 0
    rl = wl.random_lower(700, 0.6, seed=54)
    i = sp.Plan(rl.row_ptr, rl.col_idx, rl.val).info()
    assert 0 < i["ring_segments"] < i["segments"]
    st = wl.stencil3d(20, seed=41)
    i = sp.Plan(st.row_ptr, st.col_idx, st.val).info()
    assert i["segments"] == i["ring_segments"] == 0


def test_tiling_knob(sp):
    """Terms per lane change the tile shapes only: more terms per lane pack
    more rows per tile (fewer tiles); the rewritten system is unchanged."""
    s = wl.powerlaw(50000, 2000, seed=1)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite("threshold", max_width=INF, max_depth=4, max_fill=10.0)
    lp0, m0 = plan.export()
    tiles = []
    for t in (1, 2, 4, 8, 16):
        plan.set_tiling(t)
        tiles.append(plan.info()["tiles"])
    assert tiles == sorted(tiles, reverse=True) and tiles[0] > tiles[-1]
    for a, b in zip(plan.export()[0] + plan.export()[1], lp0 + m0):
        assert np.array_equal(a, b)
    lib = sp.load()
    for bad in (0, 3, 32, -4):
        assert sp.STATUS[lib.sptrsv_set_tiling(plan._h, bad)] == "ERR_ARG"


def test_hop_probe_argument_errors(sp):
    """Argument checks of the hop probe happen before any device call."""
    lib = sp.load()
    ns = ctypes.c_double()
    buf = ctypes.create_string_buffer(64)
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert lib.sptrsv_probe_hop(100, 0, None, 64, ctypes.byref(ns), None) == 1
    assert lib.sptrsv_probe_hop(1, 0, p, 64, ctypes.byref(ns), None) == 1
    assert lib.sptrsv_probe_hop(100, 0, p, 16, ctypes.byref(ns), None) == 1
    assert lib.sptrsv_probe_hop(100, 0, p, 64, None, None) == 1


def test_mlp_grad_noalloc_argument_errors(sp):
    """Sizes outside the static workspace and null pointers are refused
    before any device call."""
    lib = sp.load()
    buf = ctypes.create_string_buffer(64)
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert lib.sptrsv_mlp_grad_noalloc(p, p, p, 0, p, p, None) == 1
    assert lib.sptrsv_mlp_grad_noalloc(p, p, p, sp.MLP_NOALLOC_MAX_SAMPLES + 1, p, p, None) == 1
    assert "8192" in lib.sptrsv_last_error().decode()
    assert lib.sptrsv_mlp_grad_noalloc(None, p, p, 10, p, p, None) == 1


def test_chain_and_sink_queues(sp):
    """Rows nothing depends on are packed apart from the chain: a diagonal
    matrix is all sinks, a chain (one row per level, a segment) all chain,
    and a 2D stencil rewritten into 2-level stages has both (its first-level
    rows of each stage feed no one after the rewrite)."""
    d = sp.Plan(*(lambda s: (s.row_ptr, s.col_idx, s.val))(wl.diagonal(5000, seed=1)))
    assert d.info()["chain_items"] == 0 and d.info()["tiles"] > 0
    c = sp.Plan(*(lambda s: (s.row_ptr, s.col_idx, s.val))(wl.bidiagonal(3000, seed=1)))
    assert c.info()["chain_items"] == c.info()["tiles"]
    s = wl.stencil2d(100, seed=0)
    p = sp.Plan(s.row_ptr, s.col_idx, s.val).rewrite("threshold", max_width=10**9, max_depth=2, max_fill=12.0)
    i = p.info()
    assert 0 < i["chain_items"] < i["tiles"]
    # the chain rows are exactly the rows some row of L' depends on
    (lp_ptr, lp_col, _), _ = p.export(with_m=False)
    rows = np.repeat(np.arange(s.n), np.diff(lp_ptr))
    needed = np.zeros(s.n, bool)
    needed[lp_col[lp_col != rows]] = True
    assert 0 < needed.sum() < s.n
    for q in (d, c, p):
        q.close()
