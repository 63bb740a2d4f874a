"""Pins for the CPU oracle: checks against exact arithmetic, brute force,
closed forms and the worked example of the paper, so that a plausible slip
in the oracle (a dropped term, a wrong sign or index, a transposed operand)
fails here.  No GPU."""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import workloads as wl
from exact import (all_lower_patterns, dense, exact_rewritten_row, exact_solve,
                   longest_path_levels, rel_close)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _explicit(nlev, absorbed):
    mask = np.zeros(max(nlev, 1), dtype=np.uint8)
    for l in absorbed:
        mask[l] = 1
    return {"kind": "explicit", "absorb": mask, "max_entries": 2**62}


def _stage_starts(stage_of_level):
    start = []
    for l, s in enumerate(stage_of_level):
        start.append(start[-1] if l > 0 and s == stage_of_level[l - 1] else l)
    return start


# ------------------------------------------------ T1: every tiny pattern --

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_solve_and_levels_exhaustive(n):
    """Forward substitution (Sec. II, Algorithm 1) against an exact
    Gauss-Jordan solve, and levels against brute-force longest paths, for
    every strictly-lower pattern of size n."""
    for t, pairs in enumerate(all_lower_patterns(n)):
        s = wl.from_pairs(n, pairs, seed=t)
        x = oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
        ex = exact_solve(s.row_ptr, s.col_idx, s.val, s.b)
        # error bound scaled by the largest component (components that
        # nearly cancel cannot be held to a relative bound)
        scale = max(abs(e) for e in ex)
        for i in range(n):
            assert abs(Fraction(float(x[i])) - ex[i]) <= scale * Fraction(1e-14), (pairs, i)
        lv, nlev = oracle.levels(s.row_ptr, s.col_idx)
        bf = longest_path_levels(s.row_ptr, s.col_idx)
        assert list(lv) == bf, pairs
        assert nlev == (max(bf) + 1 if n else 0)


def _check_rewrite_exact(s, absorbed):
    """Rewrite under an explicit stage choice and compare every rewritten
    row, its b-combination and the entries added with the exact linear
    characterisation of Sec. III (Fig. 2 and 3)."""
    n = s.n
    lv, nlev = oracle.levels(s.row_ptr, s.col_idx)
    pol = _explicit(nlev, absorbed)
    sol, dol, ns = oracle.select_stages(s.row_ptr, s.col_idx, lv, nlev, pol)
    # explicit choice: a level joins the previous stage iff it is absorbed
    expect = [0]
    for l in range(1, nlev):
        expect.append(expect[-1] + (0 if l in absorbed else 1))
    assert list(sol) == expect
    (lp_ptr, lp_col, lp_val), (m_ptr, m_col, m_val) = oracle.rewrite(
        s.row_ptr, s.col_idx, s.val, lv, nlev, sol)
    A = dense(s.row_ptr, s.col_idx, s.val)
    start = _stage_starts(list(sol))
    added = [0] * max(nlev, 1)
    for i in range(n):
        a = start[lv[i]]
        in_stage = [lv[j] >= a for j in range(n)]
        if lv[i] == a:
            coeffs = {k: A[i][k] for k in range(i) if A[i][k] != 0}
            mm = {}
        else:
            coeffs, mm = exact_rewritten_row(A, i, in_stage)
        got_l = {int(lp_col[p]): lp_val[p] for p in range(lp_ptr[i], lp_ptr[i + 1] - 1)}
        got_m = {int(m_col[p]): m_val[p] for p in range(m_ptr[i], m_ptr[i + 1])}
        # the diagonal is last and untouched
        assert lp_col[lp_ptr[i + 1] - 1] == i
        assert lp_val[lp_ptr[i + 1] - 1] == s.val[s.row_ptr[i + 1] - 1]
        # value rule => no cancellation, so the symbolic structure equals the
        # exact nonzero pattern
        assert set(got_l) == set(coeffs), (i, got_l, coeffs)
        assert set(got_m) == set(mm), (i, got_m, mm)
        for k, v in coeffs.items():
            assert rel_close(got_l[k], v, 1e-13)
        for j, v in mm.items():
            assert rel_close(got_m[j], v, 1e-13)
        added[lv[i]] += len(got_l) + len(got_m) - (s.row_ptr[i + 1] - s.row_ptr[i] - 1)
    for l in range(nlev):
        assert dol[l] == (added[l] if l in absorbed else 0)
    # no rewritten row keeps a dependency inside its own stage
    for i in range(n):
        a = start[lv[i]]
        for p in range(lp_ptr[i], lp_ptr[i + 1] - 1):
            assert lv[lp_col[p]] < a or lv[i] == a


@pytest.mark.parametrize("n", [2, 3, 4])
def test_rewrite_exhaustive_all_stage_choices(n):
    for t, pairs in enumerate(all_lower_patterns(n)):
        s = wl.from_pairs(n, pairs, seed=100 + t)
        _, nlev = oracle.levels(s.row_ptr, s.col_idx)
        for r in range(nlev):
            for absorbed in itertools.combinations(range(1, nlev), r):
                _check_rewrite_exact(s, set(absorbed))


def test_rewrite_sampled_n5_to_n9():
    rng = np.random.default_rng(7)
    for t in range(150):
        n = int(rng.integers(5, 10))
        s = wl.random_lower(n, float(rng.uniform(0.2, 0.8)), seed=1000 + t)
        _, nlev = oracle.levels(s.row_ptr, s.col_idx)
        absorbed = {l for l in range(1, nlev) if rng.random() < 0.6}
        _check_rewrite_exact(s, absorbed)


# ---------------------------------------------------- T2: closed forms --

def _unit_bidiagonal(n, rng):
    rp = np.concatenate([[0, 1], 1 + 2 * np.arange(1, n)]).astype(np.int32)
    ci = np.empty(rp[-1], dtype=np.int32)
    v = np.empty(rp[-1], dtype=np.float64)
    ci[0], v[0] = 0, 1.0
    for i in range(1, n):
        ci[rp[i]], v[rp[i]] = i - 1, -1.0
        ci[rp[i] + 1], v[rp[i] + 1] = i, 1.0
    b = rng.integers(-1000, 1000, size=n).astype(np.float64)
    return rp, ci, v, b


def test_unit_bidiagonal_gives_prefix_sums():
    rng = np.random.default_rng(1)
    rp, ci, v, b = _unit_bidiagonal(5000, rng)
    x = oracle.solve(rp, ci, v, b)
    assert np.array_equal(x, np.cumsum(b))
    lv, nlev = oracle.levels(rp, ci)
    assert nlev == 5000 and np.array_equal(lv, np.arange(5000))


def test_unit_bidiagonal_full_merge_is_identity_plus_ones():
    """Absorbing every level into stage 0 rewrites row i into
    x_i = b_0 + ... + b_i: L' = I and M = strictly-lower ones."""
    rng = np.random.default_rng(2)
    n = 200
    rp, ci, v, b = _unit_bidiagonal(n, rng)
    lv, nlev = oracle.levels(rp, ci)
    sol, _, ns = oracle.select_stages(rp, ci, lv, nlev, _explicit(nlev, range(1, nlev)))
    assert ns == 1
    lp, m = oracle.rewrite(rp, ci, v, lv, nlev, sol)
    assert np.array_equal(lp[0], np.arange(n + 1))
    assert np.array_equal(lp[1], np.arange(n)) and np.all(lp[2] == 1.0)
    assert np.array_equal(np.diff(m[0]), np.arange(n))
    for i in range(n):
        assert np.array_equal(m[1][m[0][i]:m[0][i + 1]], np.arange(i))
    assert np.all(m[2] == 1.0)
    x = oracle.solve_rewritten(lp, m, b)
    assert np.array_equal(x, np.cumsum(b))


def test_diagonal_gives_b_over_d():
    s = wl.diagonal(1000, seed=3)
    x = oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
    assert np.array_equal(x, s.b / s.val)
    lv, nlev = oracle.levels(s.row_ptr, s.col_idx)
    assert nlev == 1 and not lv.any()
    p = oracle.plan(s.row_ptr, s.col_idx, s.val, {"kind": "threshold", "max_width": 10**9,
                                                   "max_depth": 10**9, "max_fill": 1e9})
    assert p["nstages"] == 1 and p["m"][0][-1] == 0
    assert np.array_equal(p["lp"][1], s.col_idx) and np.array_equal(p["lp"][2], s.val)


def test_stencil_levels_closed_form():
    g = 37
    s = wl.stencil2d(g, seed=4)
    lv, nlev = oracle.levels(s.row_ptr, s.col_idx)
    i = np.arange(g * g)
    assert np.array_equal(lv, i // g + i % g) and nlev == 2 * g - 1
    g = 11
    s = wl.stencil3d(g, seed=5)
    lv, nlev = oracle.levels(s.row_ptr, s.col_idx)
    i = np.arange(g ** 3)
    assert np.array_equal(lv, i % g + (i // g) % g + i // (g * g)) and nlev == 3 * g - 2


def test_level_sets_are_stable_sort_by_level():
    s = wl.powerlaw(30000, 500, seed=9)
    lv, nlev = oracle.levels(s.row_ptr, s.col_idx)
    ptr, rows = oracle.level_sets(lv, nlev)
    assert np.array_equal(rows, np.argsort(lv, kind="stable"))
    assert np.array_equal(ptr, np.concatenate([[0], np.cumsum(np.bincount(lv, minlength=nlev))]))


# ------------------------------------------- the worked example (Fig. 2) --

def test_fig2_chain_golden():
    """Sec. III, Fig. 2: row 3 depends on row 1, row 1 on row 0.  One
    rewrite (row 1's original equation) moves row 3 up one level and makes it
    depend on row 0; a second rewrite (row 0's equation) leaves it with no
    dependency, and its old level becomes empty and disappears."""
    with open(os.path.join(GOLDEN, "fig2_chain.json")) as f:
        g = json.load(f)
    s = wl.from_pairs(g["n"], g["pairs"], seed=11)
    lv, nlev = oracle.levels(s.row_ptr, s.col_idx)
    assert list(lv) == g["levels"]
    for step in g["steps"]:
        pol = _explicit(nlev, step["absorbed_levels"])
        p = oracle.plan(s.row_ptr, s.col_idx, s.val, pol)
        r = g["row"]
        lp_ptr, lp_col, _ = p["lp"]
        m_ptr, m_col, _ = p["m"]
        assert list(lp_col[lp_ptr[r]:lp_ptr[r + 1] - 1]) == step["deps"]
        assert list(m_col[m_ptr[r]:m_ptr[r + 1]]) == step["b_terms"]
        assert int(p["level_rw"][r]) == step["level"]
        assert p["nlev_rw"] == step["nlev"]
        x = oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
        xr = oracle.solve_rewritten(p["lp"], p["m"], s.b)
        assert np.allclose(xr, x, rtol=1e-15, atol=0)


# ---------------------------------------- stage selection, by hand --------

def test_threshold_stages_hand_computed_chain():
    """Chain of 5 rows, widths all 1.  Entries added when absorbing into a
    stage that starts at level a: row a+1 adds 0 (one x-term becomes one
    b-term), row a+2 adds 1, ... (x_{a-1} survives once a > 0)."""
    s = wl.bidiagonal(5, seed=0)  # nnz = 9
    lv, nlev = oracle.levels(s.row_ptr, s.col_idx)
    pol = {"kind": "threshold", "max_width": 4, "max_depth": 3, "max_fill": 100.0}
    sol, dol, ns = oracle.select_stages(s.row_ptr, s.col_idx, lv, nlev, pol)
    assert list(sol) == [0, 0, 0, 1, 1] and ns == 2
    assert list(dol) == [0, 0, 1, 0, 1]
    pol["max_fill"] = 0.1  # budget floor(0.9) = 0
    sol, dol, ns = oracle.select_stages(s.row_ptr, s.col_idx, lv, nlev, pol)
    assert list(sol) == [0, 0, 1, 2, 3]
    pol["max_fill"] = 100.0
    pol["max_width"] = 0  # nothing is thin
    sol, _, ns = oracle.select_stages(s.row_ptr, s.col_idx, lv, nlev, pol)
    assert list(sol) == [0, 1, 2, 3, 4] and ns == 5
    pol["max_width"] = 1
    pol["max_entries"] = 9  # total may not grow: only the 0-entry level 1 joins
    sol, _, _ = oracle.select_stages(s.row_ptr, s.col_idx, lv, nlev, pol)
    assert list(sol) == [0, 0, 1, 2, 3]


def test_threshold_width_rule_on_2d_stencil():
    """5-point 2D stencil on g x g: level s has min(s+1, 2g-1-s) rows.  With
    max_width = 2 only levels 1 and 2g-3 are thin besides the corners."""
    g = 6
    s = wl.stencil2d(g, seed=1)
    lv, nlev = oracle.levels(s.row_ptr, s.col_idx)
    pol = {"kind": "threshold", "max_width": 2, "max_depth": 64, "max_fill": 10.0}
    sol, dol, ns = oracle.select_stages(s.row_ptr, s.col_idx, lv, nlev, pol)
    widths = [min(l + 1, 2 * g - 1 - l) for l in range(nlev)]
    expect = [0]
    for l in range(1, nlev):
        expect.append(expect[-1] + (0 if widths[l] <= 2 else 1))
    assert list(sol) == expect


# ------------------------------------------------------ T3: invariants --

@settings(max_examples=60, deadline=None, derandomize=True)
@given(n=st.integers(1, 120), density=st.floats(0.0, 0.5), seed=st.integers(0, 10**6),
       width=st.integers(0, 12), depth=st.integers(1, 40), fill=st.floats(0.0, 4.0))
def test_invariants_random(n, density, seed, width, depth, fill):
    s = wl.random_lower(n, density, seed=seed)
    pol = {"kind": "threshold", "max_width": width, "max_depth": depth, "max_fill": fill}
    p = oracle.plan(s.row_ptr, s.col_idx, s.val, pol)
    lv, nlev = p["level"], p["nlev"]
    # level(i) = 1 + max level(deps), on L and on L'
    for (rp, ci), lvl in (((s.row_ptr, s.col_idx), lv),
                          ((p["lp"][0], p["lp"][1]), p["level_rw"])):
        for i in range(n):
            deps = [lvl[c] for c in ci[rp[i]:rp[i + 1]] if c < i]
            assert lvl[i] == (1 + max(deps) if deps else 0)
    sol = p["stage_of_level"]
    assert sol[0] == 0 and np.all(np.diff(sol) >= 0) and np.all(np.diff(sol) <= 1)
    start = _stage_starts(list(sol))
    widths = np.bincount(lv, minlength=nlev)
    for l in range(1, nlev):
        if sol[l] == sol[l - 1]:
            assert widths[l] <= width and l - start[l] + 1 <= depth
    assert p["delta_of_level"].sum() <= int(np.floor(fill * s.nnz))
    assert p["nlev_rw"] <= p["nstages"]
    lp_ptr, lp_col, lp_val = p["lp"]
    m_ptr, m_col, m_val = p["m"]
    for i in range(n):
        a = start[lv[i]]
        if lv[i] == a:  # first level of a stage: row untouched, bit for bit
            assert np.array_equal(lp_col[lp_ptr[i]:lp_ptr[i + 1]], s.col_idx[s.row_ptr[i]:s.row_ptr[i + 1]])
            assert np.array_equal(lp_val[lp_ptr[i]:lp_ptr[i + 1]], s.val[s.row_ptr[i]:s.row_ptr[i + 1]])
            assert m_ptr[i] == m_ptr[i + 1]
        else:
            assert all(lv[c] < a for c in lp_col[lp_ptr[i]:lp_ptr[i + 1] - 1])
            assert all(lv[c] >= a for c in m_col[m_ptr[i]:m_ptr[i + 1]])
    # L' = (I + M) L, in exact arithmetic, to rounding of the stored values
    A = dense(s.row_ptr, s.col_idx, s.val)
    for i in range(0, n, max(1, n // 15)):
        row = list(A[i])
        for p_ in range(m_ptr[i], m_ptr[i + 1]):
            j, mij = int(m_col[p_]), Fraction(float(m_val[p_]))
            row = [r + mij * a_ for r, a_ in zip(row, A[j])]
        got = {int(lp_col[q]): Fraction(float(lp_val[q])) for q in range(lp_ptr[i], lp_ptr[i + 1])}
        scale = max(abs(v) for v in row)
        for k in range(n):
            ref = got.get(k, Fraction(0))
            assert abs(row[k] - ref) <= scale * Fraction(1e-13)
    # same solution up to rounding; components that nearly cancel are held
    # to 1e-3 of the largest one (the floored reading of tests/gate.py)
    x = oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
    xr = oracle.solve_rewritten(p["lp"], p["m"], s.b)
    floor = 1e-3 * np.max(np.abs(x)) if n else 0.0
    assert np.all(np.abs(xr - x) <= 1e-12 * np.maximum(np.abs(x), floor))


@settings(max_examples=40, deadline=None, derandomize=True)
@given(n=st.integers(2, 150), density=st.floats(0.01, 0.4), seed=st.integers(0, 10**6),
       depth=st.integers(2, 30), fill=st.floats(0.5, 8.0))
def test_stage_rhs_identity(n, density, seed, depth, fill):
    """The right-hand side of the rewritten rows, b' = b + M b, equals D y
    with L_B y = b, L_B the entries of L whose two levels share a stage and D
    the diagonal (Sec. III: within a stage the rewriting eliminates exactly
    the in-stage couplings, so (I + M) restricted to a stage is D L_SS^-1).
    Both sides from the oracle: its M, and its solve of the block system."""
    s = wl.random_lower(n, density, seed=seed)
    pol = {"kind": "threshold", "max_width": 10**9, "max_depth": depth, "max_fill": fill}
    p = oracle.plan(s.row_ptr, s.col_idx, s.val, pol)
    stage = p["stage_of_level"][p["level"]]
    rows = np.repeat(np.arange(n), np.diff(s.row_ptr))
    keep = stage[rows] == stage[s.col_idx]
    bp = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(np.bincount(rows[keep], minlength=n), out=bp[1:])
    y = oracle.solve(bp, s.col_idx[keep].astype(np.int32), s.val[keep], s.b)
    m_ptr, m_col, m_val = p["m"]
    mb = np.array([np.dot(m_val[m_ptr[i]:m_ptr[i + 1]], s.b[m_col[m_ptr[i]:m_ptr[i + 1]]]) for i in range(n)])
    diag = s.val[s.row_ptr[1:] - 1]
    lhs, rhs = s.b + mb, diag * y
    floor = 1e-3 * np.max(np.abs(rhs))
    assert np.all(np.abs(lhs - rhs) <= 1e-12 * np.maximum(np.abs(rhs), floor))


def test_long_double_is_closer_to_exact():
    """The extended-precision twin is at least as close to the exact
    solution as the FP64 oracle (sampled rows of a 2D stencil)."""
    s = wl.stencil2d(12, seed=2)
    ex = exact_solve(s.row_ptr, s.col_idx, s.val, s.b)
    x = oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
    xl = oracle.solve_ld(s.row_ptr, s.col_idx, s.val, s.b)
    for i in range(s.n):
        e64 = abs(Fraction(float(x[i])) - ex[i])
        eld = abs(Fraction(float(xl[i])) - ex[i])
        assert eld <= e64 or eld <= abs(ex[i]) * Fraction(2.0 ** -53)


def _drifting_chain(n, seed):
    """Unit lower bidiagonal L with sub-diagonal -a, a = 1 - 2^-20, and b in
    [0.5, 1): x_i = b_i + a x_{i-1}.  Every step rounds a product and a sum,
    and with a so close to 1 those errors are carried forward almost
    undamped, so FP64 substitution drifts away from the exact solution."""
    a = 1.0 - 2.0 ** -20
    rng = np.random.default_rng(seed)
    b = rng.uniform(0.5, 1.0, n)
    rp = np.concatenate([[0], np.arange(1, n + 1) * 2 - 1]).astype(np.int32)
    ci = np.empty(2 * n - 1, np.int32)
    v = np.empty(2 * n - 1)
    ci[0], v[0] = 0, 1.0
    for i in range(1, n):
        ci[2 * i - 1], v[2 * i - 1] = i - 1, -a
        ci[2 * i], v[2 * i] = i, 1.0
    exact, xa = [], Fraction(0)
    for i in range(n):
        xa = Fraction(float(b[i])) + Fraction(a) * xa
        exact.append(xa)
    return rp, ci, v, b, exact


def _ulps(x, exact):
    import math
    return [abs(Fraction(float(xi)) - e) / Fraction(math.ulp(float(e))) for xi, e in zip(x, exact)]


def test_long_double_solve_is_extended_precision():
    """The extended-precision twin (the reference of the FP32 + refinement
    gate) really carries more than 53 bits: on a chain where the FP64
    substitution of Algorithm 1 drifts over ten ulps from the exact solution,
    the twin, rounded once to FP64 at the end, stays within one ulp of the
    exact solution at every component.  A twin that computed in double would
    reproduce the FP64 drift and fail."""
    rp, ci, v, b, exact = _drifting_chain(400, seed=7)
    e64 = _ulps(oracle.solve(rp, ci, v, b), exact)
    eld = _ulps(oracle.solve_ld(rp, ci, v, b), exact)
    # the FP64 oracle demonstrably drifts on this system (the test has teeth)
    assert max(e64) > 8 and sum(e > 4 for e in e64) > 100
    # 64-bit significand: 400 steps add at most ~400 * 2^-64 relative before
    # the final rounding's half ulp
    assert max(eld) <= 1, max(eld)
    # and it is strictly closer wherever FP64 is off by more than an ulp
    assert all(l < d for l, d in zip(eld, e64) if d > 1)


def test_flops_hand_counted_fig2():
    """FLOPs of the plans of the Fig. 2 chain (rows 1, 2 depend on row 0,
    row 3 on row 1), counted by hand: a multiply and an add per off-diagonal
    x-term or b-term, one division per row.
      L:      row 0: 1; rows 1-3: 2 + 1 each              = 10
      step 1: row 3 holds x_0 and b_1: 2 + 2 + 1 = 5      = 12
      step 2: rows 1, 2 hold b_0 (3 each), row 3 b_0, b_1 = 12"""
    with open(os.path.join(GOLDEN, "fig2_chain.json")) as f:
        g = json.load(f)
    s = wl.from_pairs(g["n"], g["pairs"], seed=11)
    assert oracle.flops(s.row_ptr) == 10
    nlev = oracle.levels(s.row_ptr, s.col_idx)[1]
    got = []
    for step in g["steps"]:
        p = oracle.plan(s.row_ptr, s.col_idx, s.val, _explicit(nlev, step["absorbed_levels"]))
        got.append(oracle.flops(p["lp"][0], p["m"][0]))
    assert got == [12, 12]


# ------------------------------------------ backward substitution (U x = b) --

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_solve_upper_exhaustive(n):
    """Backward substitution against exact Gauss-Jordan on the transposes of
    every strictly-lower pattern."""
    for t, pairs in enumerate(all_lower_patterns(n)):
        s = wl.transpose(wl.from_pairs(n, pairs, seed=t))
        x = oracle.solve_upper(s.row_ptr, s.col_idx, s.val, s.b)
        ex = exact_solve(s.row_ptr, s.col_idx, s.val, s.b)
        scale = max(abs(e) for e in ex)
        for i in range(n):
            assert abs(Fraction(float(x[i])) - ex[i]) <= scale * Fraction(1e-14), (pairs, i)


def test_solve_upper_suffix_sums():
    """Unit upper bidiagonal (1 on the diagonal, -1 above) gives suffix sums."""
    rng = np.random.default_rng(5)
    n = 3000
    rp, ci, v, b = _unit_bidiagonal(n, rng)
    U = wl.transpose(wl.System("bd", rp, ci, v, b))
    x = oracle.solve_upper(U.row_ptr, U.col_idx, U.val, b)
    assert np.array_equal(x, np.cumsum(b[::-1])[::-1])


# ------------------------------------- level-set execution on host cores --

@pytest.mark.parametrize("make,pol", [
    (lambda: wl.stencil2d(40, seed=0), {"kind": "none"}),
    (lambda: wl.stencil2d(40, seed=0), {"kind": "threshold", "max_width": 10**9, "max_depth": 4, "max_fill": 10.0}),
    (lambda: wl.powerlaw(20000, 1500, seed=3), {"kind": "threshold", "max_width": 4, "max_depth": 64,
                                                "max_fill": 1.0}),
    (lambda: wl.banded(3000, 200, 8, 24, seed=2), {"kind": "threshold", "max_width": 10**9, "max_depth": 16,
                                                   "max_fill": 20.0}),
])
def test_levelset_solve_matches_serial(make, pol):
    """Sec. II: rows of a level are independent, so the level-set execution
    (a barrier between levels, rows of a level on several threads) gives the
    serial result bit for bit, on the plain system (against Algorithm 1) and
    on rewritten ones (against the serial rewritten solve)."""
    s = make()
    p = oracle.plan(s.row_ptr, s.col_idx, s.val, pol)
    ref = oracle.solve_rewritten(p["lp"], p["m"], s.b)
    if pol["kind"] == "none":
        assert np.array_equal(ref, oracle.solve(s.row_ptr, s.col_idx, s.val, s.b))
    for threads in (1, 4):
        x = oracle.solve_levelset(p["sched_ptr"], p["sched_rows"], p["lp"], p["m"], s.b, threads=threads)
        assert np.array_equal(x, ref), threads


# ------------------------------------- merging repeated terms (Fig. 3) --

def _unmerged_terms(rp, ci, level, a, i):
    """Row i rewritten against a stage starting at level a *without*
    merging: every in-stage dependency replaced by its original equation,
    recursively, each path kept as a term of its own.  Returns the lists of
    x-term and b-term columns, one entry per path (brute force)."""
    xs, bs = [], []
    for q in range(rp[i], rp[i + 1] - 1):
        j = int(ci[q])
        if level[j] < a:
            xs.append(j)
        else:
            bs.append(j)
            x2, b2 = _unmerged_terms(rp, ci, level, a, j)
            xs += x2
            bs += b2
    return xs, bs


def _stage_start(level, stage_of_level, i):
    lv = level[i]
    a = lv
    while a > 0 and stage_of_level[a - 1] == stage_of_level[lv]:
        a -= 1
    return a


@pytest.mark.parametrize("seed", range(12))
def test_rearrangement_merges_repeated_terms(seed):
    """Fig. 3: after substitution the equation is rearranged so that each x
    and b appears once.  Against the unmerged expansion (one term per path,
    computed by brute force): the plan's x-terms and b-terms are exactly the
    distinct columns the paths reach, and its FLOPs never exceed the
    unmerged count."""
    rng = np.random.default_rng(seed)
    s = wl.random_lower(10, rng.uniform(0.2, 0.6), seed=seed)
    rp, ci = s.row_ptr, s.col_idx
    level, nlev = oracle.levels(rp, ci)
    mask = (rng.random(nlev) < 0.7).astype(np.uint8)
    o = oracle.plan(rp, ci, s.val, {"kind": "explicit", "absorb": mask, "max_entries": 2**40})
    (lpp, lpc, _), (mp, mc, _) = o["lp"], o["m"]
    unmerged = 0
    for i in range(s.n):
        a = _stage_start(level, o["stage_of_level"], i)
        if level[i] == a:
            xs, bs = [int(c) for c in ci[rp[i]:rp[i + 1] - 1]], []
        else:
            xs, bs = _unmerged_terms(rp, ci, level, a, i)
        assert sorted(set(xs)) == [int(c) for c in lpc[lpp[i]:lpp[i + 1] - 1]], i
        assert sorted(set(bs)) == [int(c) for c in mc[mp[i]:mp[i + 1]]], i
        unmerged += 2 * (len(xs) + len(bs)) + 1
    assert oracle.flops(lpp, mp) <= unmerged


def test_rearrangement_saving_on_a_diamond_and_none_on_a_chain():
    """Row 3 reaches row 0 through rows 1 and 2 (a diamond), all in one stage:
    merged, b_0 appears once instead of twice, a saving of one multiply-add
    (2 FLOPs).  On a chain every column is reached by one path: nothing to
    merge."""
    diamond = wl.from_pairs(4, [(1, 0), (2, 0), (3, 1), (3, 2)], seed=1)
    lv, nlev = oracle.levels(diamond.row_ptr, diamond.col_idx)
    assert list(lv) == [0, 1, 1, 2]
    o = oracle.plan(diamond.row_ptr, diamond.col_idx, diamond.val,
                    {"kind": "explicit", "absorb": np.array([0, 1, 1], np.uint8), "max_entries": 2**40})
    xs, bs = _unmerged_terms(diamond.row_ptr, diamond.col_idx, lv, 0, 3)
    assert sorted(xs) == [] and sorted(bs) == [0, 0, 1, 2]
    (lpp, _, _), (mp, mc, _) = o["lp"], o["m"]
    assert list(mc[mp[3]:mp[4]]) == [0, 1, 2]
    # rows 1, 2 hold b_0 (3 FLOPs each); row 3 merged holds b_0, b_1, b_2 (7),
    # unmerged four b-terms (9)
    assert oracle.flops(lpp, mp) == 1 + 3 + 3 + 7 and 1 + 3 + 3 + 9 - oracle.flops(lpp, mp) == 2
    chain = wl.bidiagonal(6, seed=2)
    lv, nlev = oracle.levels(chain.row_ptr, chain.col_idx)
    o = oracle.plan(chain.row_ptr, chain.col_idx, chain.val,
                    {"kind": "explicit", "absorb": np.ones(nlev, np.uint8), "max_entries": 2**40})
    for i in range(6):
        xs, bs = _unmerged_terms(chain.row_ptr, chain.col_idx, lv, 0, i)
        assert len(bs) == len(set(bs)) and len(xs) == 0
