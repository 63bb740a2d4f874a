"""CPU oracle for level-scheduled SpTRSV with equation rewriting.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The oracle shares no code
with the GPU library (``paper_2103_11445_amd``) and neither imports the other.

The arithmetic lives in ``oracle.c`` (plain C, compiled with gcc and
``-ffp-contract=off``); this module only marshals numpy arrays through ctypes.
Every function cites the passage of the paper (arXiv:2103.11445) it follows;
the readings the paper leaves open are listed at the top of ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ORACLE_LIB points the loader at another build of oracle.c; the mutation
# check (tests/oracle_mutations.py) uses it to run the pins against copies of
# the oracle with a planted mistake
_LIB = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

KIND = {"none": 0, "threshold": 1, "explicit": 2}


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` next to the source with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC",
                        "-shared", _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        L = ctypes.c_int64
        D = ctypes.c_double
        sig = {
            "oracle_solve": (None, [I, P, P, P, P, P]),
            "oracle_solve_ld": (None, [I, P, P, P, P, P]),
            "oracle_solve_upper": (None, [I, P, P, P, P, P]),
            "oracle_levels": (I, [I, P, P, P]),
            "oracle_level_sets": (None, [I, P, I, P, P]),
            "oracle_select_stages": (I, [I, P, P, P, I, I, I, I, D, L, P, I, P, P]),
            "oracle_rewrite_count": (None, [I, P, P, P, I, P, P, P]),
            "oracle_rewrite": (I, [I, P, P, P, P, I, P, P, P, P, P, P, P]),
            "oracle_solve_rewritten": (None, [I, P, P, P, P, P, P, P, P]),
            "oracle_solve_levelset": (None, [I, P, P, I, P, P, P, P, P, P, P, P, I]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(row_ptr, col_idx, val=None):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    v = None if val is None else np.ascontiguousarray(val, dtype=np.float64)
    return rp, ci, v


# ---------------------------------------------------------------- solves --

def solve(row_ptr, col_idx, val, b) -> np.ndarray:
    """Serial forward substitution in FP64 (Sec. II, Algorithm 1).  ``b`` of
    shape (n,) or (n, k); columns are solved one after another."""
    rp, ci, v = _csr(row_ptr, col_idx, val)
    n = rp.size - 1
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 2:
        return np.stack([solve(rp, ci, v, b[:, c]) for c in range(b.shape[1])], axis=1)
    b = np.ascontiguousarray(b)
    x = np.empty(n, dtype=np.float64)
    _load().oracle_solve(n, _p(rp), _p(ci), _p(v), _p(b), _p(x))
    return x


def solve_upper(row_ptr, col_idx, val, b) -> np.ndarray:
    """Backward substitution in FP64 for an upper-triangular CSR matrix
    (diagonal first in each row).  ``b`` of shape (n,) or (n, k)."""
    rp, ci, v = _csr(row_ptr, col_idx, val)
    n = rp.size - 1
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 2:
        return np.stack([solve_upper(rp, ci, v, b[:, c]) for c in range(b.shape[1])], axis=1)
    b = np.ascontiguousarray(b)
    x = np.empty(n, dtype=np.float64)
    _load().oracle_solve_upper(n, _p(rp), _p(ci), _p(v), _p(b), _p(x))
    return x


def solve_ld(row_ptr, col_idx, val, b) -> np.ndarray:
    """Forward substitution in x87 extended precision, rounded to FP64."""
    rp, ci, v = _csr(row_ptr, col_idx, val)
    n = rp.size - 1
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 2:
        return np.stack([solve_ld(rp, ci, v, b[:, c]) for c in range(b.shape[1])], axis=1)
    b = np.ascontiguousarray(b)
    x = np.empty(n, dtype=np.float64)
    _load().oracle_solve_ld(n, _p(rp), _p(ci), _p(v), _p(b), _p(x))
    return x


# ------------------------------------------------------ levels and stages --

def levels(row_ptr, col_idx):
    """Level of each row of DAG_L (0-based) and the number of levels."""
    rp, ci, _ = _csr(row_ptr, col_idx)
    n = rp.size - 1
    lv = np.empty(n, dtype=np.int32)
    nlev = _load().oracle_levels(n, _p(rp), _p(ci), _p(lv))
    return lv, int(nlev)


def level_sets(level, nlev):
    """(level_ptr int32[nlev+1], rows int32[n]): rows of each level,
    ascending."""
    lv = np.ascontiguousarray(level, dtype=np.int32)
    ptr = np.empty(nlev + 1, dtype=np.int32)
    rows = np.empty(lv.size, dtype=np.int32)
    _load().oracle_level_sets(lv.size, _p(lv), nlev, _p(ptr), _p(rows))
    return ptr, rows


def select_stages(row_ptr, col_idx, level, nlev, policy: dict):
    """Stage of every level under ``policy`` (keys: kind in
    {'none','threshold','explicit'}, max_width, max_depth, max_fill,
    max_entries, absorb) and the entries each absorbed level adds."""
    rp, ci, _ = _csr(row_ptr, col_idx)
    n = rp.size - 1
    lv = np.ascontiguousarray(level, dtype=np.int32)
    sol = np.zeros(max(nlev, 1), dtype=np.int32)
    dol = np.zeros(max(nlev, 1), dtype=np.int64)
    absorb = policy.get("absorb")
    if absorb is None:
        absorb = np.zeros(1, dtype=np.uint8)
        alen = 0
    else:
        absorb = np.ascontiguousarray(absorb, dtype=np.uint8)
        alen = absorb.size
    ns = _load().oracle_select_stages(
        n, _p(rp), _p(ci), _p(lv), nlev, KIND[policy.get("kind", "threshold")],
        int(policy.get("max_width", 4)), int(policy.get("max_depth", 64)),
        float(policy.get("max_fill", 0.25)),
        int(policy.get("max_entries", 2**31 - 1)), _p(absorb), alen,
        _p(sol), _p(dol))
    return sol[:nlev].copy(), dol[:nlev].copy(), int(ns)


def rewrite(row_ptr, col_idx, val, level, nlev, stage_of_level):
    """Rewritten system: L' (CSR, int64 row pointer) and M (CSR, int64 row
    pointer) such that L' x = b + M b has the solution of L x = b."""
    rp, ci, v = _csr(row_ptr, col_idx, val)
    n = rp.size - 1
    lv = np.ascontiguousarray(level, dtype=np.int32)
    sol = np.ascontiguousarray(stage_of_level, dtype=np.int32)
    if sol.size == 0:
        sol = np.zeros(1, dtype=np.int32)
    lib = _load()
    nl = ctypes.c_int64()
    nm = ctypes.c_int64()
    lib.oracle_rewrite_count(n, _p(rp), _p(ci), _p(lv), nlev, _p(sol),
                             ctypes.byref(nl), ctypes.byref(nm))
    lp_ptr = np.empty(n + 1, dtype=np.int64)
    lp_col = np.empty(max(nl.value, 1), dtype=np.int32)
    lp_val = np.empty(max(nl.value, 1), dtype=np.float64)
    m_ptr = np.empty(n + 1, dtype=np.int64)
    m_col = np.empty(max(nm.value, 1), dtype=np.int32)
    m_val = np.empty(max(nm.value, 1), dtype=np.float64)
    if n == 0:
        lp_ptr[0] = m_ptr[0] = 0
    elif lib.oracle_rewrite(n, _p(rp), _p(ci), _p(v), _p(lv), nlev, _p(sol),
                            _p(lp_ptr), _p(lp_col), _p(lp_val),
                            _p(m_ptr), _p(m_col), _p(m_val)) != 0:
        raise MemoryError("oracle_rewrite: allocation failed")
    return ((lp_ptr, lp_col[:nl.value], lp_val[:nl.value]),
            (m_ptr, m_col[:nm.value], m_val[:nm.value]))


def solve_rewritten(lp, m, b) -> np.ndarray:
    """Serial solve of L' x = b + M b (Sec. III, Fig. 3)."""
    lp_ptr, lp_col, lp_val = (np.ascontiguousarray(a) for a in lp)
    m_ptr, m_col, m_val = (np.ascontiguousarray(a) for a in m)
    n = lp_ptr.size - 1
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 2:
        return np.stack([solve_rewritten(lp, m, b[:, c]) for c in range(b.shape[1])], axis=1)
    b = np.ascontiguousarray(b)
    x = np.empty(n, dtype=np.float64)
    _load().oracle_solve_rewritten(n, _p(lp_ptr), _p(lp_col), _p(lp_val),
                                   _p(m_ptr), _p(m_col), _p(m_val), _p(b), _p(x))
    return x


def solve_levelset(level_ptr, rows, lp, m, b, threads: int = 1) -> np.ndarray:
    """Level-set solve of L' x = b + M b on ``threads`` host cores (OpenMP,
    a barrier between levels; Sec. II), over the level sets (level_ptr, rows)
    of L'.  ``m=None`` for a plain system."""
    level_ptr = np.ascontiguousarray(level_ptr, dtype=np.int32)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    lp_ptr = np.ascontiguousarray(lp[0], dtype=np.int64)
    lp_col = np.ascontiguousarray(lp[1], dtype=np.int32)
    lp_val = np.ascontiguousarray(lp[2], dtype=np.float64)
    n = lp_ptr.size - 1
    if m is None:
        m = (np.zeros(n + 1, np.int64), np.zeros(1, np.int32), np.zeros(1, np.float64))
    m_ptr = np.ascontiguousarray(m[0], dtype=np.int64)
    m_col = np.ascontiguousarray(m[1], dtype=np.int32)
    m_val = np.ascontiguousarray(m[2], dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty(n, dtype=np.float64)
    _load().oracle_solve_levelset(n, _p(level_ptr), _p(rows), level_ptr.size - 1, _p(lp_ptr), _p(lp_col),
                                  _p(lp_val), _p(m_ptr), _p(m_col), _p(m_val), _p(b), _p(x), int(threads))
    return x


# -------------------------------------------------------------- the plan --

def plan(row_ptr, col_idx, val, policy: dict | None = None) -> dict:
    """Everything the analysis and rewrite steps produce, computed by the
    oracle: levels of L, stages, L' and M, levels of L' and the schedule
    (level sets of L', ascending row ids within a level)."""
    policy = policy or {"kind": "none"}
    rp, ci, v = _csr(row_ptr, col_idx, val)
    lv, nlev = levels(rp, ci)
    sol, dol, ns = select_stages(rp, ci, lv, nlev, policy)
    lp, m = rewrite(rp, ci, v, lv, nlev, sol)
    lp_ptr = lp[0].astype(np.int32) if lp[0][-1] < 2**31 else None
    lv2, nlev2 = levels(lp_ptr, lp[1]) if lp_ptr is not None else (None, None)
    sched_ptr, sched_rows = level_sets(lv2, nlev2)
    return {
        "level": lv, "nlev": nlev, "stage_of_level": sol, "delta_of_level": dol,
        "nstages": ns, "lp": lp, "m": m, "level_rw": lv2, "nlev_rw": nlev2,
        "sched_ptr": sched_ptr, "sched_rows": sched_rows,
    }


def flops(row_ptr, m_ptr=None) -> int:
    """FLOP count of one solve: a multiply and an add per stored
    off-diagonal x-term or b-term, one division per row."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    n = rp.size - 1
    off = int(rp[-1]) - n
    nm = 0 if m_ptr is None else int(np.asarray(m_ptr)[-1])
    return 2 * (off + nm) + n
