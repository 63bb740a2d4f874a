"""Level-scheduled sparse lower-triangular solve with equation rewriting on
MI355X (gfx950) -- Python binding of ``libsptrsv.so``.

This module only marshals arguments to the C ABI declared in
``include/sptrsv.h``: every step of analysis, rewriting and solving runs in
the library (host passes in C++, the solve in HIP kernels).  PyTorch is used
for device memory and streams only.  If the library is not built, importing
works but every call raises :class:`SptrsvError`; there is no fallback.

Method: arXiv:2103.11445 -- forward substitution over the level sets of
DAG_L (Sec. II) with rows of thin levels rewritten into earlier levels by
substituting their dependencies' equations (Sec. III).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = ["Plan", "Policy", "SptrsvError", "library_path", "load", "STATUS", "mlp_forward",
           "mlp_grad", "mlp_grad_noalloc", "mlp_adam", "probe_hop"]

_HERE = os.path.dirname(os.path.abspath(__file__))
# SPTRSV_LIB points the loader at another build of the same sources (the
# sanitizer check, tests/sanitizer_check.py, runs the host tests against an
# AddressSanitizer / UBSan build of the host passes)
_LIB_PATH = os.environ.get("SPTRSV_LIB") or os.path.join(_HERE, "libsptrsv.so")

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_CSR", 3: "ERR_DIAG", 4: "ERR_OVERFLOW",
          5: "ERR_OOM", 6: "ERR_HIP", 7: "ERR_STATE", 8: "ERR_TIMEOUT"}
KIND = {"none": 0, "threshold": 1, "explicit": 2, "learned": 3}
RHS_MODE = {"auto": 0, "mpass": 1, "stage": 2}
MLP_INPUTS = 6
MLP_PARAMS = 4673
INT32_MAX = 2**31 - 1


class SptrsvError(RuntimeError):
    """A library call returned a non-zero status."""

    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class Policy(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("max_width", ctypes.c_int32),
                ("max_depth", ctypes.c_int32), ("max_fill", ctypes.c_double),
                ("max_entries", ctypes.c_int64), ("absorb", ctypes.c_void_p),
                ("absorb_len", ctypes.c_int32), ("model", ctypes.c_void_p)]


class _Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("levels", ctypes.c_int32), ("stages", ctypes.c_int32),
                ("levels_rw", ctypes.c_int32), ("nnz", ctypes.c_int64), ("nnz_rw", ctypes.c_int64),
                ("nnz_m", ctypes.c_int64), ("flops", ctypes.c_int64), ("flops_rw", ctypes.c_int64),
                ("bytes", ctypes.c_int64), ("bytes_rw", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("precision", ctypes.c_int32), ("seg_tiles", ctypes.c_int64),
                ("rhs_mode", ctypes.c_int32), ("nnz_rhs", ctypes.c_int64),
                ("rhs_segments", ctypes.c_int32), ("reg_chunks", ctypes.c_int32),
                ("segments", ctypes.c_int32), ("ring_segments", ctypes.c_int32),
                ("chain_items", ctypes.c_int64), ("nnz_streamed", ctypes.c_int64),
                ("m_stored", ctypes.c_int32), ("compact_cols", ctypes.c_int32),
                ("compact_terms", ctypes.c_int64)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load ``libsptrsv.so`` (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise SptrsvError(6, f"{_LIB_PATH} is not built; run python -m paper_2103_11445_amd.build")
    lib = ctypes.CDLL(_LIB_PATH)
    P, I32, I64, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    S = ctypes.c_int
    sig = {
        "sptrsv_policy_default": (None, [P]),
        "sptrsv_analyse": (S, [I32, P, P, P, P]),
        "sptrsv_analyse_upper": (S, [I32, P, P, P, P]),
        "sptrsv_analyse_batch": (S, [I32, P, P, P, P, P, P]),
        "sptrsv_solve_graph": (S, [P, P, P, P]),
        "sptrsv_rewrite": (S, [P, P]),
        "sptrsv_device_bytes": (S, [P, P]),
        "sptrsv_upload": (S, [P, P, ctypes.c_size_t, P]),
        "sptrsv_solve": (S, [P, P, P, P]),
        "sptrsv_solve_fp32": (S, [P, P, P, P]),
        "sptrsv_solve_refined": (S, [P, P, P, I32, ctypes.c_double, P]),
        "sptrsv_refine_stats": (S, [P, P, P, P]),
        "sptrsv_set_precision": (S, [P, I32]),
        "sptrsv_set_rhs_mode": (S, [P, I32]),
        "sptrsv_set_tiling": (S, [P, I32]),
        "sptrsv_solve_stamped": (S, [P, P, P, P, P]),
        "sptrsv_plan_stamp_levels": (S, [P, P]),
        "sptrsv_plan_level_features": (S, [P, P]),
        "sptrsv_mlp_forward": (S, [P, P, P, I32, P]),
        "sptrsv_mlp_grad_workspace": (S, [I32, P]),
        "sptrsv_mlp_grad": (S, [P, P, P, I32, P, P, P, ctypes.c_size_t, P]),
        "sptrsv_mlp_grad_noalloc": (S, [P, P, P, I32, P, P, P]),
        "sptrsv_mlp_adam": (S, [P, P, P, P, I32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, P]),
        "sptrsv_check": (S, [P, P, P]),
        "sptrsv_set_wait_limit": (S, [P, U64]),
        "sptrsv_set_launch": (S, [P, I32]),
        "sptrsv_set_chain_share": (S, [P, I32]),
        "sptrsv_set_queues": (S, [P, I32]),
        "sptrsv_launch_shape": (S, [P, P, P]),
        "sptrsv_plan_info": (S, [P, P]),
        "sptrsv_plan_levels": (S, [P, I32, P]),
        "sptrsv_plan_stages": (S, [P, P, P]),
        "sptrsv_plan_schedule": (S, [P, P, P]),
        "sptrsv_plan_export": (S, [P, P, P, P, P, P, P]),
        "sptrsv_probe_hop": (S, [I32, I32, P, ctypes.c_size_t, P, P]),
        "sptrsv_plan_destroy": (None, [P]),
        "sptrsv_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise SptrsvError(status, load().sptrsv_last_error().decode())


def _ptr(a) -> ctypes.c_void_p:
    if a is None:
        return ctypes.c_void_p(0)
    if isinstance(a, np.ndarray):
        return ctypes.c_void_p(a.ctypes.data)
    return ctypes.c_void_p(a.data_ptr())  # torch tensor


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_policy(kind: str = "threshold", max_width: int = 4, max_depth: int = 64,
                max_fill: float = 0.25, max_entries: int = INT32_MAX, absorb=None, model=None):
    """A :class:`Policy` (and the mask array that must outlive the call).
    ``model``: a float32 CUDA tensor of MLP_PARAMS parameters (LEARNED)."""
    mask = None
    if absorb is not None:
        mask = np.ascontiguousarray(absorb, dtype=np.uint8)
    pol = Policy(KIND[kind], int(max_width), int(max_depth), float(max_fill), int(max_entries),
                 None if mask is None else mask.ctypes.data, 0 if mask is None else mask.size,
                 None if model is None else model.data_ptr())
    return pol, mask


class Plan:
    """Analysis, rewrite and solve of one triangular CSR matrix (lower by
    default; ``upper=True`` for backward substitution, diagonal first)."""

    @classmethod
    def batch(cls, systems, k=None) -> "Plan":
        """One plan for many lower-triangular systems, ``systems`` a list of
        (row_ptr, col_idx, val) and ``k`` the right-hand sides of each (default
        1).  Solve with the concatenation of row-major n_j x k_j blocks."""
        lib = load()
        count = len(systems)
        keep = [(np.ascontiguousarray(r, np.int32), np.ascontiguousarray(c, np.int32),
                 np.ascontiguousarray(v, np.float64)) for r, c, v in systems]
        ns = np.array([r.size - 1 for r, _, _ in keep], dtype=np.int32)
        ks = np.ascontiguousarray(np.ones(count, np.int32) if k is None else k, dtype=np.int32)
        ptrs = [(ctypes.c_void_p * max(count, 1))(*[a.ctypes.data for a in col]) for col in zip(*keep)] \
            if count else [(ctypes.c_void_p * 1)() for _ in range(3)]
        h = ctypes.c_void_p()
        _check(lib.sptrsv_analyse_batch(count, _ptr(ns), ctypes.cast(ptrs[0], ctypes.c_void_p),
                                        ctypes.cast(ptrs[1], ctypes.c_void_p),
                                        ctypes.cast(ptrs[2], ctypes.c_void_p), _ptr(ks), ctypes.byref(h)))
        self = cls.__new__(cls)
        self._h = h
        self.n = int(np.sum(ns.astype(np.int64) * ks))
        self._buf = None
        self._rp = None
        return self

    def __init__(self, row_ptr, col_idx, val, upper: bool = False):
        lib = load()
        self._rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        v = np.ascontiguousarray(val, dtype=np.float64)
        n = self._rp.size - 1
        h = ctypes.c_void_p()
        fn = lib.sptrsv_analyse_upper if upper else lib.sptrsv_analyse
        _check(fn(n, _ptr(self._rp), _ptr(ci), _ptr(v), ctypes.byref(h)))
        self._h = h
        self.n = n
        self._buf = None

    # ---------------------------------------------------------- host side --
    def rewrite(self, kind: str = "threshold", **kw) -> "Plan":
        pol, mask = make_policy(kind, **kw)
        _check(load().sptrsv_rewrite(self._h, ctypes.byref(pol)))
        del mask
        return self

    def info(self) -> dict:
        o = _Info()
        _check(load().sptrsv_plan_info(self._h, ctypes.byref(o)))
        return {f: getattr(o, f) for f, _ in _Info._fields_}

    def levels(self, which: int = 0) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int32)
        _check(load().sptrsv_plan_levels(self._h, which, _ptr(out)))
        return out

    def stages(self):
        nlev = self.info()["levels"]
        s = np.empty(max(nlev, 1), dtype=np.int32)
        d = np.empty(max(nlev, 1), dtype=np.int64)
        _check(load().sptrsv_plan_stages(self._h, _ptr(s), _ptr(d)))
        return s[:nlev], d[:nlev]

    def schedule(self):
        nl = self.info()["levels_rw"]
        ptr = np.empty(nl + 1, dtype=np.int32)
        rows = np.empty(self.n, dtype=np.int32)
        _check(load().sptrsv_plan_schedule(self._h, _ptr(ptr), _ptr(rows)))
        return ptr, rows

    def export(self, with_m: bool = True):
        """(L', M) as CSR triples; M is None with ``with_m=False``."""
        i = self.info()
        lp = (np.empty(self.n + 1, np.int64), np.empty(i["nnz_rw"], np.int32),
              np.empty(i["nnz_rw"], np.float64))
        m = (np.empty(self.n + 1, np.int64), np.empty(i["nnz_m"], np.int32),
             np.empty(i["nnz_m"], np.float64)) if with_m else (None, None, None)
        _check(load().sptrsv_plan_export(self._h, *(_ptr(a) for a in lp), *(_ptr(a) for a in m)))
        return lp, (m if with_m else None)

    def set_launch(self, waves_per_cu: int = 0):
        _check(load().sptrsv_set_launch(self._h, int(waves_per_cu)))
        return self

    def set_queues(self, queues: int = 2) -> "Plan":
        """Work queues of the device schedule: 2 (chain and sinks apart) or
        1 (every row in level order); repacks."""
        _check(load().sptrsv_set_queues(self._h, int(queues)))
        return self

    def set_chain_share(self, per_mille: int = 0):
        """Share of the waves (per mille) serving the chain queue (rows other
        rows depend on); 0 = chosen from the plan's work."""
        _check(load().sptrsv_set_chain_share(self._h, int(per_mille)))
        return self

    def launch_shape(self):
        """(waves, waves serving the chain queue) of the next solve."""
        w, c = ctypes.c_int32(), ctypes.c_int32()
        _check(load().sptrsv_launch_shape(self._h, ctypes.byref(w), ctypes.byref(c)))
        return w.value, c.value

    def set_wait_limit(self, ticks: int):
        _check(load().sptrsv_set_wait_limit(self._h, int(ticks)))

    def set_tiling(self, terms_per_lane: int = 4) -> "Plan":
        """Row-to-wavefront tiling: terms per lane before a row gets more
        lanes (1, 2, 4, 8 or 16; repacks)."""
        _check(load().sptrsv_set_tiling(self._h, int(terms_per_lane)))
        return self

    def set_rhs_mode(self, mode: str = "auto") -> "Plan":
        """How b' = b + M b is applied: 'auto', 'mpass' or 'stage' (repacks)."""
        _check(load().sptrsv_set_rhs_mode(self._h, RHS_MODE[mode]))
        return self

    def set_precision(self, bits: int) -> "Plan":
        """Value type of the device image: 64 or 32 (repacks; upload again)."""
        _check(load().sptrsv_set_precision(self._h, int(bits)))
        return self

    # -------------------------------------------------------- device side --
    def upload(self, device=None, stream=None) -> "Plan":
        """Allocate the device buffer with torch and copy the plan into it."""
        import torch
        nb = ctypes.c_size_t()
        _check(load().sptrsv_device_bytes(self._h, ctypes.byref(nb)))
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self._buf = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=dev)
        _check(load().sptrsv_upload(self._h, _ptr(self._buf), self._buf.numel(), _stream(stream)))
        return self

    def solve(self, b, x=None, stream=None):
        """Enqueue x = L^-1 b on ``stream`` (default: torch's current stream)
        and return x (a float64 CUDA tensor)."""
        import torch
        if x is None:
            x = torch.empty_like(b)
        _check(load().sptrsv_solve(self._h, _ptr(b), _ptr(x), _stream(stream)))
        return x

    def solve_graph(self, b, x=None, stream=None):
        """As :meth:`solve`, replaying a captured HIP graph for these b, x."""
        import torch
        if x is None:
            x = torch.empty_like(b)
        _check(load().sptrsv_solve_graph(self._h, _ptr(b), _ptr(x), _stream(stream)))
        return x

    def solve_fp32(self, b, x=None, stream=None):
        """Enqueue the FP32 solve of a plan stored in FP32 (float32 tensors)."""
        import torch
        if x is None:
            x = torch.empty_like(b)
        _check(load().sptrsv_solve_fp32(self._h, _ptr(b), _ptr(x), _stream(stream)))
        return x

    def solve_refined(self, b, x=None, iterations: int = 10, tol: float = 1e-13, stream=None):
        """Enqueue FP32 solves refined by FP64 residuals and updates (plan
        stored in FP32; float64 tensors)."""
        import torch
        if x is None:
            x = torch.empty_like(b)
        _check(load().sptrsv_solve_refined(self._h, _ptr(b), _ptr(x), int(iterations), float(tol),
                                           _stream(stream)))
        return x

    def refine_stats(self, stream=None):
        """(steps applied, relative correction of the last step)."""
        it = ctypes.c_int32()
        corr = ctypes.c_double()
        _check(load().sptrsv_refine_stats(self._h, _stream(stream), ctypes.byref(it), ctypes.byref(corr)))
        return it.value, corr.value

    def solve_stamped(self, b, x, stamps, stream=None):
        """Instrumented solve: ``stamps`` an int64 CUDA tensor of
        ``info()['tiles'] + info()['seg_tiles'] + 1`` entries."""
        _check(load().sptrsv_solve_stamped(self._h, _ptr(b), _ptr(x), _ptr(stamps), _stream(stream)))
        return x

    def stamp_levels(self) -> np.ndarray:
        i = self.info()
        out = np.empty(i["tiles"] + i["seg_tiles"], dtype=np.int32)
        _check(load().sptrsv_plan_stamp_levels(self._h, _ptr(out)))
        return out

    def level_features(self) -> np.ndarray:
        nl = self.info()["levels_rw"]
        out = np.empty((nl, MLP_INPUTS), dtype=np.float32)
        _check(load().sptrsv_plan_level_features(self._h, _ptr(out)))
        return out

    def check(self, stream=None) -> int:
        st = ctypes.c_int32()
        _check(load().sptrsv_check(self._h, _stream(stream), ctypes.byref(st)))
        return st.value

    def close(self):
        if getattr(self, "_h", None):
            load().sptrsv_plan_destroy(self._h)
            self._h = None
        self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def probe_hop(hops: int = 20000, same_xcd: bool = False, scratch=None, stream=None) -> float:
    """Mean nanoseconds of one dependency hop (device-scope publish seen by a
    device-scope poll on another compute unit)."""
    import torch
    if scratch is None:
        scratch = torch.zeros(8, dtype=torch.int64, device="cuda")
    ns = ctypes.c_double()
    _check(load().sptrsv_probe_hop(int(hops), int(bool(same_xcd)), _ptr(scratch), scratch.numel() * 8,
                                   ctypes.byref(ns), _stream(stream)))
    return ns.value


# ------------------------------------------------------------- cost model --

def mlp_forward(params, x, y=None, stream=None):
    """y = model(x) for the rows of x (float32 CUDA tensors; x of shape
    (m, MLP_INPUTS))."""
    import torch
    if y is None:
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    _check(load().sptrsv_mlp_forward(_ptr(params), _ptr(x), _ptr(y), int(x.shape[0]), _stream(stream)))
    return y


def mlp_grad(params, x, t, grad=None, loss=None, workspace=None, stream=None):
    """Gradient of the mean squared error of the model on (x, t); returns
    (grad, loss) as CUDA tensors (loss a one-element tensor)."""
    import torch
    m = int(x.shape[0])
    nb = ctypes.c_size_t()
    _check(load().sptrsv_mlp_grad_workspace(m, ctypes.byref(nb)))
    if workspace is None or workspace.numel() < nb.value:
        workspace = torch.empty(nb.value, dtype=torch.uint8, device=x.device)
    if grad is None:
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
    _check(load().sptrsv_mlp_grad(_ptr(params), _ptr(x), _ptr(t), m, _ptr(grad), _ptr(loss),
                                  _ptr(workspace), workspace.numel(), _stream(stream)))
    return grad, loss


MLP_NOALLOC_MAX_SAMPLES = 8192


def mlp_grad_noalloc(params, x, t, grad=None, loss=None, stream=None):
    """As :func:`mlp_grad` with the library's static device workspace (no
    allocation by the library; at most MLP_NOALLOC_MAX_SAMPLES samples).
    ``grad`` and ``loss`` are allocated here only when not given."""
    import torch
    m = int(x.shape[0])
    if grad is None:
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
    _check(load().sptrsv_mlp_grad_noalloc(_ptr(params), _ptr(x), _ptr(t), m, _ptr(grad), _ptr(loss),
                                          _stream(stream)))
    return grad, loss


def mlp_adam(params, grad, m1, m2, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
             eps: float = 1e-8, stream=None):
    """One Adam step in place on params (float32 CUDA tensors)."""
    _check(load().sptrsv_mlp_adam(_ptr(params), _ptr(grad), _ptr(m1), _ptr(m2), int(step), float(lr),
                                  float(beta1), float(beta2), float(eps), _stream(stream)))
    return params
