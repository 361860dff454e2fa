"""ctypes binding of libpfk (argument marshalling only).

Names follow the C ABI of include/pfk.h.  Device vectors are torch tensors of
dtype float64 on a HIP device; host arrays are numpy float64.  Nothing here
computes: every operation is a call into the library.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libpfk.so")

FCG, PIPEFCG, GCR, PIPEGCR, FGMRES, PIPEFGMRES = range(6)
PIPEGCR_W = 6
PIPEFCG_NAIVE = 7
METHODS = {"fcg": FCG, "pipefcg": PIPEFCG, "gcr": GCR, "pipegcr": PIPEGCR,
           "fgmres": FGMRES, "pipefgmres": PIPEFGMRES, "pipegcr_w": PIPEGCR_W,
           "pipefcg_naive": PIPEFCG_NAIVE}
PC_NONE, PC_JACOBI, PC_JACOBI_PCG, PC_JACOBI_GMRES, PC_BLOCK_JACOBI_PCG, PC_NOISY = range(6)
PC_KINDS = {"none": PC_NONE, "jacobi": PC_JACOBI, "jacobi_pcg": PC_JACOBI_PCG,
            "jacobi_gmres": PC_JACOBI_GMRES, "block_jacobi_pcg": PC_BLOCK_JACOBI_PCG, "noisy": PC_NOISY}
FP64, FP32_BF16COEF = 0, 1

STATUS_NAMES = {0: "ok", 1: "not_converged", -1: "err_arg", -2: "err_oom", -3: "err_hip",
                -4: "err_nonfinite", -5: "err_breakdown"}

# every symbol include/pfk.h declares
EXPORTED = [
    "pfk_default_opts", "pfk_operator_create", "pfk_operator_destroy", "pfk_operator_size",
    "pfk_operator_apply", "pfk_operator_diag_inv", "pfk_precond_create", "pfk_precond_create_noisy",
    "pfk_precond_destroy",
    "pfk_precond_apply", "pfk_workspace_bytes", "pfk_solve", "pfk_solve_noalloc", "pfk_session_create",
    "pfk_session_start", "pfk_session_iterate", "pfk_session_sync", "pfk_session_destroy",
    "pfk_session_profile", "pfk_estimate_sigma", "pfk_last_error",
    "pfk_operator_set_tiling", "pfk_operator_get_tiling", "pfk_operator_autotune",
    "pfk_batch_create", "pfk_batch_destroy", "pfk_batch_add", "pfk_batch_step", "pfk_batch_poll",
    "pfk_batch_info", "pfk_batch_remove", "pfk_batch_workspace_bytes", "pfk_solve_batched",
    "pfk_batch_set_barrier_limit",
    "pfk_server_create", "pfk_server_destroy", "pfk_server_submit", "pfk_server_progress",
    "pfk_server_result", "pfk_server_stats",
]


class Tuning(C.Structure):
    _fields_ = [("tile_x", C.c_int), ("stencil_target", C.c_int), ("stencil_blocks", C.c_int),
                ("vector_blocks", C.c_int),
                ("ms_per_iteration", C.c_double), ("ms_default", C.c_double), ("candidates", C.c_int)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_active", C.c_int), ("step_iters", C.c_int), ("mmax", C.c_int),
                ("launch_direct", C.c_int), ("stall_window", C.c_int), ("max_restarts", C.c_int)]


class ServerStatus(C.Structure):
    _fields_ = [("queued", C.c_longlong), ("active", C.c_longlong), ("completed", C.c_longlong),
                ("bytes_in_use", C.c_size_t), ("bytes_held", C.c_size_t)]


class PfkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class SolveOpts(C.Structure):
    _fields_ = [("truncation", C.c_int), ("shift_sigma", C.c_double), ("graph_iters", C.c_int),
                ("use_graph", C.c_int), ("host_sync", C.c_int), ("max_restarts", C.c_int),
                ("force_breakdown_at", C.c_int), ("persistent", C.c_int), ("norm", C.c_int),
                ("timestamps", C.c_int), ("stall_window", C.c_int), ("side_delay", C.c_int)]


class _Info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("status", C.c_int), ("true_rel_resid", C.c_double),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int), ("history_len", C.c_int),
                ("natural_history", C.POINTER(C.c_double)), ("natural_len", C.c_int),
                ("iter_time_us", C.POINTER(C.c_double)), ("iter_time_len", C.c_int)]


@dataclass
class SolveInfo:
    status: int
    iterations: int
    restarts: int
    converged: bool
    true_rel_resid: float
    history: np.ndarray
    natural: np.ndarray = None      # sqrt|gamma_i| per iteration (CG/CR types), else empty
    iter_time_us: np.ndarray = None  # device time of each history entry (opts timestamps=1), else empty

    @property
    def status_name(self) -> str:
        return STATUS_NAMES.get(self.status, str(self.status))


_lib_handle = None


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """Load libpfk.so (raises if it has not been built)."""
    global _lib_handle
    if _lib_handle is not None:
        return _lib_handle
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_1511_07226_amd.build`")
    L = C.CDLL(_LIB_PATH)
    vp, i64p = C.c_void_p, C.POINTER(C.c_int64)
    sig = {
        "pfk_default_opts": (None, [C.POINTER(SolveOpts)]),
        "pfk_operator_create": (C.c_int, [C.c_int, i64p, vp, vp, C.c_int, C.POINTER(vp)]),
        "pfk_operator_destroy": (None, [vp]),
        "pfk_operator_size": (C.c_int64, [vp]),
        "pfk_operator_apply": (C.c_int, [vp, vp, vp, vp]),
        "pfk_operator_diag_inv": (C.c_int, [vp, vp, vp]),
        "pfk_precond_create": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(vp)]),
        "pfk_precond_create_noisy": (C.c_int, [vp, C.c_double, C.c_uint64, C.POINTER(vp)]),
        "pfk_precond_destroy": (None, [vp]),
        "pfk_precond_apply": (C.c_int, [vp, vp, vp, vp]),
        "pfk_workspace_bytes": (C.c_size_t, [vp, vp, C.c_int, C.c_int, C.c_int]),
        "pfk_solve": (C.c_int, [vp, vp, C.c_int, vp, vp, C.c_double, C.c_int, C.c_int, vp, C.c_size_t,
                                vp, C.POINTER(SolveOpts), C.POINTER(_Info)]),
        "pfk_solve_noalloc": (C.c_int, [vp, vp, C.c_int, vp, vp, C.c_double, C.c_int, C.c_int, vp,
                                        C.POINTER(SolveOpts), C.POINTER(_Info)]),
        "pfk_session_create": (C.c_int, [vp, vp, C.c_int, vp, vp, C.c_double, C.c_int, C.c_int, vp,
                                         C.c_size_t, vp, C.POINTER(SolveOpts), C.POINTER(vp)]),
        "pfk_session_start": (C.c_int, [vp]),
        "pfk_session_iterate": (C.c_int, [vp, C.c_int]),
        "pfk_session_sync": (C.c_int, [vp, C.POINTER(_Info)]),
        "pfk_session_destroy": (None, [vp]),
        "pfk_session_profile": (C.c_int, [vp, C.c_int, C.c_int, C.POINTER(C.c_char_p),
                                          C.POINTER(C.c_double), C.POINTER(C.c_int)]),
        "pfk_estimate_sigma": (C.c_int, [vp, vp, C.c_int, C.POINTER(C.c_double), vp]),
        "pfk_last_error": (C.c_char_p, []),
        "pfk_operator_set_tiling": (C.c_int, [vp, C.c_int, C.c_int, C.c_int]),
        "pfk_operator_get_tiling": (C.c_int, [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "pfk_operator_autotune": (C.c_int, [vp, vp, C.c_int, C.c_int, C.c_int, vp, C.POINTER(Tuning)]),
        "pfk_batch_create": (C.c_int, [C.c_int, C.c_int, C.c_int, vp, C.POINTER(SolveOpts), C.POINTER(vp)]),
        "pfk_batch_destroy": (None, [vp]),
        "pfk_batch_add": (C.c_int, [vp, vp, vp, vp, vp, C.c_double, C.c_int, vp, C.c_size_t,
                                    C.POINTER(C.c_int)]),
        "pfk_batch_step": (C.c_int, [vp, C.c_int]),
        "pfk_batch_poll": (C.c_int, [vp, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "pfk_batch_info": (C.c_int, [vp, C.c_int, C.POINTER(_Info)]),
        "pfk_batch_remove": (C.c_int, [vp, C.c_int]),
        "pfk_batch_set_barrier_limit": (C.c_int, [vp, C.c_longlong]),
        "pfk_batch_workspace_bytes": (C.c_size_t, [vp, vp, C.c_int, C.c_int, C.c_int]),
        "pfk_server_create": (C.c_int, [C.POINTER(ServerConfig), vp, C.POINTER(vp)]),
        "pfk_server_destroy": (None, [vp]),
        "pfk_server_submit": (C.c_int, [vp, vp, vp, C.c_int, vp, vp, C.c_double, C.c_int,
                                        C.POINTER(C.c_longlong)]),
        "pfk_server_progress": (C.c_int, [vp, C.POINTER(C.c_longlong), C.c_int, C.POINTER(C.c_int)]),
        "pfk_server_result": (C.c_int, [vp, C.c_longlong, C.POINTER(_Info)]),
        "pfk_server_stats": (C.c_int, [vp, C.POINTER(ServerStatus)]),
        "pfk_solve_batched": (C.c_int, [C.c_int, C.POINTER(vp), C.POINTER(vp), C.c_int, C.POINTER(vp),
                                        C.POINTER(vp), C.POINTER(C.c_double), C.c_int, C.c_int, vp, C.c_size_t,
                                        vp, C.POINTER(SolveOpts), C.POINTER(_Info)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib_handle = L
    return L


def _check(code: int, allow_positive: bool = False) -> int:
    if code < 0 or (code > 0 and not allow_positive):
        raise PfkError(code, lib().pfk_last_error().decode())
    return code


def _stream_ptr(stream) -> int | None:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev_ptr(t, N: int | None = None, name: str = "vector") -> int:
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 torch tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if N is not None and t.numel() != N:
        raise ValueError(f"{name} has {t.numel()} values, expected {N}")
    return t.data_ptr()


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().pfk_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Operator:
    """A = -div(eta grad .) [+ upwind div(v .)] on n^dim interior nodes."""

    def __init__(self, dim: int, n: int, eta: np.ndarray, vel: np.ndarray | None = None):
        eta = np.ascontiguousarray(eta, dtype=np.float64)
        if eta.size != (n + 2) ** dim:
            raise ValueError("eta must hold (n+2)^dim values")
        nn = (C.c_int64 * 3)(n, n, n if dim == 3 else 1)
        velp = None
        if vel is not None:
            vel = np.ascontiguousarray(vel, dtype=np.float64)
            if vel.size != 3 * (n + 2) ** 3:
                raise ValueError("vel must hold 3*(n+2)^3 values")
            velp = vel.ctypes.data
        h = C.c_void_p()
        _check(lib().pfk_operator_create(dim, nn, eta.ctypes.data, velp, 0, C.byref(h)))
        self._h = h
        self.dim, self.n = dim, n
        self.N = int(lib().pfk_operator_size(h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib_handle is not None:
            _lib_handle.pfk_operator_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def apply(self, x, y=None, stream=None):
        import torch
        if y is None:
            y = torch.empty_like(x)
        _check(lib().pfk_operator_apply(self._h, _dev_ptr(x, self.N, "x"), _dev_ptr(y, self.N, "y"),
                                        _stream_ptr(stream)))
        return y

    def tiling(self) -> tuple:
        """(tile_x, stencil workgroups, vector workgroups) of this operator's launches."""
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        _check(lib().pfk_operator_get_tiling(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def set_tiling(self, tile_x: int, stencil_target: int, vector_blocks: int):
        _check(lib().pfk_operator_set_tiling(self._h, int(tile_x), int(stencil_target), int(vector_blocks)))

    def autotune(self, B, method: str = "pipefcg", mmax: int = 30, reps: int = 5, stream=None) -> dict:
        """Time candidate launch geometries on this GPU and keep the fastest."""
        t = Tuning()
        _check(lib().pfk_operator_autotune(self._h, B.handle, METHODS[method], int(mmax), int(reps),
                                           _stream_ptr(stream), C.byref(t)))
        return t.as_dict()

    def diag_inv(self, stream=None):
        import torch
        d = torch.empty(self.N, dtype=torch.float64, device="cuda")
        _check(lib().pfk_operator_diag_inv(self._h, d.data_ptr(), _stream_ptr(stream)))
        return d


class Precond:
    """Flexible preconditioner B of the given kind on operator A.

    kind "noisy" is the seeded Gaussian-noise preconditioner of the section
    2.2.1 study (``eta``, ``seed``; the other arguments are ignored).
    """

    def __init__(self, A: Operator, kind: str = "jacobi_pcg", inner_its: int = 5,
                 precision: int = FP64, block: int = 8, eta: float = 0.0, seed: int = 0):
        h = C.c_void_p()
        if kind == "noisy":
            _check(lib().pfk_precond_create_noisy(A.handle, float(eta), int(seed), C.byref(h)))
        else:
            _check(lib().pfk_precond_create(A.handle, PC_KINDS[kind], inner_its, precision, block, C.byref(h)))
        self._h = h
        self.A = A
        self.kind, self.inner_its, self.precision, self.block = kind, inner_its, precision, block
        self.eta, self.seed = eta, seed

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib_handle is not None:
            _lib_handle.pfk_precond_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def apply(self, v, y=None, stream=None):
        import torch
        if y is None:
            y = torch.empty_like(v)
        _check(lib().pfk_precond_apply(self._h, _dev_ptr(v, self.A.N, "v"), _dev_ptr(y, self.A.N, "y"),
                                       _stream_ptr(stream)))
        return y


def workspace_bytes(A: Operator, B: Precond, method: str, mmax: int, maxit: int) -> int:
    return int(lib().pfk_workspace_bytes(A.handle, B.handle, METHODS[method], mmax, maxit))


def estimate_sigma(A: Operator, B: Precond, its: int = 10, stream=None) -> float:
    """PIPEFGMRES shift: Rayleigh quotient of v -> A B(v) after `its` power steps."""
    sig = C.c_double()
    _check(lib().pfk_estimate_sigma(A.handle, B.handle, int(its), C.byref(sig), _stream_ptr(stream)))
    return sig.value


def _info_struct(cap: int, info=None):
    """An info record with host buffers for the histories (row 0: the
    residual measure, row 1: the natural norm, row 2: device timestamps)."""
    info = _Info() if info is None else info
    hist = np.zeros((3, max(cap, 1)), dtype=np.float64)
    info.history = hist[0].ctypes.data_as(C.POINTER(C.c_double))
    info.natural_history = hist[1].ctypes.data_as(C.POINTER(C.c_double))
    info.iter_time_us = hist[2].ctypes.data_as(C.POINTER(C.c_double))
    info.history_cap = cap
    return info, hist


def _to_info(code: int, info: _Info, hist: np.ndarray) -> SolveInfo:
    return SolveInfo(code, info.iterations, info.restarts, bool(info.converged), info.true_rel_resid,
                     hist[0, : info.history_len].copy(), hist[1, : info.natural_len].copy(),
                     hist[2, : info.iter_time_len].copy())


def solve(A: Operator, B: Precond, method: str, b, x, rtol: float = 1e-8, maxit: int = 500,
          mmax: int = 30, workspace=None, stream=None, **opts) -> SolveInfo:
    """Solve A x = b in place on x (device float64 tensors).  Returns SolveInfo."""
    o = default_opts(**opts)
    info, hist = _info_struct(maxit + 1)
    wsp, wsb = (None, 0)
    if workspace is not None:
        wsp, wsb = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    code = lib().pfk_solve(A.handle, B.handle, METHODS[method], _dev_ptr(b, A.N, "b"), _dev_ptr(x, A.N, "x"),
                           float(rtol), int(maxit), int(mmax), wsp, wsb, _stream_ptr(stream), C.byref(o),
                           C.byref(info))
    _check(code, allow_positive=True)
    return _to_info(code, info, hist)


def solve_noalloc(A: Operator, B: Precond, method: str, b, x, rtol: float = 1e-8, maxit: int = 500,
                  mmax: int = 30, stream=None, **opts) -> SolveInfo:
    """solve() through pfk_solve_noalloc: the library's fixed device workspace,
    one stream, no allocation (for callers that cannot allocate)."""
    o = default_opts(**opts)
    info, hist = _info_struct(maxit + 1)
    code = lib().pfk_solve_noalloc(A.handle, B.handle, METHODS[method], _dev_ptr(b, A.N, "b"),
                                   _dev_ptr(x, A.N, "x"), float(rtol), int(maxit), int(mmax), _stream_ptr(stream),
                                   C.byref(o), C.byref(info))
    _check(code, allow_positive=True)
    return _to_info(code, info, hist)


class Session:
    """Asynchronous solve: start(), iterate(k), sync()."""

    def __init__(self, A: Operator, B: Precond, method: str, b, x, rtol: float = 1e-8, maxit: int = 500,
                 mmax: int = 30, workspace=None, stream=None, **opts):
        self.A, self.B, self.b, self.x = A, B, b, x
        self.maxit = maxit
        o = default_opts(**opts)
        wsp, wsb = (None, 0)
        if workspace is not None:
            wsp, wsb = workspace.data_ptr(), workspace.numel() * workspace.element_size()
        h = C.c_void_p()
        _check(lib().pfk_session_create(A.handle, B.handle, METHODS[method], _dev_ptr(b, A.N, "b"),
                                        _dev_ptr(x, A.N, "x"), float(rtol), int(maxit), int(mmax), wsp, wsb,
                                        _stream_ptr(stream), C.byref(o), C.byref(h)))
        self._h = h
        self._ws = workspace

    def start(self):
        _check(lib().pfk_session_start(self._h))

    def iterate(self, iters: int):
        _check(lib().pfk_session_iterate(self._h, int(iters)))

    def sync(self) -> SolveInfo:
        info, hist = _info_struct(self.maxit + 1)
        code = lib().pfk_session_sync(self._h, C.byref(info))
        _check(code, allow_positive=True)
        return _to_info(code, info, hist)

    def profile(self, iters: int) -> dict:
        """Per-kernel event timing over `iters` directly launched iterations:
        {kernel name: (total ms, launches)}."""
        cap = 64
        names = (C.c_char_p * cap)()
        ms = (C.c_double * cap)()
        cnt = (C.c_int * cap)()
        n = lib().pfk_session_profile(self._h, int(iters), cap, names, ms, cnt)
        _check(min(n, 0))
        return {names[i].decode(): (ms[i], cnt[i]) for i in range(min(n, cap))}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pfk_session_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many systems advanced by shared launches: add(), step(k), poll(), info()."""

    def __init__(self, method: str, mmax: int = 30, capacity: int = 64, stream=None, **opts):
        o = default_opts(**opts)
        h = C.c_void_p()
        _check(lib().pfk_batch_create(METHODS[method], int(mmax), int(capacity), _stream_ptr(stream), C.byref(o),
                                      C.byref(h)))
        self._h = h
        self.method, self.mmax, self.capacity = method, mmax, capacity
        self._keep = {}            # slot -> objects that must outlive the member
        self._maxit = {}

    def add(self, A: Operator, B: Precond, b, x, rtol: float = 1e-8, maxit: int = 500, workspace=None) -> int:
        wsp, wsb = (None, 0)
        if workspace is not None:
            wsp, wsb = workspace.data_ptr(), workspace.numel() * workspace.element_size()
        slot = C.c_int(-1)
        _check(lib().pfk_batch_add(self._h, A.handle, B.handle, _dev_ptr(b, A.N, "b"), _dev_ptr(x, A.N, "x"),
                                   float(rtol), int(maxit), wsp, wsb, C.byref(slot)))
        self._keep[slot.value] = (A, B, b, x, workspace)
        self._maxit[slot.value] = maxit
        return slot.value

    def step(self, iters: int):
        _check(lib().pfk_batch_step(self._h, int(iters)))

    def poll(self):
        """Returns (finished slots, number still running)."""
        cap = self.capacity
        fin = (C.c_int * cap)()
        nf, nr = C.c_int(0), C.c_int(0)
        _check(lib().pfk_batch_poll(self._h, fin, cap, C.byref(nf), C.byref(nr)))
        return [fin[i] for i in range(nf.value)], nr.value

    def info(self, slot: int) -> SolveInfo:
        info, hist = _info_struct(self._maxit[slot] + 1)
        code = lib().pfk_batch_info(self._h, int(slot), C.byref(info))
        _check(code, allow_positive=True)
        return _to_info(code, info, hist)

    def set_barrier_limit(self, polls: int):
        """Test hook: polls before a persistent launch's grid barrier gives up."""
        _check(lib().pfk_batch_set_barrier_limit(self._h, int(polls)))

    def remove(self, slot: int):
        _check(lib().pfk_batch_remove(self._h, int(slot)))
        self._keep.pop(slot, None)
        self._maxit.pop(slot, None)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pfk_batch_destroy(self._h)
            self._h = None
        self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batched(As, Bs, method: str, bs, xs, rtol=1e-8, maxit: int = 500, mmax: int = 30, workspace=None,
                  stream=None, **opts):
    """Solve every system (lists of operators, preconditioners, b and x tensors)
    in one batch.  Returns (status code, [SolveInfo])."""
    n = len(As)
    o = default_opts(**opts)
    rt = [float(rtol)] * n if np.isscalar(rtol) else [float(v) for v in rtol]
    arrA = (C.c_void_p * n)(*[a.handle.value for a in As])
    arrB = (C.c_void_p * n)(*[b.handle.value for b in Bs])
    arrb = (C.c_void_p * n)(*[_dev_ptr(v, a.N, "b") for v, a in zip(bs, As)])
    arrx = (C.c_void_p * n)(*[_dev_ptr(v, a.N, "x") for v, a in zip(xs, As)])
    arrr = (C.c_double * n)(*rt)
    infos = (_Info * n)()
    hists = [_info_struct(maxit + 1, infos[i])[1] for i in range(n)]
    wsp, wsb = (None, 0)
    if workspace is not None:
        wsp, wsb = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    code = lib().pfk_solve_batched(n, arrA, arrB, METHODS[method], arrb, arrx, arrr, int(maxit), int(mmax),
                                   wsp, wsb, _stream_ptr(stream), C.byref(o), infos)
    _check(code, allow_positive=True)
    return code, [_to_info(infos[i].status, infos[i], hists[i]) for i in range(n)]


class Server:
    """Request queue in front of continuously refilled batches:
    submit(), progress() -> completed ids, result(id), stats()."""

    def __init__(self, hbm_budget: int, max_active: int = 64, step_iters: int = 10, mmax: int = 30, stream=None,
                 launch_direct: bool = False, stall_window: int = 0, max_restarts: int = 0):
        cfg = ServerConfig(int(hbm_budget), int(max_active), int(step_iters), int(mmax), int(bool(launch_direct)),
                           int(stall_window), int(max_restarts))
        h = C.c_void_p()
        _check(lib().pfk_server_create(C.byref(cfg), _stream_ptr(stream), C.byref(h)))
        self._h = h
        self.max_active = max_active
        self._keep = {}
        self._maxit = {}

    def submit(self, A: Operator, B: Precond, method: str, b, x, rtol: float = 1e-8, maxit: int = 500) -> int:
        rid = C.c_longlong(-1)
        _check(lib().pfk_server_submit(self._h, A.handle, B.handle, METHODS[method], _dev_ptr(b, A.N, "b"),
                                       _dev_ptr(x, A.N, "x"), float(rtol), int(maxit), C.byref(rid)))
        self._keep[rid.value] = (A, B, b, x)
        self._maxit[rid.value] = maxit
        return rid.value

    def progress(self) -> list:
        cap = 4 * self.max_active + 16
        done = (C.c_longlong * cap)()
        n = C.c_int(0)
        _check(lib().pfk_server_progress(self._h, done, cap, C.byref(n)))
        return [done[i] for i in range(n.value)]

    def result(self, rid: int) -> SolveInfo:
        info, hist = _info_struct(self._maxit[rid] + 1)
        code = lib().pfk_server_result(self._h, int(rid), C.byref(info))
        _check(code, allow_positive=True)
        self._keep.pop(rid, None)
        return _to_info(code, info, hist)

    def stats(self) -> dict:
        st = ServerStatus()
        _check(lib().pfk_server_stats(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pfk_server_destroy(self._h)
            self._h = None
        self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
