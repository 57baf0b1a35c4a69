"""Python binding of the gfx950 t-SVT library (``libtsvd.so``).

Argument marshalling only: every step of t-SVT and of the two ADMM solvers
runs in the library's HIP kernels.  Tensors are torch tensors on the GPU
(``torch`` provides device memory and the current stream); the names and
arguments follow the C ABI in ``include/tsvd.h``:

    tsvt(X, tau)                          -> (Z, multirank)
    tsvd_complete(X_obs, mask, rho, tol)  -> (X, info)
    trpca(X, lam, mu, tol)                -> (L, S, info)
    batch_run([problem, ...])             -> [(status, info), ...]
    submit(problem) -> ticket;  poll(ticket) -> None | (status, info)
    cancel(ticket)

``SolverState`` holds the checkpoint of a solve (``tsvd_state``): pass it as
``state=`` to ``tsvd_complete`` / ``trpca`` with ``save=True`` to keep the
final iterates, and with ``load=True`` to resume from them.

Problems for the batched and served forms are built with
``complete_problem`` / ``trpca_problem``, which allocate their outputs.

There is no CPU fallback: if the library is missing, importing the module
still works, but every call raises ``LibraryNotBuilt``.
"""

from __future__ import annotations

import atexit
import ctypes
import os
import threading
import weakref

__all__ = [
    "LibraryNotBuilt", "TsvdError", "Info", "library_path", "load_library", "tsvt",
    "tsvd_complete", "trpca", "Handle", "PREC_FP64", "PREC_FP32", "SHRINK_L1", "SHRINK_L112",
    "Problem", "complete_problem", "trpca_problem", "batch_run", "submit", "poll", "serve_stats",
    "tsvd_factors", "compress", "COMPRESS_TSVD", "COMPRESS_TUBAL", "SolverState", "cancel", "tsvt_noalloc",
    "close_all",
]

HERE = os.path.dirname(os.path.abspath(__file__))

PREC_FP64, PREC_FP32 = 0, 1
DTYPE_F64, DTYPE_F32 = 0, 1
SHRINK_L1, SHRINK_L112 = 0, 1
COMPRESS_TSVD, COMPRESS_TUBAL = 1, 2

STATUS = {0: "TSVD_OK", -1: "TSVD_E_INVALID", -2: "TSVD_E_SHAPE", -3: "TSVD_E_NOMEM",
          -4: "TSVD_E_HIP", -5: "TSVD_E_NONFINITE", -6: "TSVD_E_UNSUPPORTED", -7: "TSVD_E_BUSY",
          -8: "TSVD_E_CANCELLED", -9: "TSVD_E_TIMEOUT"}
E_BUSY, E_CANCELLED, E_TIMEOUT = -7, -8, -9
KIND_COMPLETE, KIND_TRPCA = 0, 1


class LibraryNotBuilt(RuntimeError):
    pass


class TsvdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Shape(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int64 * 4)]


class StateRecord(ctypes.Structure):
    _fields_ = [("z", ctypes.c_void_p), ("dual", ctypes.c_void_p), ("s", ctypes.c_void_p),
                ("v", ctypes.c_void_p), ("penalty", ctypes.c_double), ("dual_scale", ctypes.c_double),
                ("iter", ctypes.c_int32), ("load", ctypes.c_int32), ("save", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class AdmmOpts(ctypes.Structure):
    _fields_ = [("growth", ctypes.c_double), ("rho_max", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_sweeps", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("state", ctypes.POINTER(StateRecord))]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("sweeps_total", ctypes.c_int32), ("sweeps_last", ctypes.c_int32),
                ("primal", ctypes.c_double), ("change", ctypes.c_double),
                ("rho_final", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("work", ctypes.c_double),
                ("work_is_bytes", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("slice_sweeps", ctypes.c_double), ("pairs_visited", ctypes.c_double),
                ("rotations", ctypes.c_double), ("kept_rank", ctypes.c_double)]


class ProblemRecord(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dtype", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("shrink", ctypes.c_int32), ("shape", Shape), ("x", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("penalty", ctypes.c_double), ("lam", ctypes.c_double),
                ("tol", ctypes.c_double), ("opts", AdmmOpts), ("out", ctypes.c_void_p),
                ("out_s", ctypes.c_void_p), ("deadline_s", ctypes.c_double)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("finished", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("running", ctypes.c_int64), ("iterations", ctypes.c_int64),
                ("arena_bytes", ctypes.c_int64), ("arena_used", ctypes.c_int64),
                ("peak_running", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def library_path() -> str:
    return os.environ.get("TSVD_LIBRARY", os.path.join(HERE, "libtsvd.so"))


_lib = None
_lock = threading.Lock()

# C signatures, in the order of include/tsvd.h
_SIGNATURES = {
    "tsvd_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]),
    "tsvd_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "tsvd_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "tsvt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, Shape, ctypes.c_int, ctypes.c_double,
                            ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "tsvd_complete": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, Shape,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.POINTER(AdmmOpts), ctypes.c_void_p,
                                     ctypes.POINTER(Info)]),
    "trpca": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, Shape, ctypes.c_int, ctypes.c_double,
                             ctypes.c_double, ctypes.c_double, ctypes.c_int,
                             ctypes.POINTER(AdmmOpts), ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.POINTER(Info)]),
    "tsvt_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, Shape, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "tsvd_factors": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, Shape, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "tsvd_compress": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, Shape, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.POINTER(ctypes.c_double)]),
    "tsvd_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "tsvd_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(KernelStat), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int)]),
    "tsvd_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ProblemRecord), ctypes.c_int32,
                                      ctypes.POINTER(Info), ctypes.POINTER(ctypes.c_int32)]),
    "tsvd_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ProblemRecord),
                                   ctypes.POINTER(ctypes.c_uint64)]),
    "tsvd_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(Info)]),
    "tsvd_cancel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "tsvd_serve_stats_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServeStats)]),
    "tsvd_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "tsvd_last_error": (ctypes.c_char_p, []),
}


def load_library():
    """Load libtsvd.so (once) and set the C signatures."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        path = library_path()
        if not os.path.exists(path):
            raise LibraryNotBuilt(
                f"{path} not found: build it with `python -m paper_1407_1785_amd.build`")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def _check(status: int):
    if status != 0:
        msg = load_library().tsvd_last_error().decode(errors="replace")
        raise TsvdError(status, msg)


class Handle:
    """Owns a library handle (workspace, twiddles) on one device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.tsvd_create(int(device), int(hbm_budget_bytes), ctypes.byref(h)))
        self._h = h
        self.device = int(device)
        self._served = {}   # ticket -> Problem, kept alive until finished
        _all_handles.add(self)

    @property
    def ptr(self):
        return self._h

    def profile(self, enable: bool):
        """Start (clearing old statistics) or stop per-kernel event timing."""
        _check(load_library().tsvd_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """Per-kernel-family statistics: name -> dict(launches, total_ms,
        work, work_is_bytes)."""
        cap = 32
        buf = (KernelStat * cap)()
        cnt = ctypes.c_int()
        _check(load_library().tsvd_profile_read(self._h, buf, cap, ctypes.byref(cnt)))
        out = {}
        for k in range(min(cnt.value, cap)):
            st = buf[k]
            out[st.name.decode()] = dict(launches=st.launches, total_ms=st.total_ms, work=st.work,
                                         work_is_bytes=bool(st.work_is_bytes), slice_sweeps=st.slice_sweeps,
                                         pairs_visited=st.pairs_visited, rotations=st.rotations,
                                         kept_rank=st.kept_rank)
        return out

    def close(self):
        """Destroy the library handle: stops its serving worker (joining the
        thread) and frees its device memory.  Idempotent."""
        self._served = {}
        if self._h:
            load_library().tsvd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_handles: dict[int, Handle] = {}
_all_handles = weakref.WeakSet()


def close_all():
    """Close every open handle (the module's shared ones and those made by
    callers).  Registered with atexit, so the serving workers are joined and
    the device memory freed while the HIP runtime is still loaded, not from
    a finaliser at interpreter teardown."""
    for h in list(_all_handles):
        try:
            h.close()
        except Exception:
            pass
    _handles.clear()


atexit.register(close_all)


def handle_for(tensor) -> Handle:
    """The module's shared handle for the tensor's device."""
    return _handle_for(tensor)


def _handle_for(tensor) -> Handle:
    dev = tensor.device.index if tensor.device.index is not None else 0
    h = _handles.get(dev)
    if h is None:
        h = _handles[dev] = Handle(dev)
    return h


def _prepare(tensor, name):
    import torch

    if not isinstance(tensor, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not tensor.is_cuda:
        raise ValueError(f"{name} must be on a GPU")
    if tensor.dim() not in (3, 4):
        raise ValueError(f"{name} must have 3 or 4 modes")
    if not tensor.is_contiguous():
        tensor = tensor.contiguous()
    return tensor


def _dtype_code(tensor):
    import torch

    if tensor.dtype == torch.float64:
        return DTYPE_F64
    if tensor.dtype == torch.float32:
        return DTYPE_F32
    raise TypeError("tensors must be float64 or float32")


def _shape(tensor) -> Shape:
    s = Shape()
    s.ndim = tensor.dim()
    for k, v in enumerate(tensor.shape):
        s.n[k] = int(v)
    return s


def _bind_stream(handle: Handle, tensor):
    import torch

    stream = torch.cuda.current_stream(tensor.device)
    _check(load_library().tsvd_set_stream(handle.ptr, ctypes.c_void_p(stream.cuda_stream)))


def _opts(growth, rho_max, max_iter, precision, max_sweeps, state=None):
    o = AdmmOpts()
    o.growth = float(growth or 0.0)
    o.rho_max = float(rho_max or 0.0)
    o.max_iter = int(max_iter or 0)
    o.precision = int(precision)
    o.max_sweeps = int(max_sweeps or 0)
    o.pad = 0
    if state is not None:
        o.state = ctypes.pointer(state.record)
    return o


class SolverState:
    """Checkpoint of a completion (Z, Q) or RPCA (L, S, W) solve, with the
    Fourier-domain right singular vectors of the last prox (the Jacobi warm
    start; ``with_v=False`` leaves them out, and a resumed solve then starts
    its first SVDs cold).  Owns its device tensors (``z``, ``dual``, ``s``,
    ``v``) and the ``tsvd_state`` record; ``penalty``, ``dual_scale`` and
    ``iter`` mirror the record's fields."""

    def __init__(self, like, rpca: bool = False, with_v: bool = True):
        import torch

        like = _prepare(like, "like")
        self.z = torch.zeros_like(like)
        self.dual = torch.zeros_like(like)
        self.s = torch.zeros_like(like) if rpca else None
        n = min(like.shape[0], like.shape[1])
        self.v = (torch.zeros((_n_slices(like), n, n, 2), dtype=like.dtype, device=like.device)
                  if with_v else None)
        r = StateRecord()
        r.z, r.dual = self.z.data_ptr(), self.dual.data_ptr()
        r.s = self.s.data_ptr() if self.s is not None else None
        r.v = self.v.data_ptr() if self.v is not None else None
        r.penalty, r.dual_scale = 1.0, 1.0
        self.record = r

    def _arm(self, load: bool, save: bool):
        self.record.load = 1 if load else 0
        self.record.save = 1 if save else 0

    @property
    def penalty(self):
        return self.record.penalty

    @property
    def dual_scale(self):
        return self.record.dual_scale

    @property
    def iter(self):
        return self.record.iter


def _n_slices(tensor) -> int:
    if tensor.dim() == 3:
        return tensor.shape[2] // 2 + 1
    return tensor.shape[2] * (tensor.shape[3] // 2 + 1)


def tsvt(X, tau: float, precision: int = PREC_FP64, handle: Handle | None = None):
    """t-SVT of X with threshold tau (include/tsvd.h, ``tsvt``).

    Returns (Z, multirank) with Z a new tensor like X and multirank a list of
    the per-slice counts of singular values above tau."""
    import torch

    X = _prepare(X, "X")
    handle = handle or _handle_for(X)
    _bind_stream(handle, X)
    Z = torch.empty_like(X)
    h = _n_slices(X)
    ranks = (ctypes.c_int32 * h)()
    _check(load_library().tsvt(handle.ptr, ctypes.c_void_p(X.data_ptr()), _shape(X), _dtype_code(X),
                               float(tau), int(precision), ctypes.c_void_p(Z.data_ptr()), ranks))
    return Z, list(ranks)


def tsvt_noalloc(X, tau: float, precision: int = PREC_FP64, handle: Handle | None = None, Z=None):
    """t-SVT through the no-allocation entry point (include/tsvd.h,
    ``tsvt_noalloc``): the library allocates nothing; ``Z`` (optional) is the
    caller's output tensor.  Returns (Z, multirank)."""
    import torch

    X = _prepare(X, "X")
    handle = handle or _handle_for(X)
    _bind_stream(handle, X)
    if Z is None:
        Z = torch.empty_like(X)
    h = _n_slices(X)
    ranks = (ctypes.c_int32 * h)()
    _check(load_library().tsvt_noalloc(handle.ptr, ctypes.c_void_p(X.data_ptr()), _shape(X), _dtype_code(X),
                                       float(tau), int(precision), ctypes.c_void_p(Z.data_ptr()), ranks))
    return Z, list(ranks)


def tsvd_factors(M, precision: int = PREC_FP64, handle: Handle | None = None):
    """Real t-SVD factors of M (include/tsvd.h, ``tsvd_factors``).

    Returns (U, S, V): U of shape (n1, n0) + trailing, S (n0,) + trailing
    (the singular tubes S(i, i, :)), V (n2, n0) + trailing, n0 = min(n1, n2),
    new tensors like M."""
    import torch

    M = _prepare(M, "M")
    handle = handle or _handle_for(M)
    _bind_stream(handle, M)
    n1, n2 = M.shape[0], M.shape[1]
    n0 = min(n1, n2)
    trail = tuple(M.shape[2:])
    U = torch.empty((n1, n0) + trail, dtype=M.dtype, device=M.device)
    S = torch.empty((n0,) + trail, dtype=M.dtype, device=M.device)
    V = torch.empty((n2, n0) + trail, dtype=M.dtype, device=M.device)
    _check(load_library().tsvd_factors(handle.ptr, ctypes.c_void_p(M.data_ptr()), _shape(M), _dtype_code(M),
                                       int(precision), ctypes.c_void_p(U.data_ptr()),
                                       ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(V.data_ptr())))
    return U, S, V


def compress(M, method: int, k: int, precision: int = PREC_FP64, handle: Handle | None = None):
    """Compression of a third-order M by Method 1 (COMPRESS_TSVD, the k
    largest Fourier-domain singular values) or Method 2 (COMPRESS_TUBAL, the
    first k singular tubes) (include/tsvd.h, ``tsvd_compress``).
    Returns (M_k, ratio)."""
    import torch

    M = _prepare(M, "M")
    handle = handle or _handle_for(M)
    _bind_stream(handle, M)
    out = torch.empty_like(M)
    ratio = ctypes.c_double(0.0)
    _check(load_library().tsvd_compress(handle.ptr, ctypes.c_void_p(M.data_ptr()), _shape(M), _dtype_code(M),
                                        int(precision), int(method), int(k), ctypes.c_void_p(out.data_ptr()),
                                        ctypes.byref(ratio)))
    return out, ratio.value


def tsvd_complete(X_obs, mask, rho: float = 1e-2, tol: float = 1e-8, growth: float = 1.1,
                  rho_max: float = 1e3, max_iter: int = 300, precision: int = PREC_FP64,
                  max_sweeps: int = 0, handle: Handle | None = None, state: SolverState | None = None,
                  load: bool = False, save: bool = True):
    """TNN completion (include/tsvd.h, ``tsvd_complete``).  Returns (X, info).
    With ``state``: start from it if ``load``, write the final state into it
    if ``save``."""
    import torch

    X_obs = _prepare(X_obs, "X_obs")
    mask = _prepare(mask, "mask")
    if mask.dtype != torch.uint8:
        mask = mask.to(torch.uint8)
    if mask.shape != X_obs.shape or mask.device != X_obs.device:
        raise ValueError("mask must match X_obs in shape and device")
    handle = handle or _handle_for(X_obs)
    _bind_stream(handle, X_obs)
    out = torch.empty_like(X_obs)
    info = Info()
    if state is not None:
        state._arm(load, save)
    opts = _opts(growth, rho_max, max_iter, precision, max_sweeps, state)
    _check(load_library().tsvd_complete(handle.ptr, ctypes.c_void_p(X_obs.data_ptr()),
                                        ctypes.c_void_p(mask.data_ptr()), _shape(X_obs),
                                        _dtype_code(X_obs), float(rho), float(tol),
                                        ctypes.byref(opts), ctypes.c_void_p(out.data_ptr()),
                                        ctypes.byref(info)))
    return out, info


def trpca(X, lam: float, mu: float = 1e-3, tol: float = 1e-7, shrink: int = SHRINK_L1,
          growth: float = 1.2, mu_max: float = 1e10, max_iter: int = 500,
          precision: int = PREC_FP64, max_sweeps: int = 0, handle: Handle | None = None,
          state: SolverState | None = None, load: bool = False, save: bool = True):
    """Tensor robust PCA (include/tsvd.h, ``trpca``).  Returns (L, S, info).
    ``state`` as for ``tsvd_complete``."""
    import torch

    X = _prepare(X, "X")
    handle = handle or _handle_for(X)
    _bind_stream(handle, X)
    L = torch.empty_like(X)
    S = torch.empty_like(X)
    info = Info()
    if state is not None:
        state._arm(load, save)
    opts = _opts(growth, mu_max, max_iter, precision, max_sweeps, state)
    _check(load_library().trpca(handle.ptr, ctypes.c_void_p(X.data_ptr()), _shape(X),
                                _dtype_code(X), float(lam), float(mu), float(tol), int(shrink),
                                ctypes.byref(opts), ctypes.c_void_p(L.data_ptr()),
                                ctypes.c_void_p(S.data_ptr()), ctypes.byref(info)))
    return L, S, info


class Problem:
    """One completion (Sec. 4) or tensor-RPCA (Sec. 5) problem for the
    batched and served forms; owns its output tensors (``out`` = X or L,
    ``out_s`` = S) and keeps its inputs alive."""

    def __init__(self, kind, x, mask=None, penalty=1e-2, lam=0.0, tol=1e-8, shrink=SHRINK_L1,
                 growth=0.0, rho_max=0.0, max_iter=0, precision=None, max_sweeps=0, deadline_s=0.0):
        import torch

        self.kind = int(kind)
        self.x = _prepare(x, "x")
        self.mask = None
        if self.kind == KIND_COMPLETE:
            m = _prepare(mask, "mask")
            if m.dtype != torch.uint8:
                m = m.to(torch.uint8)
            if m.shape != self.x.shape or m.device != self.x.device:
                raise ValueError("mask must match x in shape and device")
            self.mask = m
        self.out = torch.empty_like(self.x)
        self.out_s = torch.empty_like(self.x) if self.kind == KIND_TRPCA else None
        dt = _dtype_code(self.x)
        if precision is None:
            precision = PREC_FP32 if dt == DTYPE_F32 else PREC_FP64
        rec = ProblemRecord()
        rec.kind = self.kind
        rec.dtype = dt
        rec.precision = int(precision)
        rec.shrink = int(shrink)
        rec.shape = _shape(self.x)
        rec.x = self.x.data_ptr()
        rec.mask = self.mask.data_ptr() if self.mask is not None else None
        rec.penalty = float(penalty)
        rec.lam = float(lam)
        rec.tol = float(tol)
        rec.opts = _opts(growth, rho_max, max_iter, precision, max_sweeps)
        rec.out = self.out.data_ptr()
        rec.out_s = self.out_s.data_ptr() if self.out_s is not None else None
        rec.deadline_s = float(deadline_s)
        self.record = rec

    @property
    def device(self):
        return self.x.device


def complete_problem(X_obs, mask, rho=1e-2, tol=1e-8, growth=1.1, rho_max=1e3, max_iter=300,
                     precision=None, max_sweeps=0, deadline_s=0.0) -> Problem:
    return Problem(KIND_COMPLETE, X_obs, mask, rho, 0.0, tol, SHRINK_L1, growth, rho_max, max_iter,
                   precision, max_sweeps, deadline_s)


def trpca_problem(X, lam, mu=1e-3, tol=1e-7, shrink=SHRINK_L1, growth=1.2, mu_max=1e10, max_iter=500,
                  precision=None, max_sweeps=0, deadline_s=0.0) -> Problem:
    return Problem(KIND_TRPCA, X, None, mu, lam, tol, shrink, growth, mu_max, max_iter, precision,
                   max_sweeps, deadline_s)


def _sync_inputs(problems):
    import torch

    for dev in {p.device for p in problems}:
        torch.cuda.current_stream(dev).synchronize()


def batch_run(problems, handle: Handle | None = None):
    """Solve the problems together (include/tsvd.h, ``tsvd_batch_run``).
    Returns [(status, Info)] in order; outputs are in each problem's
    ``out`` / ``out_s``."""
    problems = list(problems)
    if not problems:
        return []
    handle = handle or _handle_for(problems[0].x)
    _sync_inputs(problems)
    n = len(problems)
    recs = (ProblemRecord * n)(*[p.record for p in problems])
    infos = (Info * n)()
    stats = (ctypes.c_int32 * n)()
    _check(load_library().tsvd_batch_run(handle.ptr, recs, n, infos, stats))
    return [(int(stats[i]), infos[i]) for i in range(n)]


def submit(problem: Problem, handle: Handle | None = None) -> int:
    """Queue a problem on the handle's serving worker (``tsvd_submit``)."""
    handle = handle or _handle_for(problem.x)
    _sync_inputs([problem])
    ticket = ctypes.c_uint64()
    _check(load_library().tsvd_submit(handle.ptr, ctypes.byref(problem.record), ctypes.byref(ticket)))
    handle._served[ticket.value] = problem
    return ticket.value


def poll(ticket: int, handle: Handle | None = None, device: int = 0):
    """None while the ticket runs; else (status, Info) (``tsvd_poll``)."""
    handle = handle or _handles.get(device)
    if handle is None:
        raise TsvdError(-1, "no handle")
    info = Info()
    st = load_library().tsvd_poll(handle.ptr, ctypes.c_uint64(int(ticket)), ctypes.byref(info))
    if st == E_BUSY:
        return None
    if st == -1:
        _check(st)
    handle._served.pop(int(ticket), None)
    return st, info


def cancel(ticket: int, handle: Handle | None = None, device: int = 0):
    """Cancel a queued or running request (``tsvd_cancel``); poll() then
    reports E_CANCELLED unless it had already finished."""
    handle = handle or _handles.get(device)
    if handle is None:
        raise TsvdError(-1, "no handle")
    _check(load_library().tsvd_cancel(handle.ptr, ctypes.c_uint64(int(ticket))))


def serve_stats(handle: Handle | None = None, device: int = 0) -> dict:
    handle = handle or _handles.get(device)
    if handle is None:
        return ServeStats().as_dict()
    out = ServeStats()
    _check(load_library().tsvd_serve_stats_read(handle.ptr, ctypes.byref(out)))
    return out.as_dict()
