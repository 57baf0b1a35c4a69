"""Python binding of the gfx950 t-SVT library (``libtsvd.so``).

Argument marshalling only: every step of t-SVT and of the two ADMM solvers
runs in the library's HIP kernels.  Tensors are torch tensors on the GPU
(``torch`` provides device memory and the current stream); the names and
arguments follow the C ABI in ``include/tsvd.h``:

    tsvt(X, tau)                          -> (Z, multirank)
    tsvd_complete(X_obs, mask, rho, tol)  -> (X, info)
    trpca(X, lam, mu, tol)                -> (L, S, info)

There is no CPU fallback: if the library is missing, importing the module
still works, but every call raises ``LibraryNotBuilt``.
"""

from __future__ import annotations

import ctypes
import os
import threading

__all__ = [
    "LibraryNotBuilt", "TsvdError", "Info", "library_path", "load_library", "tsvt",
    "tsvd_complete", "trpca", "Handle", "PREC_FP64", "PREC_FP32", "SHRINK_L1", "SHRINK_L112",
]

HERE = os.path.dirname(os.path.abspath(__file__))

PREC_FP64, PREC_FP32 = 0, 1
DTYPE_F64, DTYPE_F32 = 0, 1
SHRINK_L1, SHRINK_L112 = 0, 1

STATUS = {0: "TSVD_OK", -1: "TSVD_E_INVALID", -2: "TSVD_E_SHAPE", -3: "TSVD_E_NOMEM",
          -4: "TSVD_E_HIP", -5: "TSVD_E_NONFINITE", -6: "TSVD_E_UNSUPPORTED"}


class LibraryNotBuilt(RuntimeError):
    pass


class TsvdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Shape(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int64 * 4)]


class AdmmOpts(ctypes.Structure):
    _fields_ = [("growth", ctypes.c_double), ("rho_max", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_sweeps", ctypes.c_int32), ("reserved", ctypes.c_int32)]


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
                ("work_is_bytes", ctypes.c_int32), ("reserved", ctypes.c_int32)]


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
    "tsvd_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "tsvd_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(KernelStat), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int)]),
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
                                         work_is_bytes=bool(st.work_is_bytes))
        return out

    def close(self):
        if self._h:
            load_library().tsvd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_handles: dict[int, Handle] = {}


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


def _opts(growth, rho_max, max_iter, precision, max_sweeps):
    o = AdmmOpts()
    o.growth = float(growth or 0.0)
    o.rho_max = float(rho_max or 0.0)
    o.max_iter = int(max_iter or 0)
    o.precision = int(precision)
    o.max_sweeps = int(max_sweeps or 0)
    o.reserved = 0
    return o


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


def tsvd_complete(X_obs, mask, rho: float = 1e-2, tol: float = 1e-8, growth: float = 1.1,
                  rho_max: float = 1e3, max_iter: int = 300, precision: int = PREC_FP64,
                  max_sweeps: int = 0, handle: Handle | None = None):
    """TNN completion (include/tsvd.h, ``tsvd_complete``).  Returns (X, info)."""
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
    opts = _opts(growth, rho_max, max_iter, precision, max_sweeps)
    _check(load_library().tsvd_complete(handle.ptr, ctypes.c_void_p(X_obs.data_ptr()),
                                        ctypes.c_void_p(mask.data_ptr()), _shape(X_obs),
                                        _dtype_code(X_obs), float(rho), float(tol),
                                        ctypes.byref(opts), ctypes.c_void_p(out.data_ptr()),
                                        ctypes.byref(info)))
    return out, info


def trpca(X, lam: float, mu: float = 1e-3, tol: float = 1e-7, shrink: int = SHRINK_L1,
          growth: float = 1.2, mu_max: float = 1e10, max_iter: int = 500,
          precision: int = PREC_FP64, max_sweeps: int = 0, handle: Handle | None = None):
    """Tensor robust PCA (include/tsvd.h, ``trpca``).  Returns (L, S, info)."""
    import torch

    X = _prepare(X, "X")
    handle = handle or _handle_for(X)
    _bind_stream(handle, X)
    L = torch.empty_like(X)
    S = torch.empty_like(X)
    info = Info()
    opts = _opts(growth, mu_max, max_iter, precision, max_sweeps)
    _check(load_library().trpca(handle.ptr, ctypes.c_void_p(X.data_ptr()), _shape(X),
                                _dtype_code(X), float(lam), float(mu), float(tol), int(shrink),
                                ctypes.byref(opts), ctypes.c_void_p(L.data_ptr()),
                                ctypes.c_void_p(S.data_ptr()), ctypes.byref(info)))
    return L, S, info
