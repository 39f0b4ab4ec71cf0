"""Python binding of libnbody.so.

Argument marshalling only: tensors are checked (float32, contiguous, on the
current HIP device, right shape), their device pointers and torch's current
stream are handed to the C ABI (include/nbody.h), and a failing status is
raised as :class:`NBodyError`.  Every arithmetic step runs in the HIP
kernels of the library; there is no CPU fallback, and a missing library
raises at first use.
"""

from __future__ import annotations

import contextlib
import ctypes
import os

import numpy as np
import torch

from . import build as _build

FORWARD, BACKWARD, BATCHED = 0, 1, 2
ABI_VERSION = 4

_STATUS = {
    0: "NBODY_OK",
    1: "NBODY_ERROR_INVALID_ARGUMENT",
    2: "NBODY_ERROR_UNSUPPORTED_DEVICE",
    3: "NBODY_ERROR_OUT_OF_MEMORY",
    4: "NBODY_ERROR_LAUNCH_FAILED",
    5: "NBODY_ERROR_INTERNAL",
}


class NBodyError(RuntimeError):
    """A libnbody call returned a non-zero status."""

    def __init__(self, status: int, detail: str):
        self.status = int(status)
        self.name = _STATUS.get(self.status, f"status {status}")
        super().__init__(f"{self.name}: {detail}")


_LIB = None
_vp, _i64, _f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_float


def lib() -> ctypes.CDLL:
    """The loaded libnbody.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        path = os.environ.get("NBODY_LIBRARY", _build.LIBRARY)
        if not os.path.exists(path):
            raise NBodyError(5, f"{path} is not built; run `python -m paper_0904_3659_amd.build`")
        L = ctypes.CDLL(path)
        L.nbody_abi_version.restype = ctypes.c_int
        L.nbody_status_string.restype = ctypes.c_char_p
        L.nbody_status_string.argtypes = [ctypes.c_int]
        L.nbody_last_error.restype = ctypes.c_char_p
        L.nbody_forces.argtypes = [_vp, _vp, _i64, _f32, _vp, _vp, _vp]
        L.nbody_forces_ex.argtypes = [_vp, _vp, _i64, _f32, _vp, _vp, ctypes.c_uint32, _vp]
        L.nbody_forces_noalloc.argtypes = [_vp, _vp, _i64, _f32, _vp, _vp, _vp]
        L.nbody_forces_backward.argtypes = [_vp, _vp, _i64, _f32, _vp, _vp, _vp, _vp, _vp]
        L.nbody_forces_batched.argtypes = [ctypes.POINTER(_i64), _i64, _vp, _vp, _f32, _vp, _vp, _vp]
        L.nbody_axpy.argtypes = [_vp, _vp, _i64, _f32, _vp]
        L.nbody_kick_drift.argtypes = [_vp, _vp, _vp, _i64, _f32, _f32, _vp]
        L.nbody_leapfrog.argtypes = [_vp, _vp, _vp, _vp, _i64, _f32, _f32, _i64, _vp, _vp]
        L.nbody_leapfrog_adjoint.argtypes = [_vp, _vp, _i64, _f32, _f32, _i64, ctypes.c_uint32,
                                             _vp, _vp, _vp, _vp]
        L.nbody_variant_count.argtypes = [ctypes.c_int]
        L.nbody_variant_count.restype = ctypes.c_int
        L.nbody_variant_name.argtypes = [ctypes.c_int, ctypes.c_int]
        L.nbody_variant_name.restype = ctypes.c_char_p
        L.nbody_set_variant.argtypes = [ctypes.c_int, ctypes.c_int]
        L.nbody_autotune.argtypes = [ctypes.c_int, ctypes.POINTER(_i64), _i64, _vp]
        L.nbody_autotune_batched.argtypes = [ctypes.POINTER(_i64), _i64, _vp, _vp, _f32, _vp]
        L.nbody_profile_enable.argtypes = [ctypes.c_int]
        L.nbody_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_double)]
        L.nbody_variant_plan.argtypes = [ctypes.c_int, ctypes.c_int, _i64, ctypes.c_int,
                                         ctypes.c_int, _i64, ctypes.POINTER(ctypes.c_int)]
        L.nbody_variant_plan.restype = _i64
        L.nbody_selected_variant.argtypes = [ctypes.c_int, _i64]
        L.nbody_selected_variant.restype = ctypes.c_int
        for f in ("nbody_forces", "nbody_forces_ex", "nbody_forces_noalloc",
                  "nbody_forces_backward", "nbody_forces_batched",
                  "nbody_axpy",
                  "nbody_kick_drift", "nbody_leapfrog", "nbody_leapfrog_adjoint",
                  "nbody_set_variant", "nbody_autotune", "nbody_autotune_batched",
                  "nbody_release_workspace",
                  "nbody_profile_enable", "nbody_profile_read"):
            getattr(L, f).restype = ctypes.c_int
        if L.nbody_abi_version() != ABI_VERSION:
            raise NBodyError(5, f"ABI version {L.nbody_abi_version()} != {ABI_VERSION}")
        _LIB = L
    return _LIB


def _check(status: int) -> None:
    if status != 0:
        raise NBodyError(status, lib().nbody_last_error().decode(errors="replace"))


def _ptr(t: torch.Tensor | None):
    # an int: ctypes passes it as the void* the argtypes declare
    return None if t is None else t.data_ptr()


_ONE_DEVICE = None


def _on(device: torch.device):
    """Make ``device`` current for the call (a no-op when it already is)."""
    global _ONE_DEVICE
    if _ONE_DEVICE is None:
        _ONE_DEVICE = torch.cuda.device_count() == 1
    if _ONE_DEVICE or device.index is None or device.index == torch.cuda.current_device():
        return _NULL
    return torch.cuda.device(device)


_NULL = contextlib.nullcontext()


# torch's current-stream handle without building a Stream object (the
# public accessor below costs ~1.5 us per call, a sixth of a small call)
_RAW_STREAM = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream(device: torch.device):
    if _RAW_STREAM is not None and device.index is not None:
        return _RAW_STREAM(device.index)
    return torch.cuda.current_stream(device).cuda_stream


_F32 = torch.float32


def _want(t: torch.Tensor, name: str, shape, device=None) -> None:
    # the common case in one expression (a small call spends more time here
    # than in the library); anything else goes through the checks below,
    # which name what is wrong
    if (type(t) is torch.Tensor and t.is_cuda and t.dtype is _F32 and t.is_contiguous()
            and t.shape == shape
            and (device is None or _ONE_DEVICE is True or t.get_device() == device.index)):
        return
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a HIP device, got {t.device}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.shape != shape:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _eps2(eps2) -> float:
    e = float(eps2)
    if not (e >= 0.0) or e == float("inf"):
        raise ValueError(f"eps2 must be finite and >= 0, got {eps2}")
    return e


# ---------------------------------------------------------------- evaluation

F64_SUM = 1  # NBODY_FORCES_F64_SUM


def forces(x: torch.Tensor, m: torch.Tensor, eps2: float, *, out=None, potential: bool = True,
           f64_sum: bool = False):
    """Eq. (gravity): (a [n,3], p [n]) in the paper's sign, j != i.

    ``out`` may supply preallocated (a, p).  With ``potential=False`` the
    potential is not stored and ``p`` is returned as None.  ``f64_sum`` keeps
    each row's running sum (over j-tiles and j-splits) in float64.
    """
    sh = x.shape
    n = sh[0] if len(sh) == 2 else -1
    _want(x, "x", (n, 3))
    dev = x.device
    _want(m, "m", (n,), dev)
    if out is None:
        a = torch.empty((n, 3), dtype=torch.float32, device=dev)
        p = torch.empty((n,), dtype=torch.float32, device=dev) if potential else None
    else:
        a, p = out
        _want(a, "a", (n, 3), dev)
        if p is not None:
            _want(p, "p", (n,), dev)
    with _on(dev):
        if f64_sum:
            _check(lib().nbody_forces_ex(_ptr(x), _ptr(m), n, _eps2(eps2), _ptr(a), _ptr(p),
                                         F64_SUM, _stream(dev)))
        else:
            _check(lib().nbody_forces(_ptr(x), _ptr(m), n, _eps2(eps2), _ptr(a), _ptr(p),
                                      _stream(dev)))
    return a, p


class BoundForces:
    """:func:`forces` on fixed tensors, for latency-bound loops: the tensors
    are checked once, here, and each call passes the stored device pointers
    and torch's current stream straight to ``nbody_forces`` (about 2 µs less
    host time per call than :func:`forces` at small n).  The object holds
    the tensors; resizing or replacing their storage afterwards (``set_``,
    ``resize_``, assigning ``.data``) is not checked and must not happen
    while it is in use.  Writing new values into them is fine.

        call = BoundForces(x, m, eps2, a, p)
        call()            # a, p = forces of the current x, m
    """

    __slots__ = ("_fn", "_args", "_dev", "_keep")

    def __init__(self, x: torch.Tensor, m: torch.Tensor, eps2: float, a: torch.Tensor,
                 p: torch.Tensor | None = None):
        sh = x.shape
        n = sh[0] if len(sh) == 2 else -1
        _want(x, "x", (n, 3))
        dev = x.device
        _want(m, "m", (n,), dev)
        _want(a, "a", (n, 3), dev)
        if p is not None:
            _want(p, "p", (n,), dev)
        self._fn = lib().nbody_forces
        self._args = (_ptr(x), _ptr(m), n, _eps2(eps2), _ptr(a), _ptr(p))
        self._dev = dev
        self._keep = (x, m, a, p)

    def __call__(self) -> None:
        dev = self._dev
        with _on(dev):
            status = self._fn(*self._args, _stream(dev))
        if status:
            _check(status)


def forces_noalloc(x: torch.Tensor, m: torch.Tensor, eps2: float, a: torch.Tensor,
                   p: torch.Tensor | None = None):
    """:func:`forces` through ``nbody_forces_noalloc``: the library
    allocates nothing for the call (its workspace is a fixed 64 MiB device
    region per device).  The caller supplies the outputs ``a`` [n,3] and,
    optionally, ``p`` [n]; calls that overlap in time on one device race."""
    sh = x.shape
    n = sh[0] if len(sh) == 2 else -1
    _want(x, "x", (n, 3))
    dev = x.device
    _want(m, "m", (n,), dev)
    _want(a, "a", (n, 3), dev)
    if p is not None:
        _want(p, "p", (n,), dev)
    with _on(dev):
        _check(lib().nbody_forces_noalloc(_ptr(x), _ptr(m), n, _eps2(eps2), _ptr(a), _ptr(p),
                                          _stream(dev)))
    return a, p


def forces_backward(x, m, eps2, grad_a=None, grad_p=None, *, need_grad_m: bool = True, out=None):
    """Vector-Jacobian product of :func:`forces`: (dL/dx [n,3], dL/dm [n] or None)."""
    sh = x.shape
    n = sh[0] if len(sh) == 2 else -1
    _want(x, "x", (n, 3))
    dev = x.device
    _want(m, "m", (n,), dev)
    if grad_a is not None:
        _want(grad_a, "grad_a", (n, 3), dev)
    if grad_p is not None:
        _want(grad_p, "grad_p", (n,), dev)
    if out is None:
        gx = torch.empty((n, 3), dtype=torch.float32, device=dev)
        gm = torch.empty((n,), dtype=torch.float32, device=dev) if need_grad_m else None
    else:
        gx, gm = out
        _want(gx, "grad_x", (n, 3), dev)
        if gm is not None:
            _want(gm, "grad_m", (n,), dev)
    with _on(dev):
        _check(lib().nbody_forces_backward(_ptr(x), _ptr(m), n, _eps2(eps2), _ptr(grad_a),
                                           _ptr(grad_p), _ptr(gx), _ptr(gm), _stream(dev)))
    return gx, gm


def _offsets_array(offsets) -> np.ndarray:
    if isinstance(offsets, torch.Tensor):
        if offsets.device.type != "cpu":
            raise ValueError("offsets must be a host (CPU) array")
        offsets = offsets.numpy()
    o = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if o.ndim != 1 or o.size < 1:
        raise ValueError("offsets must be a 1-D array of num_systems + 1 values")
    return o


def forces_batched(x: torch.Tensor, m: torch.Tensor, offsets, eps2: float, *, out=None):
    """Eq. (gravity) on independent systems [offsets[s], offsets[s+1]).

    ``offsets`` is a host array (numpy, list or CPU tensor) of int64.
    """
    o = _offsets_array(offsets)
    sh = x.shape
    n = sh[0] if len(sh) == 2 else -1
    _want(x, "x", (n, 3))
    dev = x.device
    _want(m, "m", (n,), dev)
    if int(o[-1]) != n:
        raise ValueError(f"offsets[-1] = {int(o[-1])} but x holds {n} particles")
    if out is None:
        a = torch.empty((n, 3), dtype=torch.float32, device=dev)
        p = torch.empty((n,), dtype=torch.float32, device=dev)
    else:
        a, p = out
        _want(a, "a", (n, 3), dev)
        _want(p, "p", (n,), dev)
    with _on(dev):
        _check(lib().nbody_forces_batched(o.ctypes.data_as(ctypes.POINTER(_i64)), o.size - 1,
                                          _ptr(x), _ptr(m), _eps2(eps2), _ptr(a), _ptr(p),
                                          _stream(dev)))
    return a, p


def axpy_(y: torch.Tensor, xv: torch.Tensor, alpha: float) -> torch.Tensor:
    """In place y += alpha * xv on the device (leap-frog kick and drift)."""
    _want(y, "y", tuple(y.shape))
    _want(xv, "x", tuple(y.shape), y.device)
    with _on(y.device):
        _check(lib().nbody_axpy(_ptr(y), _ptr(xv), y.numel(), float(alpha), _stream(y.device)))
    return y


def kick_drift_(x: torch.Tensor, v: torch.Tensor, a: torch.Tensor, kick: float, dt: float):
    """In place v += kick * a, then x += dt * v (one leap-frog kick + drift)."""
    sh = x.shape
    n = sh[0] if len(sh) == 2 else -1
    _want(x, "x", (n, 3))
    _want(v, "v", (n, 3), x.device)
    _want(a, "a", (n, 3), x.device)
    with _on(x.device):
        _check(lib().nbody_kick_drift(_ptr(x), _ptr(v), _ptr(a), n, float(kick), float(dt),
                                      _stream(x.device)))
    return x, v


LEAPFROG_FINAL = 1    # NBODY_LEAPFROG_FINAL
LEAPFROG_INITIAL = 2  # NBODY_LEAPFROG_INITIAL


def _steps(steps) -> int:
    s = int(steps)
    if s < 0:
        raise ValueError(f"steps must be >= 0, got {steps}")
    return s


def leapfrog_(x, v, a, m, eps2: float, dt: float, steps: int, *, x_hist=None):
    """In place: ``steps`` kick-drift-kick steps of (x, v) on the device
    (nbody_leapfrog), with a = a(x) in the paper's sign on entry and exit.
    ``x_hist`` ([steps, n, 3]) receives the positions after each step."""
    n = int(m.shape[0]) if m.dim() == 1 else -1
    steps = _steps(steps)
    _want(m, "m", (n,))
    for name, t in (("x", x), ("v", v), ("a", a)):
        _want(t, name, (n, 3), m.device)
    if x_hist is not None:
        _want(x_hist, "x_hist", (steps, n, 3), m.device)
    with _on(m.device):
        _check(lib().nbody_leapfrog(_ptr(x), _ptr(v), _ptr(a), _ptr(m), n, _eps2(eps2), float(dt),
                                    steps, _ptr(x_hist), _stream(m.device)))
    return x, v, a


def leapfrog_adjoint_(pos, m, eps2: float, dt: float, lx, lv, lm, *, flags: int = 0):
    """In place: the reverse sweep over the ``pos.shape[0] - 1`` steps whose
    positions ``pos`` holds (nbody_leapfrog_adjoint): (lx, lv) from the
    segment's end to its start, dL/dm added to lm.  ``flags``: LEAPFROG_FINAL
    and/or LEAPFROG_INITIAL."""
    n = int(m.shape[0]) if m.dim() == 1 else -1
    steps = int(pos.shape[0]) - 1 if pos.dim() == 3 else -1
    if steps < 0:
        raise ValueError(f"pos must have shape [steps + 1, n, 3], got {tuple(pos.shape)}")
    _want(m, "m", (n,))
    _want(pos, "pos", (steps + 1, n, 3), m.device)
    _want(lx, "lx", (n, 3), m.device)
    _want(lv, "lv", (n, 3), m.device)
    _want(lm, "lm", (n,), m.device)
    with _on(m.device):
        _check(lib().nbody_leapfrog_adjoint(_ptr(pos), _ptr(m), n, _eps2(eps2), float(dt), steps,
                                            int(flags), _ptr(lx), _ptr(lv), _ptr(lm),
                                            _stream(m.device)))
    return lx, lv, lm


# ---------------------------------------------------------------- autograd

class NBodyForces(torch.autograd.Function):
    """(a, p) = forces(x, m, eps2) with the library's adjoint as backward."""

    @staticmethod
    def forward(ctx, x, m, eps2):
        a, p = forces(x, m, eps2)
        ctx.save_for_backward(x, m)
        ctx.eps2 = float(eps2)
        ctx.set_materialize_grads(False)
        return a, p

    @staticmethod
    def backward(ctx, grad_a, grad_p):
        x, m = ctx.saved_tensors
        if grad_a is None and grad_p is None:
            return None, None, None
        grad_a = None if grad_a is None else grad_a.contiguous()
        grad_p = None if grad_p is None else grad_p.contiguous()
        gx, gm = forces_backward(x, m, ctx.eps2, grad_a, grad_p,
                                 need_grad_m=ctx.needs_input_grad[1])
        return gx, gm, None


# ---------------------------------------------------------------- variants

def variant_count(kind: int) -> int:
    return int(lib().nbody_variant_count(kind))


def variant_names(kind: int) -> list[str]:
    return [lib().nbody_variant_name(kind, k).decode() for k in range(variant_count(kind))]


def set_variant(kind: int, index: int) -> None:
    """Force a kernel variant for ``kind`` (-1 restores automatic choice)."""
    _check(lib().nbody_set_variant(kind, index))


def selected_variant(kind: int, n: int) -> int:
    return int(lib().nbody_selected_variant(kind, n))


def autotune(kind: int, sizes, device=None) -> None:
    """Time every variant of ``kind`` at each size and keep the fastest."""
    s = np.ascontiguousarray(np.asarray(sizes, dtype=np.int64))
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    with _on(dev):
        _check(lib().nbody_autotune(kind, s.ctypes.data_as(ctypes.POINTER(_i64)), s.size, _stream(dev)))


def autotune_batched(x: torch.Tensor, m: torch.Tensor, offsets, eps2: float) -> int:
    """Time every batched variant on this ensemble, keep the fastest for its
    mean system size, and return that variant's index."""
    o = _offsets_array(offsets)
    sh = x.shape
    n = sh[0] if len(sh) == 2 else -1
    _want(x, "x", (n, 3))
    _want(m, "m", (n,), x.device)
    if int(o[-1]) != n:
        raise ValueError(f"offsets[-1] = {int(o[-1])} but x holds {n} particles")
    with _on(x.device):
        _check(lib().nbody_autotune_batched(o.ctypes.data_as(ctypes.POINTER(_i64)), o.size - 1,
                                            _ptr(x), _ptr(m), _eps2(eps2), _stream(x.device)))
    systems = o.size - 1
    return selected_variant(BATCHED, n // systems if systems > 0 else 0)


def variant_plan(kind: int, index: int, n: int, num_cu: int, blocks_per_cu: int,
                 free_bytes: int) -> tuple[int, bool]:
    """(workspace bytes, timed by the variant timer) of a variant at size n,
    from host arithmetic only (``nbody_variant_plan``)."""
    timed = ctypes.c_int(0)
    b = lib().nbody_variant_plan(kind, index, n, num_cu, blocks_per_cu, free_bytes,
                                 ctypes.byref(timed))
    if b < 0:
        raise NBodyError(1, lib().nbody_last_error().decode())
    return int(b), bool(timed.value)


def release_workspace() -> None:
    _check(lib().nbody_release_workspace())


def profile_enable(on: bool = True) -> None:
    """Record HIP events around the library's own kernels (this thread)."""
    _check(lib().nbody_profile_enable(1 if on else 0))


def profile_read(launches: bool = False):
    """(mean summed pair-kernel ms, mean whole-call ms, calls) since the last
    read; with ``launches`` also the mean number of pair kernels per call."""
    a, b, c, d = ctypes.c_double(), ctypes.c_double(), ctypes.c_int(), ctypes.c_double()
    _check(lib().nbody_profile_read(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                    ctypes.byref(d)))
    return (a.value, b.value, c.value, d.value) if launches else (a.value, b.value, c.value)


def __getattr__(name):
    # ``leapfrog`` is re-exported lazily: leapfrog.py imports this module, so
    # either may be imported first.
    if name == "leapfrog":
        from .leapfrog import leapfrog
        return leapfrog
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")
