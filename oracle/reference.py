"""FP64 reference evaluators (ctypes front end of ``libnbody_oracle.so``).

TEST INFRASTRUCTURE ONLY.  Every function takes numpy arrays (float32 inputs
are upcast exactly to float64) and returns float64 arrays.  Nothing here
touches the GPU or the HIP library.

Functions and the passages they follow:
  forces            Eq. (gravity), Sec. I: a_i and p_i with j != i.
  forces_rows       the same, for a subset of rows i.
  forces_batched    Eq. (gravity) on independent systems (offset ranges).
  forces_vjp        chain rule of Eq. (gravity) for L = sum w.a + v p.
  leapfrog          Eqs. (1)-(3) and the seven-step algorithm of Sec. III,
                    with the physical acceleration g = -a.
  leapfrog_vjp      reverse-mode sweep of the same integrator for a loss on
                    the final positions.
  energy            kinetic plus pair potential energy (for drift checks).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None
_dptr = ctypes.POINTER(ctypes.c_double)
_i64ptr = ctypes.POINTER(ctypes.c_int64)


def configure(L: ctypes.CDLL) -> ctypes.CDLL:
    """Declare the C signatures on a loaded copy of the reference library."""
    i64, dbl = ctypes.c_int64, ctypes.c_double
    L.oracle_num_threads.restype = ctypes.c_int
    L.oracle_set_num_threads.argtypes = [ctypes.c_int]
    L.oracle_set_num_threads.restype = None
    L.oracle_forces_rows.argtypes = [_dptr, _dptr, i64, dbl, _i64ptr, i64, _dptr, _dptr]
    L.oracle_forces.argtypes = [_dptr, _dptr, i64, dbl, _dptr, _dptr]
    L.oracle_forces_batched.argtypes = [_i64ptr, i64, _dptr, _dptr, dbl, _dptr, _dptr]
    L.oracle_forces_vjp.argtypes = [_dptr, _dptr, i64, dbl, _dptr, _dptr, _dptr, _dptr]
    L.oracle_leapfrog.argtypes = [_dptr, _dptr, _dptr, i64, dbl, dbl, i64, _dptr, _dptr]
    for f in ("oracle_forces_rows", "oracle_forces", "oracle_forces_batched",
              "oracle_forces_vjp", "oracle_leapfrog"):
        getattr(L, f).restype = None
    return L


def lib() -> ctypes.CDLL:
    """Load the reference library, compiling it first if it is not built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIBRARY):
            _build.build()
        _LIB = configure(ctypes.CDLL(_build.LIBRARY))
    return _LIB


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(threads: int) -> None:
    """OpenMP threads for later calls; the results do not depend on it."""
    lib().oracle_set_num_threads(int(threads))


def _d(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _p(a):
    return None if a is None else a.ctypes.data_as(_dptr)


def forces(x, m, eps2: float):
    """(a [n,3], p [n]) of Eq. (gravity) in FP64, paper sign, j != i."""
    x = _d(x, (-1, 3))
    n = x.shape[0]
    m = _d(m, (n,))
    a = np.zeros((n, 3))
    p = np.zeros(n)
    lib().oracle_forces(_p(x), _p(m), n, float(eps2), _p(a), _p(p))
    return a, p


def forces_rows(x, m, eps2: float, rows):
    """(a [r,3], p [r]) for the listed rows only (same sums as ``forces``)."""
    x = _d(x, (-1, 3))
    n = x.shape[0]
    m = _d(m, (n,))
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    if rows.size and (rows.min() < 0 or rows.max() >= n):
        raise IndexError("row index out of range")
    a = np.zeros((rows.size, 3))
    p = np.zeros(rows.size)
    lib().oracle_forces_rows(_p(x), _p(m), n, float(eps2),
                             rows.ctypes.data_as(_i64ptr), rows.size, _p(a), _p(p))
    return a, p


def forces_batched(offsets, x, m, eps2: float):
    """Eq. (gravity) per system [offsets[s], offsets[s+1])."""
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    x = _d(x, (-1, 3))
    n = x.shape[0]
    m = _d(m, (n,))
    if offsets[0] != 0 or offsets[-1] != n or np.any(np.diff(offsets) < 0):
        raise ValueError("offsets must start at 0, be non-decreasing and end at n")
    a = np.zeros((n, 3))
    p = np.zeros(n)
    lib().oracle_forces_batched(offsets.ctypes.data_as(_i64ptr), offsets.size - 1,
                                _p(x), _p(m), float(eps2), _p(a), _p(p))
    return a, p


def forces_vjp(x, m, eps2: float, w=None, v=None):
    """(dL/dx [n,3], dL/dm [n]) for L = sum_i w_i . a_i + v_i p_i."""
    x = _d(x, (-1, 3))
    n = x.shape[0]
    m = _d(m, (n,))
    w = None if w is None else _d(w, (n, 3))
    v = None if v is None else _d(v, (n,))
    gx = np.zeros((n, 3))
    gm = np.zeros(n)
    lib().oracle_forces_vjp(_p(x), _p(m), n, float(eps2), _p(w), _p(v), _p(gx), _p(gm))
    return gx, gm


def loss(x, m, eps2: float, w=None, v=None) -> float:
    """L = sum_i w_i . a_i + v_i p_i, evaluated with ``forces`` in FP64."""
    a, p = forces(x, m, eps2)
    out = 0.0
    if w is not None:
        out += float(np.sum(_d(w, a.shape) * a))
    if v is not None:
        out += float(np.sum(_d(v, p.shape) * p))
    return out


def leapfrog(x0, v0, m, eps2: float, dt: float, steps: int, trajectory: bool = False):
    """Kick-drift-kick leap-frog, Eqs. (1)-(3), with g = -a.

    Returns (x_T, v_T) or, with ``trajectory``, (x_T, v_T, traj) where
    traj[t] holds the positions after t steps (traj[0] = x0).
    """
    x = _d(x0, (-1, 3)).copy()
    n = x.shape[0]
    v = _d(v0, (n, 3)).copy()
    m = _d(m, (n,))
    g = np.zeros((n, 3))
    traj = np.zeros((steps + 1, n, 3)) if trajectory else None
    lib().oracle_leapfrog(_p(x), _p(v), _p(m), n, float(eps2), float(dt), int(steps),
                          _p(traj), _p(g))
    return (x, v, traj) if trajectory else (x, v)


def leapfrog_vjp(x0, v0, m, eps2: float, dt: float, steps: int, u, uv=None):
    """Gradients of L = sum_i u_i . x_i(T) + uv_i . v_i(T) with respect to
    x0, v0 and m (``uv`` None means the loss ignores the final velocities).

    Reverse sweep of one step (x, v) -> (x', v'), with g = -a:
        v_half = v + (dt/2) g(x);  x' = x + dt v_half;  v' = v_half + (dt/2) g(x')
    Given the adjoints (lx', lv') of the step's outputs:
        lx' += (dt/2) J_g(x')^T lv'     (and lm += (dt/2) J_g,m(x')^T lv')
        lvh  = lv' + dt lx'
        lx   = lx' + (dt/2) J_g(x)^T lvh (and lm += (dt/2) J_g,m(x)^T lvh)
        lv   = lvh
    J_g^T lam = -(VJP of a with w = lam, v = 0).  The two Jacobian products
    met at the same positions x_t (end of step t-1, start of step t) are
    applied together, so each stored position costs one product.
    """
    _, _, traj = leapfrog(x0, v0, m, eps2, dt, steps, trajectory=True)
    n = traj.shape[1]
    lx = _d(u, (n, 3)).copy()   # adjoint of x_T
    lv = np.zeros((n, 3)) if uv is None else _d(uv, (n, 3)).copy()   # adjoint of v_T
    lm = np.zeros(n)
    half = 0.5 * dt
    # Weight on g(x_t) owed by the start kick of step t (none for t = T).
    carried = np.zeros((n, 3))
    for t in range(steps, 0, -1):
        # x_t is the output of step t-1 and the input of step t: its end kick
        # (weight lv = adjoint of v_t) and the start kick of step t share g(x_t).
        gx, gm = forces_vjp(traj[t], m, eps2, w=lv + carried)
        lx = lx - half * gx
        lm = lm - half * gm
        lvh = lv + dt * lx      # drift of step t-1
        lv = lvh                # start kick of step t-1 passes lvh to v_{t-1}
        carried = lvh           # ... and owes (dt/2) J_g(x_{t-1})^T lvh
    if steps > 0:
        gx, gm = forces_vjp(traj[0], m, eps2, w=carried)
        lx = lx - half * gx
        lm = lm - half * gm
    return lx, lv, lm


def energy(x, v, m, eps2: float) -> float:
    """E = 1/2 sum m |v|^2 - 1/2 sum_i m_i p_i (softened pair energy)."""
    x = _d(x, (-1, 3))
    v = _d(v, x.shape)
    m = _d(m, (x.shape[0],))
    _, p = forces(x, m, eps2)
    return float(0.5 * np.sum(m[:, None] * v * v) - 0.5 * np.sum(m * p))
