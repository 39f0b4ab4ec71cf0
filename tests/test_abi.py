"""The C ABI without a GPU: the library loads, exports every entry point that
include/nbody.h declares, and rejects invalid arguments before any HIP call.
No compute call is made here."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_0904_3659_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nbody_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(B.LIBRARY):
        pytest.skip("libnbody.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(B.LIBRARY)
    lib.nbody_last_error.restype = ctypes.c_char_p
    lib.nbody_status_string.restype = ctypes.c_char_p
    lib.nbody_variant_name.restype = ctypes.c_char_p
    return lib


def test_every_declared_symbol_is_exported(L):
    names = declared()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIBRARY], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (nbody_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(L, n)


def test_abi_version_and_status_strings(L):
    assert L.nbody_abi_version() == 4
    for code, name in enumerate(["NBODY_OK", "NBODY_ERROR_INVALID_ARGUMENT",
                                 "NBODY_ERROR_UNSUPPORTED_DEVICE", "NBODY_ERROR_OUT_OF_MEMORY",
                                 "NBODY_ERROR_LAUNCH_FAILED", "NBODY_ERROR_INTERNAL"]):
        assert L.nbody_status_string(code).decode() == name


def test_variant_tables(L):
    for kind in (0, 1, 2):
        cnt = L.nbody_variant_count(kind)
        assert cnt >= 2
        names = [L.nbody_variant_name(kind, k).decode() for k in range(cnt)]
        assert len(set(names)) == cnt
        assert L.nbody_variant_name(kind, cnt) is None
    assert L.nbody_variant_count(7) == 0
    assert L.nbody_set_variant(0, 99) == 1
    assert L.nbody_set_variant(5, 0) == 1


vp, i64, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_float
FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: every call below fails validation


def test_forward_validation(L):
    L.nbody_forces.argtypes = [vp, vp, i64, f32, vp, vp, vp]
    assert L.nbody_forces(FAKE, FAKE, -1, 1e-4, FAKE, None, None) == 1
    assert L.nbody_forces(FAKE, FAKE, (1 << 28) + 1, 1e-4, FAKE, None, None) == 1
    assert L.nbody_forces(FAKE, FAKE, 4, -1.0, FAKE, None, None) == 1
    assert L.nbody_forces(FAKE, FAKE, 4, float("nan"), FAKE, None, None) == 1
    assert L.nbody_forces(FAKE, FAKE, 4, float("inf"), FAKE, None, None) == 1
    assert b"eps2" in L.nbody_last_error()
    assert L.nbody_forces(None, FAKE, 4, 1e-4, FAKE, None, None) == 1
    assert L.nbody_forces(FAKE, FAKE, 4, 1e-4, None, None, None) == 1
    # a overlapping x
    assert L.nbody_forces(FAKE, ctypes.c_void_p(0x90000), 4, 1e-4,
                          ctypes.c_void_p(0x10008), None, None) == 1
    assert b"overlap" in L.nbody_last_error()
    # n == 0 is a no-op that succeeds without touching the device
    assert L.nbody_forces(None, None, 0, 1e-4, None, None, None) == 0
    assert L.nbody_last_error() == b""


def test_forward_ex_validation(L):
    L.nbody_forces_ex.argtypes = [vp, vp, i64, f32, vp, vp, ctypes.c_uint32, vp]
    assert L.nbody_forces_ex(FAKE, FAKE, 4, 1e-4, FAKE, None, 2, None) == 1
    assert b"flag" in L.nbody_last_error()
    assert L.nbody_forces_ex(FAKE, FAKE, 4, -1.0, FAKE, None, 1, None) == 1
    assert L.nbody_forces_ex(FAKE, FAKE, -1, 1e-4, FAKE, None, 1, None) == 1
    assert L.nbody_forces_ex(None, None, 0, 1e-4, None, None, 1, None) == 0
    names = [L.nbody_variant_name(0, k).decode() for k in range(L.nbody_variant_count(0))]
    assert any(nm.endswith("_f64sum") for nm in names)


def test_backward_validation(L):
    L.nbody_forces_backward.argtypes = [vp, vp, i64, f32, vp, vp, vp, vp, vp]
    assert L.nbody_forces_backward(FAKE, FAKE, -3, 1e-4, None, None, FAKE, None, None) == 1
    assert L.nbody_forces_backward(FAKE, FAKE, 3, 1e-4, None, None, None, None, None) == 1
    assert L.nbody_forces_backward(FAKE, ctypes.c_void_p(0x90000), 3, 1e-4, None, None,
                                   ctypes.c_void_p(0x10004), None, None) == 1
    assert L.nbody_forces_backward(None, None, 0, 0.0, None, None, None, None, None) == 0


def test_batched_validation(L):
    L.nbody_forces_batched.argtypes = [ctypes.POINTER(i64), i64, vp, vp, f32, vp, vp, vp]

    def call(off, ns=None):
        o = np.asarray(off, dtype=np.int64)
        return L.nbody_forces_batched(o.ctypes.data_as(ctypes.POINTER(i64)),
                                      o.size - 1 if ns is None else ns, FAKE,
                                      ctypes.c_void_p(0x900000), 1e-4,
                                      ctypes.c_void_p(0xA00000), None, None)

    assert call([1, 5]) == 1
    assert call([0, 5, 3]) == 1
    assert call([0, 5], ns=-1) == 1
    assert L.nbody_forces_batched(None, 1, FAKE, FAKE, 1e-4, FAKE, None, None) == 1
    assert call([0, 0, 0]) == 0          # only empty systems: nothing to do
    assert call([0]) == 0                # no systems


def test_axpy_validation(L):
    L.nbody_axpy.argtypes = [vp, vp, i64, f32, vp]
    assert L.nbody_axpy(FAKE, FAKE, -1, 1.0, None) == 1
    assert L.nbody_axpy(FAKE, ctypes.c_void_p(0x10004), 4, 1.0, None) == 1
    assert L.nbody_axpy(FAKE, ctypes.c_void_p(0x90000), 4, float("nan"), None) == 1
    assert L.nbody_axpy(None, None, 0, 1.0, None) == 0


def test_autotune_validation(L):
    L.nbody_autotune.argtypes = [ctypes.c_int, ctypes.POINTER(i64), i64, vp]
    s = np.array([1], dtype=np.int64)
    assert L.nbody_autotune(0, s.ctypes.data_as(ctypes.POINTER(i64)), 1, None) == 1
    assert L.nbody_autotune(9, s.ctypes.data_as(ctypes.POINTER(i64)), 1, None) == 1
    assert L.nbody_autotune(0, None, 0, None) == 0


def test_kick_drift_validation(L):
    L.nbody_kick_drift.argtypes = [vp, vp, vp, i64, f32, f32, vp]
    assert L.nbody_kick_drift(FAKE, FAKE, FAKE, -1, 0.1, 0.1, None) == 1
    assert L.nbody_kick_drift(FAKE, ctypes.c_void_p(0x90000), ctypes.c_void_p(0xA0000), 4,
                              float("inf"), 0.1, None) == 1
    assert L.nbody_kick_drift(FAKE, ctypes.c_void_p(0x10004), ctypes.c_void_p(0xA0000), 4,
                              0.1, 0.1, None) == 1
    assert L.nbody_kick_drift(None, None, None, 0, 0.1, 0.1, None) == 0


def test_leapfrog_validation(L):
    L.nbody_leapfrog.argtypes = [vp, vp, vp, vp, i64, f32, f32, i64, vp, vp]
    X, V, A, M = (ctypes.c_void_p(0x100000 * k) for k in (1, 2, 3, 4))
    ok = lambda *a: L.nbody_leapfrog(*a, None)
    assert ok(X, V, A, M, -1, 1e-4, 1e-3, 1, None) == 1                 # n < 0
    assert ok(X, V, A, M, 4, -1.0, 1e-3, 1, None) == 1                  # eps2 < 0
    assert ok(X, V, A, M, 4, 1e-4, float("nan"), 1, None) == 1          # dt not finite
    assert ok(X, V, A, M, 4, 1e-4, 1e-3, -1, None) == 1                 # steps < 0
    assert ok(X, V, A, M, 4, 1e-4, 1e-3, (1 << 30) + 1, None) == 1      # steps too large
    assert ok(X, None, A, M, 4, 1e-4, 1e-3, 1, None) == 1               # NULL v
    assert ok(X, ctypes.c_void_p(0x100000 + 24), A, M, 4, 1e-4, 1e-3, 1, None) == 1  # x, v overlap
    # x_hist of 3 steps x 48 B reaches into a
    assert ok(X, V, A, M, 4, 1e-4, 1e-3, 3, ctypes.c_void_p(0x300000 - 100)) == 1
    assert ok(None, None, None, None, 0, 1e-4, 1e-3, 5, None) == 0      # n == 0
    assert ok(X, V, A, M, 4, 1e-4, 1e-3, 0, None) == 0                  # no steps


def test_leapfrog_adjoint_validation(L):
    L.nbody_leapfrog_adjoint.argtypes = [vp, vp, i64, f32, f32, i64, ctypes.c_uint32, vp, vp,
                                         vp, vp]
    P, M, LX, LV, LM = (ctypes.c_void_p(0x100000 * k) for k in (1, 2, 3, 4, 5))
    ok = lambda *a: L.nbody_leapfrog_adjoint(*a, None)
    assert ok(P, M, 4, 1e-4, 1e-3, 2, 4, LX, LV, LM) == 1               # unknown flag bit
    assert ok(P, M, -1, 1e-4, 1e-3, 2, 0, LX, LV, LM) == 1
    assert ok(P, M, 4, float("inf"), 1e-3, 2, 0, LX, LV, LM) == 1
    assert ok(P, M, 4, 1e-4, float("inf"), 2, 0, LX, LV, LM) == 1
    assert ok(P, M, 4, 1e-4, 1e-3, -2, 0, LX, LV, LM) == 1
    assert ok(P, M, 4, 1e-4, 1e-3, 2, 3, LX, None, LM) == 1             # NULL lv
    assert ok(P, M, 4, 1e-4, 1e-3, 2, 0, LX, LX, LM) == 1               # lx is lv
    # pos holds 3 x 48 B: with 0x100000 - 64 it runs into m
    assert ok(ctypes.c_void_p(0x200000 - 64), M, 4, 1e-4, 1e-3, 2, 0, LX, LV, LM) == 1
    assert ok(None, None, 0, 1e-4, 1e-3, 2, 3, None, None, None) == 0   # n == 0
    assert ok(P, M, 4, 1e-4, 1e-3, 0, 3, LX, LV, LM) == 0               # no steps


def test_autotune_batched_validation(L):
    L.nbody_autotune_batched.argtypes = [ctypes.POINTER(i64), i64, vp, vp, f32, vp]
    P = ctypes.POINTER(i64)
    ok = lambda o, s, x, m, e: L.nbody_autotune_batched(
        None if o is None else o.ctypes.data_as(P), s, x, m, e, None)
    X, M = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000)
    assert ok(None, 1, X, M, 1e-4) == 1                                   # NULL offsets
    assert ok(np.array([1, 4], dtype=np.int64), 1, X, M, 1e-4) == 1       # offsets[0] != 0
    assert ok(np.array([0, 4, 2], dtype=np.int64), 2, X, M, 1e-4) == 1    # decreasing
    assert ok(np.array([0, 4], dtype=np.int64), 1, X, M, -1.0) == 1       # eps2 < 0
    assert ok(np.array([0, 4], dtype=np.int64), 1, None, M, 1e-4) == 1    # NULL x
    assert ok(np.array([0, 4], dtype=np.int64), 1, X, ctypes.c_void_p(0x100000 + 8), 1e-4) == 1
    assert ok(np.array([0, 0, 0], dtype=np.int64), 2, None, None, 1e-4) == 0   # nothing to time
