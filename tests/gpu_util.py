"""Shared helpers of the GPU parity tests (no arithmetic of the method)."""

import numpy as np
import pytest
import torch

# Tolerance of the float32 path against the FP64 oracle: max relative error
# on |a_i| and on p_i (and the stricter vector error |a_gpu - a_ref|/|a_ref|).
TOL = 1e-4


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda", 0)


def to_dev(arr, dev):
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float32)).to(dev)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def errors(a_gpu, p_gpu, a_ref, p_ref):
    """(max |.|a|-|a_ref|.|/|a_ref|, max |a-a_ref|/|a_ref|, max |p-p_ref|/p_ref)."""
    a_gpu = np.asarray(a_gpu, np.float64)
    a_ref = np.asarray(a_ref, np.float64)
    na = np.linalg.norm(a_ref, axis=1)
    ok = na > 0
    mag = np.abs(np.linalg.norm(a_gpu, axis=1) - na)[ok] / na[ok]
    vec = np.linalg.norm(a_gpu - a_ref, axis=1)[ok] / na[ok]
    pe = np.abs(np.asarray(p_gpu, np.float64) - p_ref)[p_ref > 0] / p_ref[p_ref > 0]
    f = lambda v: float(v.max()) if v.size else 0.0
    return f(mag), f(vec), f(pe)


def assert_parity(a_gpu, p_gpu, a_ref, p_ref, tol=TOL, label=""):
    e_mag, e_vec, e_p = errors(a_gpu, p_gpu, a_ref, p_ref)
    print(f"[parity] {label} |a| {e_mag:.2e} vec {e_vec:.2e} p {e_p:.2e}", flush=True)
    assert e_mag <= tol, f"{label}: |a| rel err {e_mag:.3e} > {tol}"
    assert e_vec <= tol, f"{label}: vector rel err {e_vec:.3e} > {tol}"
    assert e_p <= tol, f"{label}: p rel err {e_p:.3e} > {tol}"
