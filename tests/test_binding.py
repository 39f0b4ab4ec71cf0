"""The Python binding without a GPU: host tensors are refused (there is no
CPU fallback), shapes, dtypes and sizes are checked before any library
call, and a missing library raises on first use."""

import os
import subprocess
import sys

import pytest
import torch

from paper_0904_3659_amd import nbody as nb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_tensors_are_refused():
    x, v, a = torch.zeros((4, 3)), torch.zeros((4, 3)), torch.zeros((4, 3))
    m = torch.ones(4)
    calls = [
        lambda: nb.forces(x, m, 1e-4),
        lambda: nb.forces_backward(x, m, 1e-4, a),
        lambda: nb.forces_batched(x, m, [0, 2, 4], 1e-4),
        lambda: nb.axpy_(x, v, 1.0),
        lambda: nb.kick_drift_(x, v, a, -0.5e-3, 1e-3),
        lambda: nb.leapfrog_(x, v, a, m, 1e-4, 1e-3, 2),
        lambda: nb.leapfrog_adjoint_(torch.zeros((3, 4, 3)), m, 1e-4, 1e-3, x, v, m.clone()),
        lambda: nb.BoundForces(x, m, 1e-4, a),
    ]
    for call in calls:
        with pytest.raises(ValueError, match="HIP device"):
            call()


def test_arguments_checked_before_the_library():
    m = torch.ones(4)
    x = torch.zeros((4, 3))
    with pytest.raises(ValueError, match="steps"):
        nb.leapfrog_(x, x, x, m, 1e-4, 1e-3, -1)
    with pytest.raises(ValueError, match="pos must have shape"):
        nb.leapfrog_adjoint_(torch.zeros((4, 3)), m, 1e-4, 1e-3, x, x, m)
    with pytest.raises(ValueError, match="eps2"):
        nb._eps2(float("nan"))
    with pytest.raises(ValueError, match="eps2"):
        nb._eps2(-1e-4)


def test_missing_library_raises():
    env = dict(os.environ, NBODY_LIBRARY=os.path.join(ROOT, "no_such_libnbody.so"))
    code = "from paper_0904_3659_amd import nbody as nb\nnb.lib()\n"
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "NBodyError" in r.stderr and "is not built" in r.stderr
