"""Library calls captured in a HIP graph (torch.cuda.CUDAGraph) and replayed:
every replay must reproduce the eager result bitwise, with eager work between
the replays, for each kernel family (row-per-wave and pair-once forward;
pair-once adjoint; persistent batched with its ticket counters; the
device-resident leap-frog segments and their reverse sweep)."""

import numpy as np
import pytest
import torch

from paper_0904_3659_amd import inputs
from tests.gpu_util import need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nb():
    need_gpu()
    from paper_0904_3659_amd import nbody
    return nbody


def _replay_matches(fn, outs, other):
    """Capture fn() on a side stream after an eager warm-up there; replay
    three times with eager calls (``other``) and fills between replays."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    s.synchronize()
    ref = [o.clone() for o in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        fn()
    torch.cuda.synchronize()
    for r in range(3):
        for o in outs:
            o.fill_(float(r) + 7.0)
        other()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, ref):
            assert torch.equal(o, e), f"replay {r}"
    del g


@pytest.mark.parametrize("n", [1000, 10000, 40000])
def test_forward_graph(nb, n):
    dev = need_gpu()
    x = to_dev(inputs.plummer_positions(n, (70, n)), dev)
    m = to_dev(inputs.lognormal_masses(n, (70, n, 1)), dev)
    a = torch.empty((n, 3), device=dev)
    p = torch.empty((n,), device=dev)
    xo = to_dev(inputs.plummer_positions(777, (71, 0)), dev)
    mo = to_dev(inputs.equal_masses(777), dev)
    _replay_matches(lambda: nb.forces(x, m, 1e-4, out=(a, p)), [a, p],
                    lambda: nb.forces(xo, mo, 1e-4))


def test_backward_graph(nb):
    dev = need_gpu()
    n = 16384
    x = to_dev(inputs.plummer_positions(n, (72, 0)), dev)
    m = to_dev(inputs.lognormal_masses(n, (72, 1)), dev)
    wa = to_dev(inputs.normal((n, 3), (72, 2)), dev)
    wp = to_dev(inputs.normal((n,), (72, 3)), dev)
    gx = torch.empty((n, 3), device=dev)
    gm = torch.empty((n,), device=dev)
    _replay_matches(lambda: nb.forces_backward(x, m, 1e-4, wa, wp, out=(gx, gm)), [gx, gm],
                    lambda: nb.forces_backward(x[:5000], m[:5000], 1e-4, wa[:5000], wp[:5000]))


def test_batched_graph(nb):
    dev = need_gpu()
    ens = inputs.ensemble(np.random.default_rng(73).integers(8, 600, 300), key=(73,))
    x, m = to_dev(ens.x, dev), to_dev(ens.m, dev)
    a = torch.empty_like(x)
    p = torch.empty_like(m)
    _replay_matches(lambda: nb.forces_batched(x, m, ens.offsets, ens.eps2, out=(a, p)), [a, p],
                    lambda: nb.forces(x[:300], m[:300], 1e-4))


@pytest.mark.parametrize("n", [1500, 20000])
def test_leapfrog_graphs(nb, n):
    # whole leap-frog segments captured as one graph: the forward steps with
    # their position history, and the reverse sweep; n = 1500 runs the
    # row-per-wave force and adjoint (element-wise update launches, the
    # adjoint's auxiliary buffer), n = 20000 the pair-once kernels with the
    # updates in their reduction epilogue
    dev = need_gpu()
    x0 = to_dev(inputs.plummer_positions(n, (75, n)), dev)
    v0 = to_dev(inputs.plummer_velocities(inputs.plummer_positions(n, (75, n)), (75, n, 1)), dev)
    m = to_dev(inputs.lognormal_masses(n, (75, n, 2)), dev)
    a0, _ = nb.forces(x0, m, 1e-4, potential=False)
    steps = 6
    x, v, a = torch.empty_like(x0), torch.empty_like(v0), torch.empty_like(a0)
    hist = torch.empty((steps, n, 3), device=dev)

    def fwd():
        x.copy_(x0)
        v.copy_(v0)
        a.copy_(a0)
        nb.leapfrog_(x, v, a, m, 1e-4, 1e-3, steps, x_hist=hist)

    xo, mo = x0[: n // 2], m[: n // 2]
    _replay_matches(fwd, [x, v, a, hist], lambda: nb.forces(xo, mo, 1e-4))

    pos = torch.cat([x0[None], hist], dim=0).contiguous()
    lx0 = to_dev(inputs.normal((n, 3), (75, n, 3)), dev)
    lv0 = to_dev(inputs.normal((n, 3), (75, n, 4)), dev)
    lm0 = torch.zeros((n,), device=dev)
    lx, lv, lm = torch.empty_like(lx0), torch.empty_like(lv0), torch.empty_like(lm0)

    def rev():
        lx.copy_(lx0)
        lv.copy_(lv0)
        lm.copy_(lm0)
        nb.leapfrog_adjoint_(pos, m, 1e-4, 1e-3, lx, lv, lm,
                             flags=nb.LEAPFROG_FINAL | nb.LEAPFROG_INITIAL)

    _replay_matches(rev, [lx, lv, lm],
                    lambda: nb.forces_backward(xo, mo, 1e-4, lx0[: n // 2], None))

