"""Library calls on several streams and from several host threads: each
(device, stream) has its own workspace and ticket counters, so concurrent
calls must give the same bits as sequential ones."""

import threading

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


def _case(n, key, dev):
    return (to_dev(inputs.plummer_positions(n, (74, key)), dev),
            to_dev(inputs.lognormal_masses(n, (74, key, 1)), dev))


def test_two_streams_overlap(nb):
    # pair-once evaluations of three block shapes and a row-per-wave one in
    # flight on two streams at once
    dev = need_gpu()
    cases = [_case(n, k, dev) for k, n in enumerate((40000, 3000, 9000, 20000))]
    ref = [nb.forces(x, m, 1e-4) for x, m in cases]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for i, (x, m) in enumerate(cases):
        s = streams[i % 2]
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            outs.append(nb.forces(x, m, 1e-4))
    torch.cuda.synchronize()
    for (a, p), (ar, pr) in zip(outs, ref):
        assert torch.equal(a, ar) and torch.equal(p, pr)


def test_host_threads(nb):
    # two host threads, each on its own stream, each repeating forward,
    # adjoint, batched and leap-frog calls
    dev = need_gpu()
    x, m = _case(30000, 10, dev)
    g = to_dev(inputs.normal((30000, 3), (74, 11)), dev)
    ens = inputs.ensemble([300, 1000, 37, 2048], key=(74, 12))
    xe, me = to_dev(ens.x, dev), to_dev(ens.m, dev)
    v = to_dev(inputs.normal((30000, 3), (74, 13)), dev) * 0.1
    a0, _ = nb.forces(x, m, 1e-4, potential=False)

    def leapfrog():
        # three device-resident steps and the reverse sweep over them
        xs, vs, as_ = x.clone(), v.clone(), a0.clone()
        pos = torch.empty((4,) + tuple(x.shape), device=dev)
        pos[0].copy_(x)
        nb.leapfrog_(xs, vs, as_, m, 1e-4, 1e-3, 3, x_hist=pos[1:])
        lx, lv, lm = g.clone(), g.clone(), torch.zeros_like(m)
        nb.leapfrog_adjoint_(pos, m, 1e-4, 1e-3, lx, lv, lm, flags=3)
        return xs, vs, lx, lv, lm

    ref = (nb.forces(x, m, 1e-4), nb.forces_backward(x, m, 1e-4, g, None),
           nb.forces_batched(xe, me, ens.offsets, ens.eps2), leapfrog())
    torch.cuda.synchronize()
    errors = []

    def work():
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for _ in range(5):
                    got = (nb.forces(x, m, 1e-4), nb.forces_backward(x, m, 1e-4, g, None),
                           nb.forces_batched(xe, me, ens.offsets, ens.eps2), leapfrog())
                    s.synchronize()
                    for pair_got, pair_ref in zip(got, ref):
                        for t_got, t_ref in zip(pair_got, pair_ref):
                            if not torch.equal(t_got, t_ref):
                                errors.append("mismatch")
        except Exception as e:  # reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=work) for _ in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors[:3]


def test_checkpointed_gradient_from_host_threads(nb):
    # the eager checkpointed leap-frog gradient recomputes positions on a
    # second stream of its own thread: two threads, each on its own stream,
    # must reproduce the single-thread gradient bitwise
    dev = need_gpu()
    n = 3000
    x0 = to_dev(inputs.plummer_positions(n, (76, 0)), dev)
    v0 = to_dev(inputs.plummer_velocities(inputs.plummer_positions(n, (76, 0)), (76, 1)), dev)
    m0 = to_dev(inputs.lognormal_masses(n, (76, 2)), dev)
    u = to_dev(inputs.normal((n, 3), (76, 3)), dev)

    def grad():
        x, v, m = (t.clone().requires_grad_(True) for t in (x0, v0, m0))
        xT, _ = nb.leapfrog(x, v, m, 1e-4, 1e-3, 24, checkpoint_every=4, graphs=False)
        return torch.autograd.grad((xT * u).sum(), (x, v, m))

    ref = grad()
    torch.cuda.synchronize()
    errors = []

    def work():
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for _ in range(3):
                    got = grad()
                    s.synchronize()
                    if not all(torch.equal(a, b) for a, b in zip(got, ref)):
                        errors.append("mismatch")
        except Exception as e:  # reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=work) for _ in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors[:3]
