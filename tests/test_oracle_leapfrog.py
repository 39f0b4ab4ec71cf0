"""Pins of the FP64 leap-frog reference (Eqs. (1)-(3), Sec. III, with the
physical acceleration g = -a) and of its reverse sweep: free motion, a
softened circular two-body orbit, time reversibility, energy drift, and
finite differences of the integrator itself."""

import math

import numpy as np
import pytest

from oracle import reference as R
from paper_0904_3659_amd import inputs


def test_free_particle():
    x0 = np.array([[0.5, -1.0, 2.0]])
    v0 = np.array([[0.25, 0.5, -0.125]])
    x, v = R.leapfrog(x0, v0, [1.0], 1e-4, 0.0625, 16)
    np.testing.assert_allclose(x, x0 + 16 * 0.0625 * v0, rtol=0, atol=1e-15)
    assert np.array_equal(v, v0)
    gx, gv, gm = R.leapfrog_vjp(x0, v0, [1.0], 1e-4, 0.0625, 16, [[1.0, 2.0, 3.0]])
    assert gx.tolist() == [[1.0, 2.0, 3.0]]
    np.testing.assert_allclose(gv, [[1.0, 2.0, 3.0]], rtol=1e-15)   # T = 16 * 1/16 = 1
    assert gm.tolist() == [0.0]


def test_softened_circular_orbit():
    # m1 = m2 = 1/2 at separation 1: relative acceleration (m1+m2) d/(d^2+eps^2)^1.5
    # so the circular angular speed is omega = (1 + eps^2)^(-3/4).  Attraction
    # (g = -a) is what keeps the pair bound.
    eps2, dt, steps = 1e-2, 1e-3, 2000
    om = (1 + eps2) ** -0.75
    x0 = np.array([[-0.5, 0, 0], [0.5, 0, 0]])
    v0 = np.array([[0, -0.5 * om, 0], [0, 0.5 * om, 0]])
    x, v = R.leapfrog(x0, v0, [0.5, 0.5], eps2, dt, steps)
    sep = x[1] - x[0]
    assert np.linalg.norm(sep) == pytest.approx(1.0, abs=1e-6)
    ang = math.atan2(sep[1], sep[0])
    assert ang == pytest.approx(om * dt * steps, rel=1e-6)


def test_time_reversibility():
    n = 64
    x0 = inputs.plummer_positions(n, (50, 0)).astype(np.float64)
    v0 = inputs.plummer_velocities(x0, (50, 1)).astype(np.float64)
    m = np.full(n, 1.0 / n)
    x, v = R.leapfrog(x0, v0, m, 1e-2, 1e-3, 64)
    xb, vb = R.leapfrog(x, -v, m, 1e-2, 1e-3, 64)
    np.testing.assert_allclose(xb, x0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(-vb, v0, rtol=0, atol=1e-12)


def test_energy_drift():
    n = 256
    x0 = inputs.plummer_positions(n, (51, 0)).astype(np.float64)
    v0 = inputs.plummer_velocities(x0, (51, 1)).astype(np.float64)
    m = np.full(n, 1.0 / n)
    e0 = R.energy(x0, v0, m, 1e-2)
    x, v = R.leapfrog(x0, v0, m, 1e-2, 1e-3, 64)
    assert abs((R.energy(x, v, m, 1e-2) - e0) / e0) <= 1e-4


def test_reverse_sweep_matches_directional_differences():
    n, steps, dt, eps2, h = 24, 12, 2e-2, 5e-2, 1e-6
    g = np.random.default_rng(3)
    x0 = g.standard_normal((n, 3))
    v0 = 0.3 * g.standard_normal((n, 3))
    m = g.uniform(0.02, 0.1, n)
    u = g.standard_normal((n, 3))
    gx, gv, gm = R.leapfrog_vjp(x0, v0, m, eps2, dt, steps, u)

    def L(x, v, mm):
        return float(np.sum(u * R.leapfrog(x, v, mm, eps2, dt, steps)[0]))

    for which in range(3):
        dx = g.standard_normal(x0.shape) if which == 0 else 0 * x0
        dv = g.standard_normal(v0.shape) if which == 1 else 0 * v0
        dm = g.standard_normal(m.shape) if which == 2 else 0 * m
        fd = (L(x0 + h * dx, v0 + h * dv, m + h * dm)
              - L(x0 - h * dx, v0 - h * dv, m - h * dm)) / (2 * h)
        an = np.sum(gx * dx) + np.sum(gv * dv) + np.sum(gm * dm)
        assert fd == pytest.approx(an, rel=1e-6), which


def test_reverse_sweep_with_final_velocity_weight():
    n, steps, dt, eps2, h = 16, 9, 2e-2, 5e-2, 1e-6
    g = np.random.default_rng(4)
    x0 = g.standard_normal((n, 3))
    v0 = 0.3 * g.standard_normal((n, 3))
    m = g.uniform(0.02, 0.1, n)
    u = g.standard_normal((n, 3))
    uv = g.standard_normal((n, 3))
    gx, gv, gm = R.leapfrog_vjp(x0, v0, m, eps2, dt, steps, u, uv)

    def L(x, v, mm):
        xT, vT = R.leapfrog(x, v, mm, eps2, dt, steps)
        return float(np.sum(u * xT) + np.sum(uv * vT))

    dx, dv, dm = (g.standard_normal(x0.shape), g.standard_normal(v0.shape),
                  g.standard_normal(m.shape))
    fd = (L(x0 + h * dx, v0 + h * dv, m + h * dm) - L(x0 - h * dx, v0 - h * dv, m - h * dm)) / (2 * h)
    an = np.sum(gx * dx) + np.sum(gv * dv) + np.sum(gm * dm)
    assert fd == pytest.approx(an, rel=1e-6)
