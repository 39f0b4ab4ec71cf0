"""Property checks of the FP64 oracle over random small systems (hypothesis):
invariances and identities that Eq. (gravity) and its adjoint obey for any
positions, masses and softening, so that a mistake the fixed-case pins
happen to miss still fails on some drawn system."""

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import reference as R

SYSTEMS = st.tuples(
    st.integers(min_value=2, max_value=24),        # n
    st.integers(min_value=0, max_value=2**31 - 1),  # seed
    st.floats(min_value=1e-4, max_value=1.0),     # eps2
)


def _system(n, seed):
    g = np.random.default_rng(seed)
    x = g.uniform(-1.0, 1.0, (n, 3))
    m = g.uniform(0.1, 1.0, n)
    return x, m


def _scale(a):
    return max(1.0, float(np.abs(a).max()))


@settings(max_examples=40, deadline=None)
@given(SYSTEMS)
def test_translation_invariance(sys):
    n, seed, eps2 = sys
    x, m = _system(n, seed)
    a, p = R.forces(x, m, eps2)
    a2, p2 = R.forces(x + np.array([0.25, -0.5, 0.125]), m, eps2)
    assert np.abs(a2 - a).max() <= 1e-12 * _scale(a)
    assert np.abs(p2 - p).max() <= 1e-12 * _scale(p)


@settings(max_examples=40, deadline=None)
@given(SYSTEMS, st.floats(min_value=0.0, max_value=2 * np.pi))
def test_rotation_equivariance(sys, angle):
    n, seed, eps2 = sys
    x, m = _system(n, seed)
    c, s = np.cos(angle), np.sin(angle)
    rot = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]]) @ \
        np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])
    a, p = R.forces(x, m, eps2)
    ar, pr = R.forces(x @ rot.T, m, eps2)
    assert np.abs(ar - a @ rot.T).max() <= 1e-12 * _scale(a)
    assert np.abs(pr - p).max() <= 1e-12 * _scale(p)


@settings(max_examples=40, deadline=None)
@given(SYSTEMS)
def test_momentum_and_potential_symmetry(sys):
    n, seed, eps2 = sys
    x, m = _system(n, seed)
    a, p = R.forces(x, m, eps2)
    # pair antisymmetry of the softened force and symmetry of the potential
    d = x[:, None, :] - x[None, :, :]
    r = 1.0 / np.sqrt((d * d).sum(-1) + eps2)
    np.fill_diagonal(r, 0.0)
    bound = float((m[:, None] * m[None, :] * r ** 2).sum())
    assert np.abs((m[:, None] * a).sum(0)).max() <= 1e-12 * bound
    pair = float((m[:, None] * m[None, :] * r).sum())   # = 2 sum_{i<j} m_i m_j r_ij
    assert abs(float((m * p).sum()) - pair) <= 1e-12 * pair


@settings(max_examples=25, deadline=None)
@given(SYSTEMS)
def test_vjp_against_directional_difference(sys):
    n, seed, eps2 = sys
    x, m = _system(n, seed)
    g = np.random.default_rng(seed ^ 0x5EED)
    w, v = g.normal(size=(n, 3)), g.normal(size=n)
    dx, dm = g.normal(size=(n, 3)), g.normal(size=n)

    def loss(xx, mm):
        a, p = R.forces(xx, mm, eps2)
        return float((w * a).sum() + (v * p).sum())

    gx, gm = R.forces_vjp(x, m, eps2, w, v)
    h = 1e-6
    fd = (loss(x + h * dx, m + h * dm) - loss(x - h * dx, m - h * dm)) / (2 * h)
    an = float((gx * dx).sum() + (gm * dm).sum())
    assert an == pytest.approx(fd, rel=1e-5, abs=1e-7 * _scale(gx))
