"""Pins of the FP64 reference gradient of L = sum_i w_i . a_i + v_i p_i, with
(a, p) from Eq. (gravity): central finite differences of the FP64 forward
sum, a hand-differentiated two-body case, and two exact identities
(translation invariance and homogeneity of degree one in the masses)."""

import numpy as np
import pytest

from oracle import reference as R


def _system(n, seed):
    g = np.random.default_rng(seed)
    x = g.standard_normal((n, 3))
    m = g.uniform(0.2, 2.0, n)
    w = g.standard_normal((n, 3))
    v = g.standard_normal(n)
    return x, m, w, v


def test_two_body_gradient_by_hand():
    # d = x1 - x2 = (1,0,0), eps^2 = 3: r = s^-1/2 = 1/2, r^3 = 1/8, r^5 = 1/32.
    # L = (m2 w1 - m1 w2).d r^3 + (m2 v1 + m1 v2) r, so with c = m2 w1 - m1 w2,
    # b = m2 v1 + m1 v2:  dL/dx1 = c r^3 - 3 (c.d) r^5 d - b r^3 d = -dL/dx2,
    # dL/dm1 = -(w2.d) r^3 + v2 r,  dL/dm2 = (w1.d) r^3 + v1 r.
    # m1=1, m2=2, w1=(1,2,3), w2=(-1,0,2), v1=0.5, v2=-1.5:
    # c = (3,4,4), c.d = 3, b = -0.5.
    x = np.array([[1.0, 0, 0], [0.0, 0, 0]])
    m = np.array([1.0, 2.0])
    w = np.array([[1.0, 2, 3], [-1.0, 0, 2]])
    v = np.array([0.5, -1.5])
    gx, gm = R.forces_vjp(x, m, 3.0, w, v)
    assert gx.tolist() == [[0.15625, 0.5, 0.5], [-0.15625, -0.5, -0.5]]
    assert gm.tolist() == [-0.625, 0.375]


@pytest.mark.parametrize("n", [2, 5, 12])
def test_full_central_difference(n):
    x, m, w, v = _system(n, n)
    eps2, h = 0.05, 1e-5
    gx, gm = R.forces_vjp(x, m, eps2, w, v)
    fx = np.zeros_like(x)
    for k in range(n):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[k, c] += h
            xm[k, c] -= h
            fx[k, c] = (R.loss(xp, m, eps2, w, v) - R.loss(xm, m, eps2, w, v)) / (2 * h)
    fm = np.zeros(n)
    for k in range(n):
        mp, mmn = m.copy(), m.copy()
        mp[k] += h
        mmn[k] -= h
        fm[k] = (R.loss(x, mp, eps2, w, v) - R.loss(x, mmn, eps2, w, v)) / (2 * h)
    scale_x = np.abs(gx).max()
    assert np.max(np.abs(fx - gx)) <= 1e-7 * scale_x
    assert np.max(np.abs(fm - gm)) <= 1e-7 * np.abs(gm).max()


def test_directional_difference_medium():
    x, m, w, v = _system(400, 11)
    eps2, h = 1e-3, 1e-6
    g = np.random.default_rng(12)
    dx = g.standard_normal(x.shape)
    dm = g.standard_normal(m.shape)
    gx, gm = R.forces_vjp(x, m, eps2, w, v)
    fd = (R.loss(x + h * dx, m + h * dm, eps2, w, v)
          - R.loss(x - h * dx, m - h * dm, eps2, w, v)) / (2 * h)
    an = np.sum(gx * dx) + np.sum(gm * dm)
    assert fd == pytest.approx(an, rel=1e-6)


def test_translation_invariance():
    x, m, w, v = _system(300, 21)
    gx, _ = R.forces_vjp(x, m, 1e-3, w, v)
    assert np.max(np.abs(gx.sum(0))) <= 1e-13 * np.abs(gx).sum()


def test_mass_homogeneity():
    # a and p are linear in the masses, so sum_k m_k dL/dm_k = L.
    x, m, w, v = _system(250, 31)
    _, gm = R.forces_vjp(x, m, 1e-3, w, v)
    assert np.sum(m * gm) == pytest.approx(R.loss(x, m, 1e-3, w, v), rel=1e-12)


def test_optional_upstreams():
    x, m, w, v = _system(30, 41)
    gx_w, gm_w = R.forces_vjp(x, m, 1e-2, w, None)
    gx_v, gm_v = R.forces_vjp(x, m, 1e-2, None, v)
    gx, gm = R.forces_vjp(x, m, 1e-2, w, v)
    np.testing.assert_allclose(gx_w + gx_v, gx, rtol=1e-12, atol=1e-12 * np.abs(gx).max())
    np.testing.assert_allclose(gm_w + gm_v, gm, rtol=1e-12, atol=1e-12 * np.abs(gm).max())
    gx0, gm0 = R.forces_vjp(x, m, 1e-2, None, None)
    assert not gx0.any() and not gm0.any()
