"""Seeded workload generators: distributions, bounds and reproducibility."""

import math

import numpy as np
import pytest
from scipy import stats

from paper_0904_3659_amd import inputs


def test_plummer_radii_follow_truncated_cdf():
    x = inputs.plummer_positions(20000, (9, 9)).astype(np.float64)
    r = np.linalg.norm(x, axis=1)
    assert r.max() <= 10.0 * (1 + 1e-6)
    xmax = inputs.plummer_cdf(10.0)
    res = stats.kstest(r, lambda q: inputs.plummer_cdf(np.minimum(q, 10.0)) / xmax)
    assert res.pvalue > 1e-3
    # isotropy: mean direction near zero
    assert np.linalg.norm(np.mean(x / r[:, None], 0)) < 0.03


def test_reproducible_and_float32():
    a = inputs.plummer_positions(100, (1, 2))
    b = inputs.plummer_positions(100, (1, 2))
    c = inputs.plummer_positions(100, (1, 3))
    assert a.dtype == np.float32 and a.flags.c_contiguous and a.shape == (100, 3)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_masses():
    m = inputs.lognormal_masses(100000, (3, 1))
    assert m.dtype == np.float32 and np.all(m > 0)
    assert float(np.sum(m.astype(np.float64))) == pytest.approx(1.0, abs=1e-5)
    lm = np.log(m.astype(np.float64))
    assert np.std(lm) == pytest.approx(1.0, abs=0.02)
    e = inputs.equal_masses(1024)
    assert np.all(e == np.float32(1 / 1024))


def test_uniform_cube():
    x = inputs.uniform_cube(50000, (2, 1))
    assert x.min() >= 0.0 and x.max() < 1.0
    assert np.mean(x) == pytest.approx(0.5, abs=0.01)


def test_plummer_velocity_dispersion():
    # For the untruncated Plummer sphere (G = M = a = 1) the mean-square speed
    # is 2K/M = 3 pi / 32; truncation at r = 10 changes it by < 1%.
    x = inputs.plummer_positions(40000, (4, 0))
    v = inputs.plummer_velocities(x, (4, 4)).astype(np.float64)
    r = np.linalg.norm(x.astype(np.float64), axis=1)
    vesc = math.sqrt(2.0) * (1 + r * r) ** -0.25
    assert np.all(np.linalg.norm(v, axis=1) <= vesc * (1 + 1e-6))
    assert np.mean(np.sum(v * v, 1)) == pytest.approx(3 * math.pi / 32, rel=0.03)


def test_check_rows():
    r = inputs.check_rows(1 << 20, 4096, (3, 2))
    assert r.size == 4096 and np.unique(r).size == 4096
    assert r.min() >= 0 and r.max() < (1 << 20)


def test_ensemble_layout():
    ens = inputs.ensemble_4096(num_systems=64)
    s = ens.sizes()
    assert s.min() >= 8 and s.max() <= 2048
    assert ens.offsets[0] == 0 and ens.offsets[-1] == ens.x.shape[0] == ens.m.shape[0]
    for k in range(ens.num_systems):
        lo, hi = ens.offsets[k], ens.offsets[k + 1]
        assert np.all(ens.m[lo:hi] == np.float32(1.0 / s[k]))
    # system k is the same whatever the other systems are
    other = inputs.ensemble([s[0], 5], key=(5,))
    assert np.array_equal(other.x[: s[0]], ens.x[: s[0]])


def test_paper_experiment_standins():
    for k, (name, n, dt, eps) in enumerate(inputs.PAPER_EXPERIMENT_SETS):
        nm, x, v, m, e2, dt2 = inputs.paper_experiment_set(k)
        assert nm == name and x.shape == (n, 3) and v.shape == (n, 3) and m.shape == (n,)
        assert e2 == pytest.approx(eps * eps) and dt2 == dt
