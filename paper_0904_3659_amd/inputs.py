"""Seeded synthetic particle sets for the exact softened all-pairs sum.

This module holds none of the method's arithmetic.  It only draws random
numbers and shapes them into particle sets (positions, masses, velocities,
upstream weights).  The HIP path and the FP64 reference both read the same
float32 arrays built here: values are drawn in float64 and rounded to float32
once, so a comparison isolates the arithmetic of the two evaluators.

Workloads stand in for the paper's galaxy and random-body inputs (Sec. V-A:
N from 7,500 to 100,000, softening 0.01 to 0.1), whose data are not
published.  Every generator is keyed by a tuple fed to numpy's SeedSequence,
so a (workload, purpose, system) key always yields the same draws.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

PLUMMER_RMAX = 10.0


def rng(*key: int) -> np.random.Generator:
    """PCG64 generator for an integer key tuple."""
    return np.random.default_rng(np.random.SeedSequence([int(k) for k in key]))


def _f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _isotropic(g: np.random.Generator, n: int) -> np.ndarray:
    """Unit vectors uniform on the sphere: z ~ U(-1,1), phi ~ U(0, 2 pi)."""
    z = g.uniform(-1.0, 1.0, n)
    phi = g.uniform(0.0, 2.0 * math.pi, n)
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def plummer_cdf(r):
    """Enclosed-mass fraction of a Plummer sphere (G = M = scale radius = 1)."""
    r = np.asarray(r, dtype=np.float64)
    return r**3 / (1.0 + r * r) ** 1.5


def plummer_positions_f64(n: int, key, rmax: float = PLUMMER_RMAX) -> np.ndarray:
    """Plummer sphere truncated at radius ``rmax`` by inverse-CDF sampling.

    The enclosed-mass fraction X is drawn uniformly on [0, X(rmax)) and
    inverted exactly, r = (X^(-2/3) - 1)^(-1/2): the same law as rejecting
    r > rmax, with a fixed number of draws and no mass piled on the cut.
    """
    g = rng(*key)
    xmax = float(plummer_cdf(rmax))
    X = g.uniform(0.0, xmax, n)
    with np.errstate(divide="ignore"):
        r = 1.0 / np.sqrt(np.power(X, -2.0 / 3.0) - 1.0)
    r = np.minimum(r, rmax)  # guards only the last-ulp case of X == xmax
    return r[:, None] * _isotropic(g, n)


def plummer_positions(n: int, key, rmax: float = PLUMMER_RMAX) -> np.ndarray:
    return _f32(plummer_positions_f64(n, key, rmax))


def plummer_velocities(x: np.ndarray, key) -> np.ndarray:
    """Isotropic equilibrium velocities for a Plummer sphere (G = M = a = 1).

    Aarseth, Henon & Wielen (1974): the speed is q * v_esc(r) with
    v_esc = sqrt(2) (1 + r^2)^(-1/4) and q drawn by von Neumann rejection from
    g(q) proportional to q^2 (1 - q^2)^(7/2) (bounded by 0.1 on [0, 1]).
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    g = rng(*key)
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x1 = g.uniform(0.0, 1.0, todo.size)
        x2 = g.uniform(0.0, 0.1, todo.size)
        ok = x2 < x1 * x1 * (1.0 - x1 * x1) ** 3.5
        q[todo[ok]] = x1[ok]
        todo = todo[~ok]
    r2 = np.sum(x * x, axis=1)
    vesc = math.sqrt(2.0) * (1.0 + r2) ** -0.25
    return _f32((q * vesc)[:, None] * _isotropic(g, n))


def uniform_cube(n: int, key) -> np.ndarray:
    """Positions uniform in the unit cube [0, 1)^3."""
    return _f32(rng(*key).uniform(0.0, 1.0, (n, 3)))


def equal_masses(n: int, total: float = 1.0) -> np.ndarray:
    return _f32(np.full(n, total / max(n, 1)))


def lognormal_masses(n: int, key, sigma: float = 1.0) -> np.ndarray:
    """m_j = exp(sigma Z_j), Z ~ N(0,1), renormalised in float64 to sum 1."""
    z = rng(*key).standard_normal(n)
    m = np.exp(sigma * z)
    return _f32(m / m.sum())


def normal(shape, key) -> np.ndarray:
    """Seeded N(0,1) float32 array (upstream weights, loss directions)."""
    return _f32(rng(*key).standard_normal(shape))


def check_rows(n: int, count: int, key) -> np.ndarray:
    """Distinct row indices drawn without replacement (sampled oracle checks)."""
    count = min(count, n)
    return np.sort(rng(*key).choice(n, count, replace=False)).astype(np.int64)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    x: np.ndarray          # [n, 3] float32
    m: np.ndarray          # [n] float32
    eps2: float
    rows: np.ndarray | None = None      # sampled check rows (large n)
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def plummer_1k() -> Workload:
    """N = 1024 Plummer sphere, equal masses 1/N, eps^2 = 1e-4."""
    n = 1024
    return Workload("plummer_n1024_eq_eps2_1e-4", plummer_positions(n, (1, 0)),
                    equal_masses(n), 1e-4)


def plummer_64k() -> Workload:
    """N = 65,536 Plummer sphere, equal masses 1/N, eps^2 = 1e-4."""
    n = 65536
    return Workload("plummer_n65536_eq_eps2_1e-4", plummer_positions(n, (2, 0)),
                    equal_masses(n), 1e-4)


def cube_64k() -> Workload:
    """N = 65,536 uniform unit cube, equal masses 1/N, eps^2 = 1e-4."""
    n = 65536
    return Workload("cube_n65536_eq_eps2_1e-4", uniform_cube(n, (2, 1)),
                    equal_masses(n), 1e-4)


def plummer_1m_lognormal(n: int = 1 << 20, rows: int = 4096) -> Workload:
    """N = 2^20 Plummer sphere, log-normal (sigma 1) masses summing to 1,
    eps^2 = 1e-6, with ``rows`` seeded check rows."""
    return Workload(f"plummer_n{n}_lognormal_eps2_1e-6", plummer_positions(n, (3, 0)),
                    lognormal_masses(n, (3, 1)), 1e-6,
                    rows=check_rows(n, rows, (3, 2)))


def plummer_4m_lognormal(rows: int = 1024) -> Workload:
    """N = 2^22 Plummer sphere, log-normal (sigma 1) masses summing to 1,
    eps^2 = 1e-6, with ``rows`` seeded check rows (float32 growth study)."""
    n = 1 << 22
    return Workload(f"plummer_n{n}_lognormal_eps2_1e-6", plummer_positions(n, (7, 0)),
                    lognormal_masses(n, (7, 1)), 1e-6, rows=check_rows(n, rows, (7, 2)))


def adjoint_16k(n: int = 16384) -> Workload:
    """N = 16,384 Plummer sphere with log-normal masses and eps^2 = 1e-4.

    ``extra`` holds the upstream weights w [n,3], v [n] of the loss
    L = sum_i w_i . a_i + v_i p_i, a loss direction u [n,3] for the
    integrator test, and equilibrium velocities v0 [n,3].
    """
    x = plummer_positions(n, (4, 0))
    return Workload(f"plummer_n{n}_lognormal_eps2_1e-4_adjoint", x,
                    lognormal_masses(n, (4, 1)), 1e-4,
                    extra={"w": normal((n, 3), (4, 2, 0)),
                           "v": normal((n,), (4, 2, 1)),
                           "u": normal((n, 3), (4, 3)),
                           "v0": plummer_velocities(x, (4, 4))})


@dataclasses.dataclass
class Ensemble:
    name: str
    offsets: np.ndarray    # int64 [S + 1]
    x: np.ndarray          # [sum N_s, 3] float32
    m: np.ndarray          # [sum N_s] float32
    eps2: float

    @property
    def num_systems(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets)


def ensemble(sizes, key=(5,), eps2: float = 1e-4, name: str = "ensemble") -> Ensemble:
    """Independent Plummer systems; system s uses key + (1, s), masses 1/N_s."""
    sizes = np.asarray(sizes, dtype=np.int64)
    offsets = np.zeros(sizes.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    total = int(offsets[-1])
    x = np.empty((total, 3), dtype=np.float32)
    m = np.empty(total, dtype=np.float32)
    for s, ns in enumerate(sizes):
        lo, hi = offsets[s], offsets[s + 1]
        if ns:
            x[lo:hi] = plummer_positions(int(ns), tuple(key) + (1, s))
            m[lo:hi] = equal_masses(int(ns))
    return Ensemble(name, offsets, x, m, eps2)


def ensemble_4096(num_systems: int = 4096, nmin: int = 8, nmax: int = 2048) -> Ensemble:
    """4,096 independent Plummer systems, N_s ~ U{8..2048}, eps^2 = 1e-4."""
    sizes = rng(5, 0).integers(nmin, nmax + 1, num_systems)
    return ensemble(sizes, key=(5,), eps2=1e-4,
                    name=f"ensemble_{num_systems}x_n{nmin}-{nmax}_eq_eps2_1e-4")


# Stand-ins for the four inputs of the paper's experiments (Sec. V-A): three
# galaxy sets (figure-eight groups of 7,500 and 10,000 bodies, a cart-wheel
# collision of 18,000) and a random 100,000-body set, with the time steps and
# softening lengths the paper lists.  The galaxy initial conditions are not
# published; Plummer spheres with equilibrium velocities take their place,
# and the random set is uniform in the unit cube with velocities uniform in
# [-0.1, 0.1)^3.  Masses are 1/N.
PAPER_EXPERIMENT_SETS = (
    ("three_figure_eight_galaxies", 7500, 0.015625, 0.1),
    ("four_figure_eight_galaxies", 10000, 0.015625, 0.1),
    ("cart_wheel_galaxy", 18000, 0.0078125, 0.01),
    ("random_100000_body", 100000, 0.01, 0.01),
)


def paper_experiment_set(index: int):
    """(name, x0, v0, m, eps2, dt) of stand-in ``index`` (0..3)."""
    name, n, dt, eps = PAPER_EXPERIMENT_SETS[index]
    if index < 3:
        x = plummer_positions(n, (6, index, 0))
        v = plummer_velocities(x, (6, index, 1))
    else:
        x = uniform_cube(n, (6, index, 0))
        v = _f32(rng(6, index, 1).uniform(-0.1, 0.1, (n, 3)))
    return name, x, v, equal_masses(n), eps * eps, dt
