"""Exact softened all-pairs gravity (Fujiwara & Nakasato, arXiv:0904.3659)
on AMD Instinct MI355X (gfx950): hand-written HIP kernels behind a C ABI.

Importing the package loads nothing; the HIP library is loaded on first use
by :mod:`paper_0904_3659_amd.nbody` and raises if it is missing.
"""

# ``leapfrog`` names the submodule (the integrator); its entry point is
# ``nbody.leapfrog`` or ``leapfrog.leapfrog``.
__all__ = ["forces", "forces_backward", "forces_batched", "NBodyForces", "NBodyError"]


def __getattr__(name):
    if name in __all__:
        from . import nbody
        return getattr(nbody, name)
    raise AttributeError(name)
