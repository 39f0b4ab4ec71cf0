"""The pins catch plausible mistakes.

Each case plants one mistake (a flipped sign, a dropped term, a wrong index
or exponent) in a private copy of the FP64 reference source, builds it with
the same flags, swaps it in, and requires at least one pin to fail.  The
planted copy lives in a temporary directory; the real reference is untouched.
"""

import ctypes
import os
import shutil
import subprocess

import pytest

from oracle import build as OB
from oracle import reference as R
from tests import test_oracle_forces as TF
from tests import test_oracle_leapfrog as TL
from tests import test_oracle_vjp as TV

MUTATIONS = {
    "flip_dx": ("const double dx = x[3 * i + 0] - x[3 * j + 0];",
                "const double dx = x[3 * j + 0] - x[3 * i + 0];"),
    "drop_softening": ("dz * dz + eps2;\n            const double inv_r = 1.0 / sqrt(s);            /* s^(-1/2) */",
                       "dz * dz;\n            const double inv_r = 1.0 / sqrt(s);            /* s^(-1/2) */"),
    "wrong_exponent": ("const double inv_r3 = inv_r * inv_r * inv_r;   /* s^(-3/2) */",
                       "const double inv_r3 = inv_r * inv_r;   /* s^(-3/2) */"),
    "mass_of_i": ("pot += m[j] * inv_r;", "pot += m[i] * inv_r;"),
    "self_term_kept": ("            if (j == i)\n                continue;\n            const double dx",
                       "            const double dx"),
    "vjp_drop_r5_term": ("- 3.0 * wd * inv_r5 * d[c]", ""),
    "vjp_sign_of_j_side": ("            acc[0] -= g[0];", "            acc[0] += g[0];"),
    "vjp_dm_wrong_index": ("+ (v ? v[j] : 0.0) * inv_r;", "+ (v ? v[k] : 0.0) * inv_r;"),
    "leapfrog_repulsive": ("    for (int64_t t = 0; t < len; ++t)\n            g_work[t] = -g_work[t];\n        axpy(len, 0.5 * dt, g_work, v);        /* Eq. (3) */",
                           "    axpy(len, 0.5 * dt, g_work, v);        /* Eq. (3) */"),
    "leapfrog_full_kick": ("axpy(len, 0.5 * dt, g_work, v);        /* Eq. (3) */",
                           "axpy(len, dt, g_work, v);        /* Eq. (3) */"),
}

PINS = [
    (TF.test_two_body_exact, ()), (TF.test_cube_corners, ()),
    (TF.test_single_and_empty, ()), (TF.test_self_term_excluded_by_index, ()),
    (TF.test_acceleration_is_minus_gradient_of_potential, ()),
    (TF.test_mpmath_brute_force, (5, 2)), (TF.test_momentum_balance, ()),
    (TV.test_two_body_gradient_by_hand, ()), (TV.test_full_central_difference, (5,)),
    (TV.test_translation_invariance, ()), (TV.test_mass_homogeneity, ()),
    (TL.test_softened_circular_orbit, ()), (TL.test_energy_drift, ()),
    (TL.test_reverse_sweep_matches_directional_differences, ()),
]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(OB.SOURCE).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    planted = tmp_path / "planted.c"
    planted.write_text(src.replace(old, new))
    so = tmp_path / f"libplanted_{name}.so"
    subprocess.run(["gcc", *OB.CFLAGS, str(planted), "-o", str(so), "-lm"], check=True)
    saved = R.lib()
    R._LIB = R.configure(ctypes.CDLL(str(so)))
    failed = []
    try:
        for fn, args in PINS:
            try:
                fn(*args)
            except AssertionError:
                failed.append(fn.__name__)
    finally:
        R._LIB = saved
    assert failed, f"no pin caught the planted mistake {name}"


def test_unplanted_copy_passes(tmp_path):
    so = tmp_path / "libcopy.so"
    shutil.copy(OB.SOURCE, tmp_path / "copy.c")
    subprocess.run(["gcc", *OB.CFLAGS, str(tmp_path / "copy.c"), "-o", str(so), "-lm"], check=True)
    saved = R.lib()
    R._LIB = R.configure(ctypes.CDLL(str(so)))
    try:
        for fn, args in PINS:
            fn(*args)
    finally:
        R._LIB = saved
