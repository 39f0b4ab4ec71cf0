"""Host-side sanitizer runs (CPU only).

The FP64 reference is rebuilt with AddressSanitizer and UndefinedBehavior
Sanitizer into a small C test program that exercises every entry point
(optional NULL arguments, row subsets, empty systems, the integrator), and
the program must finish cleanly.  The host half of the HIP library
(argument checks, variant tables, tuning-cache parsing) is rebuilt the same
way, sanitizing host code only, and a test program walks its argument-check
paths, none of which touches a GPU.
"""

import os
import shutil
import subprocess

import pytest

from oracle import build as OB

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=" + "address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]

ORACLE_PROGRAM = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
void oracle_forces_rows(const double*, const double*, int64_t, double, const int64_t*, int64_t, double*, double*);
void oracle_forces(const double*, const double*, int64_t, double, double*, double*);
void oracle_forces_batched(const int64_t*, int64_t, const double*, const double*, double, double*, double*);
void oracle_forces_vjp(const double*, const double*, int64_t, double, const double*, const double*, double*, double*);
void oracle_leapfrog(double*, double*, const double*, int64_t, double, double, int64_t, double*, double*);
int main(void) {
    enum { N = 37 };
    double *x = malloc(sizeof(double) * 3 * N), *m = malloc(sizeof(double) * N);
    double *a = malloc(sizeof(double) * 3 * N), *p = malloc(sizeof(double) * N);
    double *w = malloc(sizeof(double) * 3 * N), *v = malloc(sizeof(double) * N);
    double *vel = calloc(3 * N, sizeof(double)), *g = malloc(sizeof(double) * 3 * N);
    double *traj = malloc(sizeof(double) * 3 * N * 4);
    for (int i = 0; i < N; ++i) {
        for (int c = 0; c < 3; ++c) { x[3*i+c] = (i * 7 + c * 3) % 11 - 5.0; w[3*i+c] = 0.1 * c - i * 0.01; }
        m[i] = 1.0 + i; v[i] = 0.5 - 0.02 * i;
    }
    int64_t rows[3] = {0, 36, 12};
    oracle_forces(x, m, N, 1e-2, a, p);
    oracle_forces(x, m, N, 1e-2, a, NULL);
    oracle_forces_rows(x, m, N, 1e-2, rows, 3, a, p);
    oracle_forces_rows(x, m, 0, 1e-2, NULL, 0, NULL, NULL);
    int64_t off[5] = {0, 0, 5, 6, N};
    oracle_forces_batched(off, 4, x, m, 1e-2, a, p);
    oracle_forces_vjp(x, m, N, 1e-2, w, v, a, p);
    oracle_forces_vjp(x, m, N, 1e-2, NULL, v, a, NULL);
    oracle_forces_vjp(x, m, N, 1e-2, w, NULL, a, p);
    oracle_leapfrog(x, vel, m, N, 1e-2, 1e-3, 3, traj, g);
    oracle_leapfrog(x, vel, m, N, 1e-2, 1e-3, 2, NULL, g);
    /* two-body closed form: a_1 = -m_2/8, p_1 = m_2/2 for d = 1, eps2 = 3 */
    double x2[6] = {0, 0, 0, 1, 0, 0}, m2[2] = {1, 2}, a2[6], p2[2];
    oracle_forces(x2, m2, 2, 3.0, a2, p2);
    if (a2[0] != -0.25 || p2[0] != 1.0) { printf("closed form failed\n"); return 1; }
    free(x); free(m); free(a); free(p); free(w); free(v); free(vel); free(g); free(traj);
    puts("ok");
    return 0;
}
"""


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    drv = tmp_path / "drv.c"
    drv.write_text(ORACLE_PROGRAM)
    exe = tmp_path / "drv"
    flags = [f for f in OB.CFLAGS if f not in ("-shared", "-fPIC")]
    subprocess.run(["gcc", *flags, *SAN, str(drv), OB.SOURCE, "-o", str(exe), "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "ok"


LIB_PROGRAM = r"""
#include <stdint.h>
#include <stdio.h>
#include <math.h>
#include "nbody.h"
int main(void) {
    float *F = (float *)0x10000;
    int bad = 0;
    bad |= nbody_forces(F, F, -1, 1e-4f, F, 0, 0) != NBODY_ERROR_INVALID_ARGUMENT;
    bad |= nbody_forces(F, F, 4, NAN, F, 0, 0) != NBODY_ERROR_INVALID_ARGUMENT;
    bad |= nbody_forces(F, (float *)0x90000, 4, 1e-4f, (float *)0x10008, 0, 0) != NBODY_ERROR_INVALID_ARGUMENT;
    bad |= nbody_forces(0, 0, 0, 1e-4f, 0, 0, 0) != NBODY_OK;
    bad |= nbody_forces_backward(F, F, 3, 1e-4f, 0, 0, 0, 0, 0) != NBODY_ERROR_INVALID_ARGUMENT;
    int64_t off1[3] = {0, 5, 3};
    bad |= nbody_forces_batched(off1, 2, F, F, 1e-4f, F, 0, 0) != NBODY_ERROR_INVALID_ARGUMENT;
    int64_t off0[1] = {0};
    bad |= nbody_forces_batched(off0, 0, 0, 0, 1e-4f, 0, 0, 0) != NBODY_OK;
    bad |= nbody_axpy(F, F, 4, 1.0f, 0) != NBODY_ERROR_INVALID_ARGUMENT;
    bad |= nbody_kick_drift(F, F, F, -2, 1.0f, 1.0f, 0) != NBODY_ERROR_INVALID_ARGUMENT;
    for (int k = 0; k < 3; ++k)
        for (int v = 0; v < nbody_variant_count(k); ++v)
            if (!nbody_variant_name(k, v)) bad = 1;
    bad |= nbody_set_variant(0, 1) != NBODY_OK;
    bad |= nbody_selected_variant(0, 1000) != 1;
    bad |= nbody_set_variant(0, -1) != NBODY_OK;
    bad |= nbody_selected_variant(0, 1 << 20) < 0;
    bad |= nbody_set_variant(9, 0) != NBODY_ERROR_INVALID_ARGUMENT;
    bad |= nbody_status_string((nbody_status)77)[0] == 0;
    bad |= nbody_last_error()[0] == 0;
    printf(bad ? "bad\n" : "ok\n");
    return bad;
}
"""


def test_library_host_code_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    from paper_0904_3659_amd import build as LB
    lib = tmp_path / "libnbody_san.so"
    flags = [f for f in LB.HIPFLAGS if not f.startswith("--offload-arch")]
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f]
    cache = tmp_path / "tune.json"
    cache.write_text('{"entries": [\n  {"kind": 0, "bucket": 10, "variant": "fwd_b64_k1_u8"},\n'
                     '  {"kind": 0, "bucket": 11, "variant": "no_such_variant"},\n  garbage\n]}\n')
    subprocess.run([hipcc, *flags, "--offload-arch=gfx950", *host_san, *LB.sources(), "-o", str(lib)],
                   check=True, capture_output=True)
    drv = tmp_path / "drv.c"
    drv.write_text(LIB_PROGRAM)
    exe = tmp_path / "drv"
    # the test program links the same (clang) sanitizer runtime as the library
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc)), "..", "lib", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = shutil.which("clang") or pytest.skip("clang not available")
    subprocess.run([clang, "-O1", *SAN, "-I", os.path.join(ROOT, "include"), str(drv), str(lib),
                    "-Wl,-rpath," + str(tmp_path), "-o", str(exe)], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", NBODY_TUNE_CACHE=str(cache),
               NBODY_VARIANT="1:2,9:9,0:x")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, (out.stdout + out.stderr)[-3000:]
    assert out.stdout.strip().endswith("ok")
