"""GPU parity of nbody_forces_backward (the VJP of Eq. (gravity)) against the
FP64 oracle gradient, which the CPU tests pin to finite differences."""

import numpy as np
import pytest
import torch

from oracle import reference as R
from paper_0904_3659_amd import inputs
from tests.gpu_util import host, need_gpu, to_dev

pytestmark = pytest.mark.gpu

# Normwise bound max_k |g - g_ref| / max_k |g_ref| and a per-row bound.
TOL_NORM = 1e-4
TOL_ROW = 1e-3


@pytest.fixture(scope="module")
def nb():
    need_gpu()
    from paper_0904_3659_amd import nbody
    return nbody


def _grad(nb, x, m, eps2, w, v, dev):
    gx, gm = nb.forces_backward(to_dev(x, dev), to_dev(m, dev), eps2,
                                None if w is None else to_dev(w, dev),
                                None if v is None else to_dev(v, dev))
    torch.cuda.synchronize()
    return host(gx), host(gm)


def _check(gx, gm, rx, rm, label):
    nx = np.linalg.norm(gx - rx, axis=1)
    ex = nx.max() / np.linalg.norm(rx, axis=1).max()
    em = np.abs(gm - rm).max() / np.abs(rm).max()
    big = np.linalg.norm(rx, axis=1) > 1e-2 * np.linalg.norm(rx, axis=1).max()
    row = (nx[big] / np.linalg.norm(rx, axis=1)[big]).max() if big.any() else 0.0
    print(f"[parity] {label} grad_x norm {ex:.2e} row {row:.2e} grad_m {em:.2e}", flush=True)
    assert ex <= TOL_NORM and em <= TOL_NORM and row <= TOL_ROW, label


def _system(n, seed):
    g = np.random.default_rng(seed)
    x = g.standard_normal((n, 3)).astype(np.float32)
    m = g.uniform(0.1, 1.0, n).astype(np.float32)
    w = g.standard_normal((n, 3)).astype(np.float32)
    v = g.standard_normal(n).astype(np.float32)
    return x, m, w, v


@pytest.mark.parametrize("n", [2, 3, 17, 64, 257, 1000, 3001])
def test_random_sizes(nb, n):
    dev = need_gpu()
    x, m, w, v = _system(n, n)
    gx, gm = _grad(nb, x, m, 1e-3, w, v, dev)
    rx, rm = R.forces_vjp(x, m, 1e-3, w, v)
    _check(gx, gm, rx, rm, f"random n={n}")


def test_single_particle(nb):
    dev = need_gpu()
    gx, gm = _grad(nb, np.zeros((1, 3), np.float32), np.ones(1, np.float32), 1e-4,
                   np.ones((1, 3), np.float32), np.ones(1, np.float32), dev)
    assert gx.tolist() == [[0.0, 0.0, 0.0]] and gm.tolist() == [0.0]


def test_adjoint_16k_against_oracle(nb):
    dev = need_gpu()
    wl = inputs.adjoint_16k()
    w, v = wl.extra["w"], wl.extra["v"]
    gx, gm = _grad(nb, wl.x, wl.m, wl.eps2, w, v, dev)
    rx, rm = R.forces_vjp(wl.x, wl.m, wl.eps2, w, v)
    _check(gx, gm, rx, rm, wl.name)
    # translation invariance and mass homogeneity of the GPU gradient
    assert np.abs(gx.sum(0)).max() <= 1e-5 * np.linalg.norm(gx, axis=1).sum()
    L = R.loss(wl.x, wl.m, wl.eps2, w, v)
    assert np.sum(wl.m.astype(np.float64) * gm) == pytest.approx(L, rel=1e-4)


def test_optional_upstreams(nb):
    dev = need_gpu()
    x, m, w, v = _system(500, 5)
    for ww, vv, label in ((w, None, "w only"), (None, v, "v only")):
        gx, gm = _grad(nb, x, m, 1e-3, ww, vv, dev)
        rx, rm = R.forces_vjp(x, m, 1e-3, ww, vv)
        _check(gx, gm, rx, rm, label)
    gx, gm = _grad(nb, x, m, 1e-3, None, None, dev)
    assert not gx.any() and not gm.any()


def test_every_variant(nb):
    dev = need_gpu()
    x, m, w, v = _system(2000, 9)
    rx, rm = R.forces_vjp(x, m, 1e-3, w, v)
    try:
        for k in range(nb.variant_count(nb.BACKWARD)):
            nb.set_variant(nb.BACKWARD, k)
            gx, gm = _grad(nb, x, m, 1e-3, w, v, dev)
            _check(gx, gm, rx, rm, nb.variant_names(nb.BACKWARD)[k])
    finally:
        nb.set_variant(nb.BACKWARD, -1)


@pytest.mark.parametrize("n", [1, 2, 3, 65, 129])
def test_every_variant_tiny(nb, n):
    # every adjoint variant, forced, at a few particles: one particle gives
    # exactly zero; otherwise a single ragged tile or block against the oracle
    dev = need_gpu()
    x, m, w, v = _system(n, 300 + n)
    rx, rm = R.forces_vjp(x, m, 1e-3, w, v)
    names = nb.variant_names(nb.BACKWARD)
    try:
        for k in range(nb.variant_count(nb.BACKWARD)):
            print(f"[tiny] {names[k]} n={n}", flush=True)
            nb.set_variant(nb.BACKWARD, k)
            gx, gm = _grad(nb, x, m, 1e-3, w, v, dev)
            if n == 1:
                assert not gx.any() and not gm.any(), names[k]
            else:
                _check(gx, gm, rx, rm, f"{names[k]} n={n}")
    finally:
        nb.set_variant(nb.BACKWARD, -1)


def test_autograd_function(nb):
    dev = need_gpu()
    x, m, w, v = _system(800, 11)
    xt = to_dev(x, dev).requires_grad_(True)
    mt = to_dev(m, dev).requires_grad_(True)
    a, p = nb.NBodyForces.apply(xt, mt, 1e-3)
    loss = (a * to_dev(w, dev)).sum() + (p * to_dev(v, dev)).sum()
    gx, gm = torch.autograd.grad(loss, (xt, mt))
    dx, dm = nb.forces_backward(to_dev(x, dev), to_dev(m, dev), 1e-3, to_dev(w, dev), to_dev(v, dev))
    assert torch.equal(gx, dx) and torch.equal(gm, dm)
    # only a used: grad_p is absent and passed as NULL
    xt.grad = None
    a, _ = nb.NBodyForces.apply(xt, mt, 1e-3)
    (a * to_dev(w, dev)).sum().backward()
    rx, _ = R.forces_vjp(x, m, 1e-3, w, None)
    gx = host(xt.grad)
    assert np.linalg.norm(gx - rx, axis=1).max() <= TOL_NORM * np.linalg.norm(rx, axis=1).max()


def test_deterministic(nb):
    dev = need_gpu()
    x, m, w, v = (to_dev(t, dev) for t in _system(3000, 13))
    g1 = nb.forces_backward(x, m, 1e-3, w, v)
    g2 = nb.forces_backward(x, m, 1e-3, w, v)
    assert torch.equal(g1[0], g2[0]) and torch.equal(g1[1], g2[1])


@pytest.mark.parametrize("n", [2048 * 2 + 5, 2048 * 3, 4096 * 5 + 100])
def test_pair_once_block_rings(nb, n):
    dev = need_gpu()
    x, m, w, v = _system(n, 40 + n)
    rx, rm = R.forces_vjp(x, m, 1e-3, w, v)
    names = nb.variant_names(nb.BACKWARD)
    try:
        for name in [nm for nm in names if nm.startswith("bwd_sym")]:
            nb.set_variant(nb.BACKWARD, names.index(name))
            gx, gm = _grad(nb, x, m, 1e-3, w, v, dev)
            _check(gx, gm, rx, rm, f"{name} n={n}")
            # optional upstreams through the pair-once path as well
            gx1, gm1 = _grad(nb, x, m, 1e-3, None, v, dev)
            rx1, rm1 = R.forces_vjp(x, m, 1e-3, None, v)
            _check(gx1, gm1, rx1, rm1, f"{name} n={n} v only")
    finally:
        nb.set_variant(nb.BACKWARD, -1)


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 1000, 3001, 6001])
def test_row_per_wave_adjoint(nb, n):
    # one wave per row (or per K rows), lanes splitting j: parity with and
    # without each upstream, bitwise repeatability, absent weights equal to
    # explicit zeros bitwise, and nothing stored past row n
    dev = need_gpu()
    x, m, w, v = _system(n, 70 + n)
    xd, md, wd, vd = to_dev(x, dev), to_dev(m, dev), to_dev(w, dev), to_dev(v, dev)
    names = nb.variant_names(nb.BACKWARD)
    rows = [nm for nm in names if nm.startswith("bwd_row")]
    assert rows
    try:
        for name in rows:
            nb.set_variant(nb.BACKWARD, names.index(name))
            for ww, vv, label in ((w, v, "w, v"), (w, None, "w"), (None, v, "v")):
                gx, gm = _grad(nb, x, m, 1e-3, ww, vv, dev)
                if n > 1:
                    rx, rm = R.forces_vjp(x, m, 1e-3, ww, vv)
                    _check(gx, gm, rx, rm, f"{name} n={n} {label}")
                else:
                    assert not gx.any() and not gm.any()
            gx1 = torch.full((n + 4, 3), 5.0, device=dev)
            gm1 = torch.full((n + 4,), 5.0, device=dev)
            nb.forces_backward(xd, md, 1e-3, wd, vd, out=(gx1[:n], gm1[:n]))
            gx2, gm2 = nb.forces_backward(xd, md, 1e-3, wd, vd)
            assert torch.equal(gx1[:n], gx2) and torch.equal(gm1[:n], gm2), name
            assert bool((gx1[n:] == 5.0).all()) and bool((gm1[n:] == 5.0).all()), name
            gx3, gm3 = nb.forces_backward(xd, md, 1e-3, wd, None)
            gx4, gm4 = nb.forces_backward(xd, md, 1e-3, wd, torch.zeros((n,), device=dev))
            assert torch.equal(gx3, gx4) and torch.equal(gm3, gm4), name
    finally:
        nb.set_variant(nb.BACKWARD, -1)


@pytest.mark.parametrize("n", [16384, 70000])
def test_no_potential_weights_kernel(nb, n):
    # grad_p None takes the pair-once kernel that does not form the
    # potential-weight terms; it must agree with explicit zero weights
    dev = need_gpu()
    x = to_dev(inputs.plummer_positions(n, (66, n)), dev)
    m = to_dev(inputs.lognormal_masses(n, (66, n, 1)), dev)
    ga = to_dev(inputs.normal((n, 3), (66, n, 2)), dev)
    names = nb.variant_names(nb.BACKWARD)
    v = nb.selected_variant(nb.BACKWARD, n)
    assert names[v].startswith("bwd_sym")
    zero = torch.zeros((n,), device=dev)
    # the default without weights may take another block shape: equal up
    # to float32 summation order
    gx0, gm0 = nb.forces_backward(x, m, 1e-4, ga, zero)
    gx1, gm1 = nb.forces_backward(x, m, 1e-4, ga, None)
    for g0, g1 in ((gx0, gx1), (gm0, gm1)):
        e = ((g0 - g1).abs().max() / g0.abs().max()).item()
        assert e <= 1e-5, e
    # the same variant with and without the weight terms: bitwise
    nb.set_variant(nb.BACKWARD, v)
    try:
        gx2, gm2 = nb.forces_backward(x, m, 1e-4, ga, None)
    finally:
        nb.set_variant(nb.BACKWARD, -1)
    assert torch.equal(gx0, gx2) and torch.equal(gm0, gm2)


@pytest.mark.parametrize("n", [4097, 10257])
def test_every_pair_once_variant_without_potential_weights(nb, n):
    # Each pair-once adjoint, forced: without potential weights (grad_p
    # NULL, the kernel that skips their terms) it must equal the same
    # variant with explicit zero weights bitwise, and meet the oracle.  The
    # leap-frog adjoint runs these kernels.
    dev = need_gpu()
    x, m, w, _ = _system(n, 60 + n)
    rx, rm = R.forces_vjp(x, m, 1e-3, w, None)
    xd, md, wd = to_dev(x, dev), to_dev(m, dev), to_dev(w, dev)
    zero = torch.zeros((n,), device=dev)
    names = nb.variant_names(nb.BACKWARD)
    try:
        for name in [nm for nm in names if nm.startswith("bwd_sym")]:
            print(f"[adjoint sweep] {name} n={n}", flush=True)
            nb.set_variant(nb.BACKWARD, names.index(name))
            gx0, gm0 = nb.forces_backward(xd, md, 1e-3, wd, zero)
            gx1, gm1 = nb.forces_backward(xd, md, 1e-3, wd, None)
            torch.cuda.synchronize()
            assert torch.equal(gx0, gx1) and torch.equal(gm0, gm1), name
            _check(host(gx1), host(gm1), rx, rm, f"{name} n={n} no v")
    finally:
        nb.set_variant(nb.BACKWARD, -1)


@pytest.mark.parametrize("n,variant", [(3999, "bwd_row_k2"), (4000, "bwd_sym_s2_k2_r8"),
                                       (4801, "bwd_sym_s2_k2_r8"), (9001, "bwd_sym_s2_k2_r8"),
                                       (11999, "bwd_sym_s2_k2_r8"), (25003, "bwd_sym_w1_k2_r16")])
def test_mid_n_defaults(nb, n, variant):
    # the step-split blocks (4,000 to 11,999) and sixteen rounds (24,000 to
    # 29,999) as the default, with and without potential weights, against
    # the oracle (one choice for both)
    dev = need_gpu()
    names = nb.variant_names(nb.BACKWARD)
    assert names[nb.selected_variant(nb.BACKWARD, n)] == variant
    x, m, w, v = _system(n, 73 + n)
    print(f"[adjoint default] n={n} {variant}", flush=True)
    for vv in (v, None):
        gx, gm = _grad(nb, x, m, 1e-3, w, vv, dev)
        rx, rm = R.forces_vjp(x, m, 1e-3, w, vv)
        _check(gx, gm, rx, rm, f"default n={n} {'v' if vv is not None else 'no v'}")


def test_large_n_defaults(nb):
    # the eight-round defaults from 2^16: at 70,000 bodies (4-wave blocks)
    # against the oracle; at 2^18 + 5 (8-wave blocks, ring groups) against
    # the one-round kernel of the same blocks, which differs only in the
    # order of its float32 partial sums
    dev = need_gpu()
    names = nb.variant_names(nb.BACKWARD)
    n = 70000
    x, m, w, v = _system(n, 71)
    assert names[nb.selected_variant(nb.BACKWARD, n)] == "bwd_sym_w4_k2_r8"
    gx, gm = _grad(nb, x, m, 1e-3, w, v, dev)
    rx, rm = R.forces_vjp(x, m, 1e-3, w, v)
    _check(gx, gm, rx, rm, f"default n={n}")
    n = (1 << 18) + 5
    assert names[nb.selected_variant(nb.BACKWARD, n)] == "bwd_sym_w8_k2_r8"
    x, m, w, v = (to_dev(t, dev) for t in _system(n, 72))
    g_def = nb.forces_backward(x, m, 1e-4, w, v)
    g_nov = nb.forces_backward(x, m, 1e-4, w, None)
    nb.set_variant(nb.BACKWARD, names.index("bwd_sym_w8_k2_o1"))
    try:
        g_one = nb.forces_backward(x, m, 1e-4, w, v)
        g_one_nov = nb.forces_backward(x, m, 1e-4, w, None)
    finally:
        nb.set_variant(nb.BACKWARD, -1)
    for a, b in zip(g_def + g_nov, g_one + g_one_nov):
        e = ((a - b).abs().max() / b.abs().max()).item()
        print(f"[large adjoint] n={n} eight rounds vs one: {e:.2e}", flush=True)
        assert e <= 1e-5, e


@pytest.mark.parametrize("n", [4097, 20000])
def test_adjoint_ring_groups(nb, n, monkeypatch):
    # the adjoint's ring split into many launches by a small workspace
    # limit: the oracle still holds and the result repeats bitwise
    dev = need_gpu()
    x, m, w, v = _system(n, 70 + n)
    rx, rm = R.forces_vjp(x, m, 1e-3, w, v)
    names = nb.variant_names(nb.BACKWARD)
    try:
        for name in ("bwd_sym_w1_k2_o1", "bwd_sym_w2_k2_o1", "bwd_sym_w8_k2_o1", "bwd_sym_w4_k2_r8",
                     "bwd_sym_w8_k2_r8", "bwd_sym_s2_k2_r8"):
            nb.set_variant(nb.BACKWARD, names.index(name))
            for slots in (5, 9):
                monkeypatch.setenv("NBODY_SYM_WORKSPACE", str(16 * n * slots))
                g1 = _grad(nb, x, m, 1e-3, w, v, dev)
                g2 = _grad(nb, x, m, 1e-3, w, v, dev)
                assert np.array_equal(g1[0], g2[0]) and np.array_equal(g1[1], g2[1])
                _check(g1[0], g1[1], rx, rm, f"{name} n={n} {slots} slots")
    finally:
        nb.set_variant(nb.BACKWARD, -1)
