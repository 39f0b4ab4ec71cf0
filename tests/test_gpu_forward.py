"""GPU parity of nbody_forces (Eq. (gravity), Sec. I) against the FP64 oracle,
called through the C ABI via the Python binding."""

import os

import numpy as np
import pytest
import torch

from oracle import reference as R
from paper_0904_3659_amd import inputs
from tests.gpu_util import assert_parity, errors, host, need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nb():
    need_gpu()
    from paper_0904_3659_amd import nbody
    return nbody


def _run(nb, x, m, eps2, dev):
    a, p = nb.forces(to_dev(x, dev), to_dev(m, dev), eps2)
    torch.cuda.synchronize()
    return host(a), host(p)


@pytest.mark.parametrize("n", [2, 3, 17, 63, 64, 65, 255, 256, 257, 1000, 1025, 5000])
def test_small_and_ragged_sizes(nb, n):
    dev = need_gpu()
    g = np.random.default_rng(n)
    x = g.standard_normal((n, 3)).astype(np.float32)
    m = g.uniform(0.1, 1.0, n).astype(np.float32)
    a, p = _run(nb, x, m, 1e-3, dev)
    ar, pr = R.forces(x, m, 1e-3)
    assert_parity(a, p, ar, pr, label=f"random n={n}")


def test_empty_and_single(nb):
    dev = need_gpu()
    a, p = nb.forces(torch.zeros((0, 3), device=dev), torch.zeros((0,), device=dev), 1e-4)
    assert a.shape == (0, 3) and p.shape == (0,)
    a, p = _run(nb, np.array([[0.5, 0.5, 0.5]], np.float32), np.array([2.0], np.float32), 1e-4, dev)
    assert a.tolist() == [[0.0, 0.0, 0.0]] and p.tolist() == [0.0]


def test_two_body_exact(nb):
    dev = need_gpu()
    x = np.array([[0, 0, 0], [1, 0, 0]], np.float32)
    a, p = _run(nb, x, np.array([1.0, 2.0], np.float32), 3.0, dev)
    # s = 4: a_1 = (-m_2/8, 0, 0), p_1 = m_2/2 -- within one ulp
    np.testing.assert_allclose(a, [[-0.25, 0, 0], [0.125, 0, 0]], rtol=1.2e-7, atol=0)
    np.testing.assert_allclose(p, [1.0, 0.5], rtol=1.2e-7)


def test_zero_softening(nb):
    dev = need_gpu()
    x = np.array([[0, 0, 0], [2, 0, 0], [0, 4, 0]], np.float32)
    m = np.array([1, 1, 1], np.float32)
    a, p = _run(nb, x, m, 0.0, dev)
    ar, pr = R.forces(x, m, 0.0)
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(p))
    assert_parity(a, p, ar, pr, tol=1e-6, label="eps2=0")


def test_plummer_1k(nb):
    dev = need_gpu()
    w = inputs.plummer_1k()
    a, p = _run(nb, w.x, w.m, w.eps2, dev)
    ar, pr = R.forces(w.x, w.m, w.eps2)
    assert_parity(a, p, ar, pr, label=w.name)


@pytest.mark.parametrize("make", [inputs.plummer_64k, inputs.cube_64k])
def test_64k_full_oracle(nb, make):
    dev = need_gpu()
    w = make()
    a, p = _run(nb, w.x, w.m, w.eps2, dev)
    ar, pr = R.forces(w.x, w.m, w.eps2)
    assert_parity(a, p, ar, pr, label=w.name)


def test_1m_sampled_rows(nb):
    dev = need_gpu()
    w = inputs.plummer_1m_lognormal()
    a, p = _run(nb, w.x, w.m, w.eps2, dev)
    ar, pr = R.forces_rows(w.x, w.m, w.eps2, w.rows)
    assert_parity(a[w.rows], p[w.rows], ar, pr, label=w.name + " (4096 rows)")
    # momentum balance over the whole set, relative to sum m |a|
    mom = np.abs(np.sum(w.m[:, None].astype(np.float64) * a, 0))
    assert np.max(mom) <= 1e-4 * np.sum(w.m * np.linalg.norm(a, axis=1))


def test_bitwise_deterministic(nb):
    dev = need_gpu()
    w = inputs.plummer_1k()
    x, m = to_dev(w.x, dev), to_dev(w.m, dev)
    a1, p1 = nb.forces(x, m, w.eps2)
    a2, p2 = nb.forces(x, m, w.eps2)
    assert torch.equal(a1, a2) and torch.equal(p1, p2)


def test_exact_mass_scaling(nb):
    dev = need_gpu()
    w = inputs.plummer_1k()
    x, m = to_dev(w.x, dev), to_dev(w.m, dev)
    a1, p1 = nb.forces(x, m, w.eps2)
    a2, p2 = nb.forces(x, 4.0 * m, w.eps2)
    assert torch.equal(a2, 4.0 * a1) and torch.equal(p2, 4.0 * p1)


def test_length_scaling(nb):
    dev = need_gpu()
    w = inputs.plummer_1k()
    x, m = to_dev(w.x, dev), to_dev(w.m, dev)
    a1, p1 = nb.forces(x, m, w.eps2)
    a2, p2 = nb.forces(2.0 * x, m, 4.0 * w.eps2)
    torch.testing.assert_close(a2, a1 / 4.0, rtol=3e-7, atol=0)
    torch.testing.assert_close(p2, p1 / 2.0, rtol=3e-7, atol=0)


def test_permutation_equivariance(nb):
    dev = need_gpu()
    w = inputs.plummer_1k()
    perm = np.random.default_rng(3).permutation(w.n)
    a, p = _run(nb, w.x, w.m, w.eps2, dev)
    ap, pp = _run(nb, w.x[perm], w.m[perm], w.eps2, dev)
    e = errors(ap, pp, a[perm], p[perm])
    assert max(e) <= 1e-5


@pytest.mark.parametrize("n", [700, 3000])
def test_every_variant(nb, n):
    dev = need_gpu()
    g = np.random.default_rng(100 + n)
    x = inputs.plummer_positions(n, (60, n))
    m = g.uniform(0.1, 1.0, n).astype(np.float32)
    ar, pr = R.forces(x, m, 1e-4)
    try:
        for v in range(nb.variant_count(nb.FORWARD)):
            nb.set_variant(nb.FORWARD, v)
            a, p = _run(nb, x, m, 1e-4, dev)
            assert_parity(a, p, ar, pr, label=f"{nb.variant_names(nb.FORWARD)[v]} n={n}")
    finally:
        nb.set_variant(nb.FORWARD, -1)


@pytest.mark.parametrize("n", [1, 2, 3, 65, 129])
def test_every_variant_tiny(nb, n):
    # every variant, forced, at a few particles: one particle gives exactly
    # zero; otherwise a single ragged tile or block against the oracle
    dev = need_gpu()
    g = np.random.default_rng(200 + n)
    x = g.standard_normal((n, 3)).astype(np.float32)
    m = g.uniform(0.1, 1.0, n).astype(np.float32)
    ar, pr = R.forces(x, m, 1e-3)
    names = nb.variant_names(nb.FORWARD)
    try:
        for v in range(nb.variant_count(nb.FORWARD)):
            print(f"[tiny] {names[v]} n={n}", flush=True)
            nb.set_variant(nb.FORWARD, v)
            a, p = _run(nb, x, m, 1e-3, dev)
            if n == 1:
                assert a.tolist() == [[0.0, 0.0, 0.0]] and p.tolist() == [0.0], names[v]
            else:
                assert_parity(a, p, ar, pr, label=f"{names[v]} n={n}")
    finally:
        nb.set_variant(nb.FORWARD, -1)


def test_potential_optional_and_out(nb):
    dev = need_gpu()
    w = inputs.plummer_1k()
    x, m = to_dev(w.x, dev), to_dev(w.m, dev)
    a_ref, _ = nb.forces(x, m, w.eps2)
    a, p = nb.forces(x, m, w.eps2, potential=False)
    assert p is None and torch.equal(a, a_ref)
    out = (torch.full((w.n, 3), 7.0, device=dev), torch.full((w.n,), 7.0, device=dev))
    nb.forces(x, m, w.eps2, out=out)
    assert torch.equal(out[0], a_ref)


def test_invalid_arguments(nb):
    dev = need_gpu()
    x = torch.zeros((4, 3), device=dev)
    m = torch.ones((4,), device=dev)
    with pytest.raises(ValueError):
        nb.forces(x, m, -1.0)
    with pytest.raises(ValueError):
        nb.forces(x[:, :2], m, 1e-4)
    with pytest.raises(ValueError):
        nb.forces(torch.zeros((3, 4), device=dev).t(), m, 1e-4)   # not contiguous
    with pytest.raises(TypeError):
        nb.forces(x.double(), m, 1e-4)
    # overlap of output and input is rejected by the library itself
    with pytest.raises(nb.NBodyError) as ei:
        nb.forces(x, m, 1e-4, out=(x, None))
    assert ei.value.status == 1


@pytest.mark.parametrize("variant", [None, "fwd_b256_k1_u8", "fwd_la_w16", "fwd_row_k2"])
def test_fault_injection_then_recovery(nb, variant):
    # n = 5000 makes every split gather allocate its partial-sum workspace,
    # and n = 7000 the default pair-once kernel; the row-per-wave kernels
    # allocate nothing, so only their launch can fail
    dev = need_gpu()
    n = 7000 if variant is None else 5000
    x = to_dev(inputs.plummer_positions(n, (62, n)), dev)
    m = to_dev(inputs.equal_masses(n), dev)
    names = nb.variant_names(nb.FORWARD)
    nb.set_variant(nb.FORWARD, -1 if variant is None else names.index(variant))
    faults = (("launch", 4),) if variant and variant.startswith("fwd_row") else (("launch", 4), ("alloc", 3))
    try:
        good, _ = nb.forces(x, m, 1e-4)
        for what, status in faults:
            os.environ["NBODY_FAULT"] = what
            try:
                with pytest.raises(nb.NBodyError) as ei:
                    nb.forces(x, m, 1e-4)
                assert ei.value.status == status
            finally:
                del os.environ["NBODY_FAULT"]
        again, _ = nb.forces(x, m, 1e-4)
        assert torch.equal(good, again)
    finally:
        nb.set_variant(nb.FORWARD, -1)


@pytest.mark.parametrize("n", [2048 * 2, 4096 + 1, 2048 * 5 + 17, 2048 * 7])
def test_pair_once_block_rings(nb, n):
    # even and odd block counts, a ragged last block, one and many chunks
    dev = need_gpu()
    x = inputs.plummer_positions(n, (61, n))
    m = inputs.lognormal_masses(n, (61, n, 1))
    ar, pr = R.forces(x, m, 1e-4)
    names = nb.variant_names(nb.FORWARD)
    try:
        for name in [nm for nm in names if nm.startswith("fwd_sym")]:
            nb.set_variant(nb.FORWARD, names.index(name))
            a, p = _run(nb, x, m, 1e-4, dev)
            assert_parity(a, p, ar, pr, label=f"{name} n={n}")
            # momentum balance holds to rounding: each pair term enters twice
            mom = np.abs(np.sum(m[:, None].astype(np.float64) * a, 0)).max()
            assert mom <= 1e-5 * np.sum(m * np.linalg.norm(a, axis=1))
    finally:
        nb.set_variant(nb.FORWARD, -1)


def test_default_variant_choice(nb):
    names = nb.variant_names(nb.FORWARD)
    assert names[nb.selected_variant(nb.FORWARD, 1 << 20)].startswith("fwd_sym")
    assert names[nb.selected_variant(nb.FORWARD, 65536)].startswith("fwd_sym")
    assert not names[nb.selected_variant(nb.FORWARD, 1024)].startswith("fwd_sym")
    # the pair-once workspace is bounded (ring groups): default up to 2^24
    assert names[nb.selected_variant(nb.FORWARD, 1 << 22)].startswith("fwd_sym")
    assert names[nb.selected_variant(nb.FORWARD, 1 << 24)].startswith("fwd_sym")
    assert not names[nb.selected_variant(nb.FORWARD, (1 << 24) + 1)].startswith("fwd_sym")
    # one wave per row (two rows from 3,000 bodies) below 4,500 bodies
    assert names[nb.selected_variant(nb.FORWARD, 1024)] == "fwd_row_k1"
    assert names[nb.selected_variant(nb.FORWARD, 4096)] == "fwd_row_k2"
    assert names[nb.selected_variant(nb.FORWARD, 4500)].startswith("fwd_sym")
    b = nb.variant_names(nb.BACKWARD)
    assert b[nb.selected_variant(nb.BACKWARD, 1024)] == "bwd_row_k1"
    assert b[nb.selected_variant(nb.BACKWARD, 3999)] == "bwd_row_k2"
    assert b[nb.selected_variant(nb.BACKWARD, 4000)].startswith("bwd_sym")


def test_profile_hook(nb):
    dev = need_gpu()
    w = inputs.plummer_64k()
    x, m = to_dev(w.x, dev), to_dev(w.m, dev)
    nb.profile_enable(True)
    try:
        for _ in range(3):
            nb.forces(x, m, w.eps2)
        main_ms, total_ms, calls = nb.profile_read()
        assert calls == 3 and 0.0 < main_ms <= total_ms
        assert nb.profile_read()[2] == 0          # reading clears the record
        nb.forces(torch.zeros((0, 3), device=dev), torch.zeros((0,), device=dev), 1e-4)
        assert nb.profile_read()[2] == 0          # n = 0 launches nothing
    finally:
        nb.profile_enable(False)


@pytest.mark.parametrize("n", [1, 2, 65, 1000, 4097, 20000])
def test_one_launch_split_gather(nb, n):
    # splits of a row block added by the last workgroup to arrive: parity,
    # bitwise repeatability although the last arriver changes from run to
    # run, and ticket counters left at zero for the next call of another n
    dev = need_gpu()
    x = inputs.plummer_positions(n, (63, n))
    m = inputs.lognormal_masses(n, (63, n, 1))
    ar, pr = R.forces(x, m, 1e-4)
    names = nb.variant_names(nb.FORWARD)
    xd, md = to_dev(x, dev), to_dev(m, dev)
    try:
        for name in [nm for nm in names if nm.startswith("fwd_la")]:
            nb.set_variant(nb.FORWARD, names.index(name))
            a1, p1 = nb.forces(xd, md, 1e-4)
            a2, p2 = nb.forces(xd, md, 1e-4)
            assert torch.equal(a1, a2) and torch.equal(p1, p2), name
            assert_parity(host(a1), host(p1), ar, pr, label=f"{name} n={n}")
            xs = to_dev(inputs.plummer_positions(333, (64, 0)), dev)
            ms = to_dev(inputs.equal_masses(333), dev)
            a3, p3 = nb.forces(xs, ms, 1e-4)
            ar3, pr3 = R.forces(host(xs), host(ms), 1e-4)
            assert_parity(host(a3), host(p3), ar3, pr3, label=f"{name} n=333 after n={n}")
    finally:
        nb.set_variant(nb.FORWARD, -1)


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 127, 1000, 1024, 2049, 4097, 20000])
def test_row_per_wave(nb, n):
    # one wave per row (or per K rows), lanes splitting j, a fixed butterfly
    # over the 64 lane sums: parity, bitwise repeatability, the same a with
    # and without p, and rows past n (n not a multiple of K) never stored
    dev = need_gpu()
    x = inputs.plummer_positions(n, (66, n))
    m = inputs.lognormal_masses(n, (66, n, 1))
    ar, pr = R.forces(x, m, 1e-4)
    names = nb.variant_names(nb.FORWARD)
    xd, md = to_dev(x, dev), to_dev(m, dev)
    rows = [nm for nm in names if nm.startswith("fwd_row")]
    assert rows
    try:
        for name in rows:
            nb.set_variant(nb.FORWARD, names.index(name))
            a1 = torch.full((n + 8, 3), 7.0, device=dev)
            p1 = torch.full((n + 8,), 7.0, device=dev)
            nb.forces(xd, md, 1e-4, out=(a1[:n], p1[:n]))
            a2, p2 = nb.forces(xd, md, 1e-4)
            a3, p3 = nb.forces(xd, md, 1e-4, potential=False)
            assert p3 is None
            assert torch.equal(a1[:n], a2) and torch.equal(p1[:n], p2), name
            assert torch.equal(a2, a3), name
            assert bool((a1[n:] == 7.0).all()) and bool((p1[n:] == 7.0).all()), name
            assert_parity(host(a2), host(p2), ar, pr, label=f"{name} n={n}")
    finally:
        nb.set_variant(nb.FORWARD, -1)


@pytest.mark.parametrize("n", [1024, 20000])
def test_bound_forces(nb, n):
    # the prepared call gives the bits of forces(); new values written into
    # the bound x are picked up by the next call
    dev = need_gpu()
    x = to_dev(inputs.plummer_positions(n, (69, n)), dev)
    m = to_dev(inputs.lognormal_masses(n, (69, n, 1)), dev)
    a = torch.empty((n, 3), device=dev)
    p = torch.empty((n,), device=dev)
    a_only = torch.empty((n, 3), device=dev)
    call, call_a = nb.BoundForces(x, m, 1e-4, a, p), nb.BoundForces(x, m, 1e-4, a_only)
    for step in range(2):
        call()
        call_a()
        a_ref, p_ref = nb.forces(x, m, 1e-4)
        torch.cuda.synchronize()
        assert torch.equal(a, a_ref) and torch.equal(p, p_ref) and torch.equal(a_only, a_ref), step
        x.mul_(1.5)                        # the same storage, new values
    with pytest.raises(ValueError):
        nb.BoundForces(x, m[:-1], 1e-4, a)


def test_four_million(nb):
    # n = 2^22: the default pair-once kernel runs its ring in groups of
    # offsets (bounded workspace) with float64 running sums between groups;
    # the float32-sum gather errs ~1e-5 here and the float64-sum one ~1e-7
    # (the pair terms themselves stay float32 in all three)
    dev = need_gpu()
    w = inputs.plummer_4m_lognormal()
    ar, pr = R.forces_rows(w.x, w.m, w.eps2, w.rows)
    x, m = to_dev(w.x, dev), to_dev(w.m, dev)
    names = nb.variant_names(nb.FORWARD)
    assert names[nb.selected_variant(nb.FORWARD, w.n)].startswith("fwd_sym")
    try:
        nb.set_variant(nb.FORWARD, names.index("fwd_b64_k1_u8"))
        a32, p32 = nb.forces(x, m, w.eps2)
        nb.set_variant(nb.FORWARD, -1)
        a64, p64 = nb.forces(x, m, w.eps2, f64_sum=True)
        a_def, p_def = nb.forces(x, m, w.eps2)
        a_def2, p_def2 = nb.forces(x, m, w.eps2)
        assert torch.equal(a_def, a_def2) and torch.equal(p_def, p_def2)
    finally:
        nb.set_variant(nb.FORWARD, -1)
    e32 = errors(host(a32)[w.rows], host(p32)[w.rows], ar, pr)
    e64 = errors(host(a64)[w.rows], host(p64)[w.rows], ar, pr)
    e_def = errors(host(a_def)[w.rows], host(p_def)[w.rows], ar, pr)
    print(f"[parity] {w.name} float32-sum gather {e32}  float64-sum gather {e64}  "
          f"pair-once default {e_def}", flush=True)
    assert max(e64) <= 1e-6
    assert max(e64) * 10 <= max(e32)
    assert max(e_def) <= 1e-4


def test_above_a_million_default(nb):
    # 2^20 + 4,099 bodies, ragged: the default pair-once kernel with its
    # ring in several groups, on 4,096 oracle rows
    dev = need_gpu()
    n = (1 << 20) + 4099
    x = inputs.plummer_positions(n, (67, 0))
    m = inputs.lognormal_masses(n, (67, 1))
    rows = inputs.check_rows(n, 4096, (67, 2))
    assert nb.variant_names(nb.FORWARD)[nb.selected_variant(nb.FORWARD, n)].startswith("fwd_sym")
    a, p = _run(nb, x, m, 1e-6, dev)
    ar, pr = R.forces_rows(x, m, 1e-6, rows)
    assert_parity(a[rows], p[rows], ar, pr, label=f"default n={n} (4096 rows)")


@pytest.mark.parametrize("n", [4097, 2048 * 5 + 17, 20000])
def test_ring_groups(nb, n, monkeypatch):
    # a small workspace limit splits the ring into many launches (one to a
    # few offsets each); every split meets the oracle, is bitwise
    # repeatable, and with the potential dropped gives the same a
    dev = need_gpu()
    x = inputs.plummer_positions(n, (68, n))
    m = inputs.lognormal_masses(n, (68, n, 1))
    ar, pr = R.forces(x, m, 1e-4)
    xd, md = to_dev(x, dev), to_dev(m, dev)
    names = nb.variant_names(nb.FORWARD)
    try:
        for name in ("fwd_sym_w1_k2_o1", "fwd_sym_w4_k4_o1", "fwd_sym_w8_k4_o1", "fwd_sym_w4_k4_r8",
                     "fwd_sym_w8_k4_r8"):
            nb.set_variant(nb.FORWARD, names.index(name))
            for slots in (5, 7, 12):
                monkeypatch.setenv("NBODY_SYM_WORKSPACE", str(16 * n * slots))
                print(f"[ring groups] {name} n={n} budget {slots} slots", flush=True)
                a1, p1 = nb.forces(xd, md, 1e-4)
                a2, p2 = nb.forces(xd, md, 1e-4)
                a3, _ = nb.forces(xd, md, 1e-4, potential=False)
                torch.cuda.synchronize()
                assert torch.equal(a1, a2) and torch.equal(p1, p2) and torch.equal(a1, a3)
                assert_parity(host(a1), host(p1), ar, pr, label=f"{name} n={n} {slots} slots")
    finally:
        nb.set_variant(nb.FORWARD, -1)


@pytest.mark.parametrize("n", [20000, 70000])
def test_no_potential_kernel_same_acceleration(nb, n):
    # without p the pair-once kernels skip the potential terms; the
    # acceleration must not change by a bit
    dev = need_gpu()
    x = to_dev(inputs.plummer_positions(n, (65, n)), dev)
    m = to_dev(inputs.lognormal_masses(n, (65, n, 1)), dev)
    assert nb.variant_names(nb.FORWARD)[nb.selected_variant(nb.FORWARD, n)].startswith("fwd_sym")
    a_p, p = nb.forces(x, m, 1e-4)
    a_n, none = nb.forces(x, m, 1e-4, potential=False)
    assert none is None and torch.equal(a_p, a_n)


_PAIR_ONCE_REF = {}


def _pair_once_case(n):
    """Inputs and FP64 reference for the forced pair-once sweep: the full
    oracle up to 10^4 bodies, 2,048 seeded rows above."""
    if n not in _PAIR_ONCE_REF:
        x = inputs.plummer_positions(n, (66, n))
        m = inputs.lognormal_masses(n, (66, n, 1))
        rows = None if n <= 16384 else inputs.check_rows(n, 2048, (66, n, 2))
        if rows is None:
            ar, pr = R.forces(x, m, 1e-4)
        else:
            ar, pr = R.forces_rows(x, m, 1e-4, rows)
        _PAIR_ONCE_REF[n] = (x, m, rows, ar, pr)
    return _PAIR_ONCE_REF[n]


@pytest.mark.parametrize("n", [4097, 10257, (1 << 17) + 3])
def test_every_pair_once_variant_with_and_without_potential(nb, n):
    # Each pair-once forward kernel, forced, at a ragged size: the kernel
    # without the potential (which skips its terms in the pair loop) must
    # give the acceleration of the kernel with it bitwise, and both must
    # meet the oracle.  The leap-frog runs the no-potential kernels.
    dev = need_gpu()
    x, m, rows, ar, pr = _pair_once_case(n)
    xd, md = to_dev(x, dev), to_dev(m, dev)
    names = nb.variant_names(nb.FORWARD)
    sel = slice(None) if rows is None else rows
    try:
        for name in [nm for nm in names if nm.startswith("fwd_sym")]:
            print(f"[pair-once sweep] {name} n={n}", flush=True)
            nb.set_variant(nb.FORWARD, names.index(name))
            a_p, p = nb.forces(xd, md, 1e-4)
            a_n, none = nb.forces(xd, md, 1e-4, potential=False)
            torch.cuda.synchronize()
            assert none is None
            assert torch.equal(a_p, a_n), f"{name} n={n}: a differs without the potential"
            assert_parity(host(a_p)[sel], host(p)[sel], ar, pr, label=f"{name} n={n}")
            # the no-potential kernel on its own against the oracle's a
            e_mag, e_vec, _ = errors(host(a_n)[sel], pr, ar, pr)
            assert e_mag <= 1e-4 and e_vec <= 1e-4, name
    finally:
        nb.set_variant(nb.FORWARD, -1)


@pytest.mark.parametrize("n,variant", [(9999, "fwd_sym_w1_k2_o1"), (10000, "fwd_sym_w1_k2_r8"),
                                       (39999, "fwd_sym_w1_k4_r8"), (45001, "fwd_sym_w4_k4_r8")])
def test_default_band_edges(nb, n, variant):
    # The default at the edges of its size bands against the oracle (2,048
    # seeded rows above 16,384 bodies), and the same a without p.
    dev = need_gpu()
    names = nb.variant_names(nb.FORWARD)
    assert names[nb.selected_variant(nb.FORWARD, n)] == variant
    x, m, rows, ar, pr = _pair_once_case(n)
    xd, md = to_dev(x, dev), to_dev(m, dev)
    sel = slice(None) if rows is None else rows
    print(f"[default band] {variant} n={n}", flush=True)
    a_p, p = nb.forces(xd, md, 1e-4)
    a_n, _ = nb.forces(xd, md, 1e-4, potential=False)
    torch.cuda.synchronize()
    assert torch.equal(a_p, a_n)
    assert_parity(host(a_p)[sel], host(p)[sel], ar, pr, label=f"default {variant} n={n}")
