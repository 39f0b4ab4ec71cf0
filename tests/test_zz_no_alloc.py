"""nbody_forces_noalloc (the forward with its workspace in the library's
fixed device region) against nbody_forces, through the C ABI, and captured
in a HIP graph (torch.cuda.CUDAGraph) and replayed."""

import numpy as np
import pytest
import torch

from oracle import reference as R
from paper_0904_3659_amd import inputs
from tests.gpu_util import assert_parity, host, need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nb():
    need_gpu()
    from paper_0904_3659_amd import nbody
    return nbody


def _pair(nb, n, key, dev):
    x = to_dev(inputs.plummer_positions(n, (80, key)), dev)
    m = to_dev(inputs.lognormal_masses(n, (80, key, 1)), dev)
    a_ref, p_ref = nb.forces(x, m, 1e-4)
    a = torch.full((n, 3), float("nan"), device=dev)
    p = torch.full((n,), float("nan"), device=dev)
    nb.forces_noalloc(x, m, 1e-4, a, p)
    torch.cuda.synchronize()
    return x, m, a, p, a_ref, p_ref


# Workspace the fixed region offers (its last 4 KiB hold counters).
REGION = (64 << 20) - 4096


@pytest.mark.parametrize("sizes", [(20000, 1024), (9000, 333), (4097, 3001), (70001, 5003)])
def test_two_calls_in_a_row_match_nbody_forces(nb, sizes, monkeypatch):
    # Two calls in a row, the second smaller: the region keeps the first
    # call's partial sums, which must not leak into the second result.
    # With nbody_forces held to the same workspace limit both calls plan
    # the same launches, so the results must agree bitwise; both meet the
    # oracle.
    dev = need_gpu()
    monkeypatch.setenv("NBODY_SYM_WORKSPACE", str(REGION))
    for k, n in enumerate(sizes):
        print(f"[noalloc] n={n}", flush=True)
        x, m, a, p, a_ref, p_ref = _pair(nb, n, k, dev)
        assert torch.equal(a, a_ref) and torch.equal(p, p_ref), n
        rows = np.arange(0, n, max(1, n // 512))
        ar, pr = R.forces_rows(host(x), host(m), 1e-4, rows)
        assert_parity(host(a)[rows], host(p)[rows], ar, pr, label=f"noalloc n={n}")


@pytest.mark.parametrize("n", [20000, 70001])
def test_default_limit_differs_only_in_rounding(nb, n):
    # Without that limit nbody_forces may plan one launch where the region
    # needs several: the two results then differ in rounding only
    dev = need_gpu()
    x, m, a, p, a_ref, p_ref = _pair(nb, n, 11, dev)
    rows = np.arange(0, n, max(1, n // 512))
    ar, pr = R.forces_rows(host(x), host(m), 1e-4, rows)
    assert_parity(host(a)[rows], host(p)[rows], ar, pr, label=f"noalloc n={n}")
    assert_parity(host(a_ref)[rows], host(p_ref)[rows], ar, pr, label=f"nbody_forces n={n}")


def test_ring_split_to_fit_the_region(nb):
    # 2^18 bodies: the default plan needs more than the region, so the
    # pair-once ring runs in more launches; results within the tolerance
    dev = need_gpu()
    n = (1 << 18) + 77
    print(f"[noalloc] n={n}", flush=True)
    x, m, a, p, a_ref, p_ref = _pair(nb, n, 9, dev)
    rows = inputs.check_rows(n, 1024, (80, 9, 2))
    ar, pr = R.forces_rows(host(x), host(m), 1e-4, rows)
    assert_parity(host(a)[rows], host(p)[rows], ar, pr, label=f"noalloc n={n}")
    assert_parity(host(a_ref)[rows], host(p_ref)[rows], ar, pr, label=f"nbody_forces n={n}")
    # then a small call again, bitwise that of nbody_forces (its default
    # workspace fits the region at this size)
    x, m, a, p, a_ref, p_ref = _pair(nb, 3001, 10, dev)
    assert torch.equal(a, a_ref) and torch.equal(p, p_ref)


@pytest.mark.parametrize("n", [1000, 9000, 20000, 150001])
def test_captured_noalloc_replays(nb, n):
    # 1,000: the row-per-wave kernel; 9,000: the pair-once kernel in one
    # ring group; 20,000 and 150,001: the ring split into several groups to
    # fit the region, with the float64 running sum between them
    dev = need_gpu()
    print(f"[noalloc capture] n={n}", flush=True)
    x = to_dev(inputs.plummer_positions(n, (82, n)), dev)
    m = to_dev(inputs.lognormal_masses(n, (82, n, 1)), dev)
    a_ref = torch.full((n, 3), float("nan"), device=dev)
    p_ref = torch.full((n,), float("nan"), device=dev)
    nb.forces_noalloc(x, m, 1e-4, a_ref, p_ref)
    torch.cuda.synchronize()
    a = torch.full((n, 3), float("nan"), device=dev)
    p = torch.full((n,), float("nan"), device=dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        nb.forces_noalloc(x, m, 1e-4, a, p)
    torch.cuda.synchronize()
    xs = to_dev(inputs.plummer_positions(777, (82, 1)), dev)
    ms = to_dev(inputs.equal_masses(777), dev)
    for r in range(3):
        a.fill_(float("nan"))
        p.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(a, a_ref) and torch.equal(p, p_ref), (n, r)
        # eager work on the same region between the replays
        a2 = torch.empty((777, 3), device=dev)
        nb.forces_noalloc(xs, ms, 1e-4, a2)
        torch.cuda.synchronize()


def test_too_large_is_refused(nb):
    dev = need_gpu()
    n = 1 << 22
    x = torch.zeros((n, 3), device=dev)
    m = torch.zeros((n,), device=dev)
    a = torch.empty((n, 3), device=dev)
    with pytest.raises(nb.NBodyError) as ei:
        nb.forces_noalloc(x, m, 1e-4, a)
    assert ei.value.status == 1 and "workspace" in str(ei.value)
