"""The variant timer's gate and the pair-once workspace bound, on the CPU:
nbody_variant_plan computes a variant's launch plan from its arguments
alone (no device), with the same functions the library launches with."""

import ctypes
import os

import pytest

from paper_0904_3659_amd import build as B

GiB = 1 << 30


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(B.LIBRARY):
        pytest.skip("libnbody.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(B.LIBRARY)
    lib.nbody_variant_plan.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_int)]
    lib.nbody_variant_plan.restype = ctypes.c_int64
    lib.nbody_variant_name.restype = ctypes.c_char_p
    return lib


def names(L, kind):
    return [L.nbody_variant_name(kind, k).decode() for k in range(L.nbody_variant_count(kind))]


def plan(L, kind, name, n, per_cu, free=256 * GiB, num_cu=256):
    timed = ctypes.c_int(-1)
    b = L.nbody_variant_plan(kind, names(L, kind).index(name), n, num_cu, per_cu, free,
                             ctypes.byref(timed))
    return b, timed.value


def test_pair_once_workspace_closed_form(L):
    # 2^20 bodies in 512 blocks of 2,048, two workgroups per CU on 256 CUs:
    # one chunk per block; 256 ring offsets; a 1 GiB budget holds 64 slots
    # of 16 MiB, so 5 groups of 52 offsets: (1 + 52) slots plus the float64
    # running sum (32 bytes per body)
    n = 1 << 20
    b, _ = plan(L, 0, "fwd_sym_w8_k4_o1", n, 2)
    assert b == 53 * 16 * n + 32 * n
    # eight rounds (the default here): 8 chunks per block, the same 5
    # groups of 52 offsets, (8 + 52) slots plus the running sum
    b, _ = plan(L, 0, "fwd_sym_w8_k4_r8", n, 2)
    assert b == 60 * 16 * n + 32 * n
    # small n: the whole ring in one launch, no running sum: chunks fill the
    # 2 x 256 resident workgroups (M = 8 blocks -> 64 chunks, capped at the
    # 5 x 32 tiles of a block's sequence), plus 4 ring slots
    n = 16384
    b, _ = plan(L, 0, "fwd_sym_w8_k4_o1", n, 2)
    assert b == (64 + 4) * 16 * n


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("n", [1 << 20, (1 << 21) + 5, 1 << 22])
def test_pair_once_workspace_bounded(L, kind, n):
    # the quadratic workspace (8 n^2 / P) is gone: at most 1 GiB up to 2^22
    # for every pair-once variant and occupancy
    prefix = ("fwd_sym", "bwd_sym")[kind]
    for name in [v for v in names(L, kind) if v.startswith(prefix)]:
        for per_cu in (1, 2, 8, 32):
            b, timed = plan(L, kind, name, n, per_cu)
            assert 0 < b <= GiB, (name, per_cu, b)
            assert timed == 1, (name, per_cu)


def test_gate_size_band_and_cap(L):
    fwd = names(L, 0)
    n = 1 << 20
    # the one-launch kernels are not timed beyond their size band
    for name in [v for v in fwd if v.startswith(("fwd_la", "fwd_row"))]:
        b, timed = plan(L, 0, name, n, 4)
        assert b >= 0 and timed == 0, name
        assert plan(L, 0, name, 1 << 14, 4)[1] == 1, name
    # with 1 GiB free the cap is 256 MiB: the pair-once kernels (about
    # 0.9 GiB here) are skipped, the gathers (no workspace at this size)
    # are timed
    for name in fwd:
        b, timed = plan(L, 0, name, n, 2, free=GiB)
        if name.startswith("fwd_sym"):
            assert b > GiB // 4 and timed == 0, name
        elif name.startswith("fwd_b"):
            assert b <= GiB // 4 and timed == 1, name
    # the cap is a quarter of free memory: 0.86 GiB fits with 4 GiB free,
    # not with 3 GiB
    b, timed = plan(L, 0, "fwd_sym_w8_k4_o1", n, 2, free=4 * GiB)
    assert b == 53 * 16 * n + 32 * n and timed == 1
    assert plan(L, 0, "fwd_sym_w8_k4_o1", n, 2, free=3 * GiB)[1] == 0


def test_gate_cap_from_environment(L, monkeypatch):
    # NBODY_TUNE_WORKSPACE_CAP lowers the 2 GiB ceiling
    n = 1 << 20
    assert plan(L, 0, "fwd_sym_w8_k4_o1", n, 2)[1] == 1
    monkeypatch.setenv("NBODY_TUNE_WORKSPACE_CAP", str(512 << 20))
    assert plan(L, 0, "fwd_sym_w8_k4_o1", n, 2)[1] == 0
    assert plan(L, 0, "fwd_b64_k1_u8", n, 2)[1] == 1


def test_bad_arguments(L):
    t = ctypes.c_int(7)
    assert L.nbody_variant_plan(2, 0, 1000, 256, 2, GiB, ctypes.byref(t)) == -1 and t.value == 0
    assert L.nbody_variant_plan(0, 10 ** 6, 1000, 256, 2, GiB, None) == -1
    assert L.nbody_variant_plan(0, 0, -1, 256, 2, GiB, None) == -1
    assert L.nbody_variant_plan(0, 0, 1000, 0, 2, GiB, None) == -1
    assert L.nbody_variant_plan(1, 0, 1000, 256, 0, GiB, None) == -1
    assert L.nbody_variant_plan(0, 0, 0, 256, 2, GiB, None) == 0


@pytest.mark.parametrize("kind,prefix", [(0, "fwd_row"), (1, "bwd_row")])
def test_row_per_wave_variants_need_no_workspace(L, kind, prefix):
    # one wave per row: no partials, no counters at any size; timed only in
    # the launch-latency band (up to 2^16 bodies)
    rows = [v for v in names(L, kind) if v.startswith(prefix)]
    assert rows
    for name in rows:
        for n in (1, 1000, 1 << 16):
            assert plan(L, kind, name, n, 8) == (0, 1), (name, n)
        assert plan(L, kind, name, (1 << 16) + 1, 8) == (0, 0), name
        assert plan(L, kind, name, 1 << 20, 8) == (0, 0), name


@pytest.mark.parametrize("n", [20001, 70003, (1 << 20) + 7])
def test_running_sum_is_aligned(L, n, monkeypatch):
    # with the ring in several groups the float64 running sum (32 bytes per
    # particle, read as double4) follows the partials, whose area is rounded
    # up to 256 bytes so that it starts aligned also for odd n
    monkeypatch.setenv("NBODY_SYM_WORKSPACE", str(16 * n * 7))
    for name in ("fwd_sym_w8_k4_o1", "fwd_sym_w1_k2_r8"):
        b, _ = plan(L, 0, name, n, 2)
        assert b > 0 and (b - 32 * n) % 256 == 0 and b % 256 != 0, (name, n, b)


def test_step_split_blocks_hold_k_rows(L):
    # bwd_sym_s2_k2_*: two waves share a block of 2 x 64 rows, so the plan
    # has the blocks, ring offsets and fold slots of the one-wave two-row
    # blocks: at 16,384 bodies M = 128 blocks and 64 ring offsets, each
    # block a sequence of 2 + 64 x 2 = 130 tiles.  Eight two-wave
    # workgroups per CU in eight rounds give 128 chunks per block, sixteen
    # rounds all 130 (one tile each), as sixteen one-wave workgroups per CU
    # in eight rounds do.
    n = 16384
    assert plan(L, 1, "bwd_sym_s2_k2_r8", n, 8)[0] == (128 + 64) * 16 * n
    assert plan(L, 1, "bwd_sym_s2_k2_r16", n, 8)[0] == (130 + 64) * 16 * n
    assert plan(L, 1, "bwd_sym_w1_k2_r8", n, 16)[0] == (130 + 64) * 16 * n
    assert plan(L, 1, "bwd_sym_w1_k2_r16", n, 16)[0] == (130 + 64) * 16 * n


DEFAULTS_CHILD = r"""
import ctypes, json, sys
L = ctypes.CDLL(sys.argv[1])
L.nbody_variant_name.restype = ctypes.c_char_p
L.nbody_selected_variant.argtypes = [ctypes.c_int, ctypes.c_int64]
out = {}
for kind in (0, 1):
    for n in [int(a) for a in sys.argv[2:]]:
        v = L.nbody_selected_variant(kind, n)
        out[f"{kind}:{n}"] = L.nbody_variant_name(kind, v).decode()
print(json.dumps(out))
"""


def test_default_table(tmp_path):
    # the default kernel by size (no tuning cache, nothing forced), as the
    # header and the measured crossovers give it; host code only
    import json
    import subprocess
    import sys
    if not os.path.exists(B.LIBRARY):
        pytest.skip("libnbody.so not built (run __graft_entry__.build())")
    sizes = [1024, 2999, 3000, 3999, 4000, 4096, 4499, 4500, 4800, 5499, 5500, 5999, 6000, 8000, 9999, 10000, 11999,
             12000, 17999, 18000, 20000, 23999, 24000, 29999, 30000, 39999, 40000, 65536, 1 << 18, 1 << 20, 1 << 24,
             (1 << 24) + 1]
    env = dict(os.environ, NBODY_TUNE_CACHE=str(tmp_path / "none.json"))
    env.pop("NBODY_VARIANT", None)
    r = subprocess.run([sys.executable, "-c", DEFAULTS_CHILD, B.LIBRARY, *map(str, sizes)],
                       env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    got = json.loads(r.stdout.strip().splitlines()[-1])
    fwd = {1024: "fwd_row_k1", 2999: "fwd_row_k1", 3000: "fwd_row_k2", 4096: "fwd_row_k2",
           4499: "fwd_row_k2", 4500: "fwd_sym_w1_k2_o1", 5499: "fwd_sym_w1_k2_o1",
           5500: "fwd_sym_w1_k2_o1", 9999: "fwd_sym_w1_k2_o1",
           10000: "fwd_sym_w1_k2_r8", 12000: "fwd_sym_w1_k2_r8", 17999: "fwd_sym_w1_k2_r8",
           18000: "fwd_sym_w1_k4_r8", 20000: "fwd_sym_w1_k4_r8",
           39999: "fwd_sym_w1_k4_r8", 40000: "fwd_sym_w4_k4_r8", 65536: "fwd_sym_w4_k4_r8", 1 << 18: "fwd_sym_w4_k4_r8", 1 << 20: "fwd_sym_w8_k4_r8",
           1 << 24: "fwd_sym_w8_k4_r8", (1 << 24) + 1: "fwd_b64_k1_u8_f64sum"}
    # the adjoint (nbody_selected_variant's choice, with or without potential weights)
    bwd = {1024: "bwd_row_k1", 3000: "bwd_row_k1", 3999: "bwd_row_k2", 4000: "bwd_sym_s2_k2_r8",
           4096: "bwd_sym_s2_k2_r8", 4800: "bwd_sym_s2_k2_r8", 5999: "bwd_sym_s2_k2_r8",
           6000: "bwd_sym_s2_k2_r8", 9999: "bwd_sym_s2_k2_r8",
           11999: "bwd_sym_s2_k2_r8", 12000: "bwd_sym_w1_k2_r8", 20000: "bwd_sym_w1_k2_r8",
           23999: "bwd_sym_w1_k2_r8", 24000: "bwd_sym_w1_k2_r16", 29999: "bwd_sym_w1_k2_r16",
           30000: "bwd_sym_w1_k2_r8", 40000: "bwd_sym_w4_k2_r8", 65536: "bwd_sym_w4_k2_r8",
           1 << 18: "bwd_sym_w8_k2_r8", 1 << 24: "bwd_sym_w8_k2_r8",
           (1 << 24) + 1: "bwd_b256_k1_u8"}
    for kind, table in ((0, fwd), (1, bwd)):
        for n, name in table.items():
            assert got[f"{kind}:{n}"] == name, (kind, n, got[f"{kind}:{n}"])
