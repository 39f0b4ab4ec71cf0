"""bench.py's host-side contract, checked on the CPU: one GPU only, the
CPU-baseline record, and the traffic figure's source/variant key."""

import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_0904_3659_amd import inputs  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_cpu_baseline_record():
    n = 512
    w = inputs.Workload("plummer_n512_test", inputs.plummer_positions(n, (90, 0)),
                        inputs.equal_masses(n), 1e-4)
    rec = bench.cpu_baseline(w, budget_s=0.5)
    assert rec["kind"] == "oracle" and rec["unit"] == "pair-interactions/s"
    assert rec["value"] > 0 and rec["single_thread_value"] > 0 and rec["cores"] >= 1
    assert "seeded rows" in rec["sample"]


def test_traffic_figure_is_keyed_to_variant_and_sources():
    # another variant never picks up the recorded figure
    assert bench.read_traffic("fwd_b256_k1_u8") is None
    # the recorded file parses and names the kernel source hash it was taken on
    kv = {}
    for line in open(bench.TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    assert len(kv["kernel_source_sha"]) == 16 and kv["variant"].startswith("fwd_sym")
    assert float(kv["hbm_bytes_per_launch"]) > float(kv["algorithmic_bytes_per_launch"]) > 0
    if kv["kernel_source_sha"] == bench.forward_source_sha():
        assert bench.read_traffic(kv["variant"]) == float(kv["hbm_bytes_per_launch"])


def test_cpu_baseline_keeps_its_oracle_rows():
    # the rows the CPU-baseline leg computes are the ones the bench checks
    # the timed GPU result on: same row set, oracle values for each
    n = 600
    w = inputs.Workload("plummer_n600_test", inputs.plummer_positions(n, (90, 1)),
                        inputs.lognormal_masses(n, (90, 2)), 1e-4)
    rec, rows, ar, pr = bench.cpu_baseline(w, budget_s=0.2, keep=True)
    assert rows.size > 0 and ar.shape == (rows.size, 3) and pr.shape == (rows.size,)
    assert np.all(np.diff(rows) > 0)
    # checked against themselves: zero error; a planted error is reported
    e = bench.rel_errors(ar, pr, ar, pr)
    assert e["max"] == 0.0
    bad = ar.copy()
    bad[rows.size // 2, 1] *= 1 + 3e-4
    e = bench.rel_errors(bad, pr, ar, pr)
    assert 1e-4 < e["max"] and e["a_vec"] > 1e-4


def test_hw_flop_is_keyed_like_traffic():
    for kind in ("forward", "adjoint", "batched"):
        assert bench.hw_flop(kind, "no_such_variant") is None


def test_timed_calls_within_the_profiler_record():
    # the library keeps the last 256 calls' events: a long timed loop is
    # profiled on at most 256 calls, and a loop that records its own events
    # reads back the last 256
    class Torch:
        class cuda:
            @staticmethod
            def synchronize():
                pass

    class NB:
        def __init__(self):
            self.on, self.calls = False, 0

        def profile_enable(self, on):
            self.on, self.calls = on, 0

        def profile_read(self, launches=False):
            c = min(self.calls, 256)
            self.calls = 0
            return (0.5, 0.6, c, 1.0)

    nb = NB()

    def fn():
        if nb.on:
            nb.calls += 1

    for reps, inside in ((2000, False), (50, False), (300, True)):
        wall, main_ms, total_ms = bench.timed_calls(fn, reps, Torch, nb, events_in_timed_loop=inside)
        assert wall >= 0 and main_ms == 0.5 and total_ms == 0.6
