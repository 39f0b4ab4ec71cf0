"""The throughput convention reproduces the figures the paper prints
(tests/golden/paper_tables.json: Tables I and II, text of Sec. V-B)."""

import json
import os

import pytest

from paper_0904_3659_amd import metrics

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


@pytest.mark.parametrize("prog", ["gpu-no-unrolling", "simple-unrolling", "double-unrolling"])
def test_peak_gflops_from_table_ii(prog):
    # The paper's peak of each GPU program is its N = 100000 run of Table II:
    # N^2 interactions per step, 100 steps, 38 flop per interaction.
    n = GOLD["n"][-1]
    t = GOLD["hundred_steps_seconds"][prog][-1] / 100.0
    got = metrics.gflops(n * n, t, GOLD["flop_per_interaction"]["value"])
    assert got == pytest.approx(GOLD["peak_gflops"][prog], abs=1.0)


def test_speedup_ratios_table_ii():
    d = GOLD["hundred_steps_seconds"]
    for k, want in enumerate(GOLD["double_over_simple_speedup"]["values"]):
        assert d["simple-unrolling"][k] / d["double-unrolling"][k] == pytest.approx(want, abs=0.01)


def test_optimized_code_rate():
    o = GOLD["optimized_code"]
    got = metrics.gflops(o["n"] ** 2, o["seconds_one_evaluation_approx"])
    assert got == pytest.approx(o["max_gflops_approx"], rel=0.05)


def test_pair_counts():
    assert metrics.pairs(0) == 0 and metrics.pairs(1) == 0 and metrics.pairs(2) == 2
    assert metrics.pairs(1 << 20) == 1_099_510_579_200
    assert metrics.pairs_ensemble([8, 1, 0, 2048]) == 56 + 2048 * 2047
