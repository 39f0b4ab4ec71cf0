"""The variant timer: it records a choice per size bucket, writes and reads
the tuning cache, and every choice it can make is a parity-checked variant
(tests/test_gpu_*.py run every variant against the oracle)."""

import json
import os
import subprocess
import sys

import pytest

from tests.gpu_util import need_gpu

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import torch
from paper_0904_3659_amd import nbody as nb
nb.autotune(nb.FORWARD, [1536, 5000])
nb.autotune(nb.BACKWARD, [3000])
nb.autotune(nb.BATCHED, [300])
print(json.dumps({
    "fwd": [nb.selected_variant(nb.FORWARD, 1536), nb.selected_variant(nb.FORWARD, 5000)],
    "bwd": nb.selected_variant(nb.BACKWARD, 3000),
    "bat": nb.selected_variant(nb.BATCHED, 300),
}))
"""

CHILD_READ = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import torch
from paper_0904_3659_amd import nbody as nb
print(json.dumps({"fwd": nb.selected_variant(nb.FORWARD, 1536)}))
"""


def test_autotune_writes_and_reads_cache(tmp_path):
    need_gpu()
    cache = tmp_path / "tune.json"
    env = dict(os.environ, NBODY_TUNE_CACHE=str(cache))
    out = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    chosen = json.loads(out.stdout.strip().splitlines()[-1])
    data = json.loads(cache.read_text())
    kinds = {(e["kind"], e["bucket"]) for e in data["entries"]}
    assert {(0, 10), (0, 12), (1, 11), (2, 8)} <= kinds
    # a fresh process reads the cache back and picks the same variant
    out2 = subprocess.run([sys.executable, "-c", CHILD_READ, ROOT], env=env, capture_output=True,
                          text=True, timeout=300)
    assert out2.returncode == 0, out2.stderr[-2000:]
    assert json.loads(out2.stdout.strip().splitlines()[-1])["fwd"] == chosen["fwd"][0]
