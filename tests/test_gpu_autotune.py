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


CHILD_ENSEMBLE = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import numpy as np, torch
from oracle import reference as R
from paper_0904_3659_amd import inputs
from paper_0904_3659_amd import nbody as nb
ens = inputs.ensemble([5, 0, 300, 64, 1, 700, 129, 2048, 33], key=(93,))
dev = torch.device("cuda", 0)
x, m = torch.from_numpy(ens.x).to(dev), torch.from_numpy(ens.m).to(dev)
v = nb.autotune_batched(x, m, ens.offsets, ens.eps2)
a, p = nb.forces_batched(x, m, ens.offsets, ens.eps2)
nb.set_variant(nb.BATCHED, v)
a2, p2 = nb.forces_batched(x, m, ens.offsets, ens.eps2)
nb.set_variant(nb.BATCHED, -1)
ar, pr = R.forces_batched(ens.offsets, ens.x, ens.m, ens.eps2)
ok = pr > 0
err = float(np.max(np.abs(p.cpu().numpy() - pr)[ok] / pr[ok]))
print(json.dumps({"variant": v, "same": bool(torch.equal(a, a2) and torch.equal(p, p2)),
                  "err": err, "count": nb.variant_count(nb.BATCHED)}))
"""


def test_autotune_on_the_callers_ensemble(tmp_path):
    # the ensemble tuner records a choice for the mean system size; the next
    # batched call on that ensemble uses it, and it passes parity
    need_gpu()
    env = dict(os.environ, NBODY_TUNE_CACHE=str(tmp_path / "tune.json"))
    out = subprocess.run([sys.executable, "-c", CHILD_ENSEMBLE, ROOT], env=env, cwd=ROOT,
                         capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    r = json.loads(out.stdout.strip().splitlines()[-1])
    assert 0 <= r["variant"] < r["count"]
    assert r["same"]
    assert r["err"] <= 1e-4


CHILD_GRAPH = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import torch
from paper_0904_3659_amd import inputs
from paper_0904_3659_amd import nbody as nb
dev = torch.device("cuda", 0)
ens = inputs.ensemble([300, 17, 900, 64, 2000], key=(96,))
x, m = torch.from_numpy(ens.x).to(dev), torch.from_numpy(ens.m).to(dev)
a, p = torch.empty_like(x), torch.empty_like(m)
s = torch.cuda.Stream()
s.wait_stream(torch.cuda.current_stream())
with torch.cuda.stream(s):
    nb.forces_batched(x, m, ens.offsets, ens.eps2, out=(a, p))
s.synchronize()
ref = (a.clone(), p.clone())
g = torch.cuda.CUDAGraph()
with torch.cuda.graph(g, stream=s):
    nb.forces_batched(x, m, ens.offsets, ens.eps2, out=(a, p))
torch.cuda.synchronize()
same = []
for r in range(3):
    a.fill_(7.0 + r)
    p.fill_(7.0 + r)
    s2 = torch.cuda.Stream()
    with torch.cuda.stream(s2):
        nb.autotune_batched(x.clone(), m.clone(), ens.offsets, ens.eps2)
    s2.synchronize()
    g.replay()
    torch.cuda.synchronize()
    same.append(bool(torch.equal(a, ref[0]) and torch.equal(p, ref[1])))
print(json.dumps({"same": same}))
"""


def test_ensemble_timer_keeps_a_captured_plan():
    # a batched graph captured first replays bitwise after each run of the
    # ensemble variant timer on another stream: the timer's plans stay out of
    # the shared plan cache, so none of the graph's plan is evicted
    need_gpu()
    out = subprocess.run([sys.executable, "-c", CHILD_GRAPH, ROOT], cwd=ROOT, capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert json.loads(out.stdout.strip().splitlines()[-1])["same"] == [True, True, True]


CHILD_BIG = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import torch
from paper_0904_3659_amd import nbody as nb
dev = torch.device("cuda", 0)
torch.cuda.synchronize()
free0, total = torch.cuda.mem_get_info(dev)
nb.autotune(nb.FORWARD, [1 << 20])
torch.cuda.synchronize()
free1, _ = torch.cuda.mem_get_info(dev)
print(json.dumps({"free0": free0, "free1": free1,
                  "chosen": nb.variant_names(nb.FORWARD)[nb.selected_variant(nb.FORWARD, 1 << 20)]}))
"""


def test_autotune_at_a_million_keeps_workspace_under_the_cap(tmp_path):
    # Every variant the gate admits at 2^20 is timed (the one-launch kernels
    # are outside their size band); the timer gives back the workspace it
    # grew, so the device's free memory afterwards is within the timer's
    # cap (2 GiB) of what it was before.
    need_gpu()
    env = dict(os.environ, NBODY_TUNE_CACHE=str(tmp_path / "tune.json"))
    out = subprocess.run([sys.executable, "-c", CHILD_BIG, ROOT], env=env, capture_output=True,
                         text=True, timeout=280)
    assert out.returncode == 0, out.stderr[-2000:]
    r = json.loads(out.stdout.strip().splitlines()[-1])
    print(f"[autotune 2^20] chose {r['chosen']}, free before {r['free0']} after {r['free1']}",
          flush=True)
    assert r["free0"] - r["free1"] <= 2 << 30
    assert not r["chosen"].startswith(("fwd_la", "fwd_row"))
