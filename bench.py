"""Throughput of the exact softened all-pairs sum on one MI355X.

One step is one evaluation of Eq. (gravity) (a_i and p_i for every i, j != i)
on a 2^20-particle Plummer sphere with log-normal masses and eps^2 = 1e-6,
inputs resident in HBM.  The JSON line also reports the forward at 1,024
and 65,536 bodies, the adjoint (nbody_forces_backward on a 16,384-particle
Plummer sphere), the gradient of a 64-step checkpointed leap-frog run, the
batched ensemble (4,096 Plummer systems of 8..2048 particles in one
persistent launch, against one plain launch per system), the paper's three
unrolling programs at 100,000 bodies, 100-step stand-ins for the runs of
Sec. V-A, the roofline position of the forward kernel, and the FP64 CPU
reference timed on a bounded sample of the same workload on this host's
cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--only-forward]
       python bench.py --size-sweep               (pairs/s against N instead of the legs)
       python bench.py --only-leg adjoint|batched|latency (one leg alone, for profiling its kernel)
"""

from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-interactions/s & % FP32 VALU peak (38 flop/pair): fwd, adjoint, batched"
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "forward_plummer_n1048576_traffic.txt")
CSRC = os.path.join(ROOT, "paper_0904_3659_amd", "csrc")
# Files that define each leg's pair kernel; a counter summary is used only
# while their hash matches the one it was taken on.
KERNEL_SOURCES = {
    "forward": ("forward_sym.hip", "pair_once.hpp", "pair_term.hpp"),
    "adjoint": ("backward.hip", "pair_once.hpp"),
    "batched": ("batched.hip", "pair_once.hpp", "pair_term.hpp"),
}
COUNTER_FILES = {
    "forward": os.path.join(PROFILES, "forward_plummer_n1048576_valu_counters.txt"),
    "adjoint": os.path.join(PROFILES, "adjoint_plummer_n16384_valu_counters.txt"),
    "batched": os.path.join(PROFILES, "batched_ensemble4096_valu_counters.txt"),
}
# Tolerances of the float32 path against the FP64 oracle (max relative
# error on |a_i|, the vector a_i and p_i; adjoint: normwise).
TOL = 1e-4


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_sha(kind: str = "forward") -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def forward_source_sha() -> str:
    return source_sha("forward")


def read_keys(path: str) -> dict:
    """The 'key: value' lines of a profile summary (comment lines skipped)."""
    kv = {}
    if os.path.exists(path):
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


def keyed_figure(path: str, kind: str, variant: str, key: str):
    """Figure ``key`` of a committed profile summary, or None if the summary
    is absent, was taken on another variant, or on another source of the
    kernel."""
    kv = read_keys(path)
    if kv.get("kernel_source_sha") != source_sha(kind) or kv.get("variant") != variant:
        return None
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


def read_traffic(variant: str):
    """HBM bytes per evaluation of the forward pair kernel(s) from the
    committed counter summary (None if stale, see keyed_figure)."""
    return keyed_figure(TRAFFIC_FILE, "forward", variant, "hbm_bytes_per_launch")


def hw_flop(kind: str, variant: str):
    """FP32 operations per call counted by the hardware (SQ_INSTS_VALU_*_F32
    x 64 lanes, an FMA counting 2) from the committed counter summary, or
    None if stale."""
    return keyed_figure(COUNTER_FILES[kind], kind, variant, "hw_fp32_flop_per_call")


def frac_hw(kind: str, variant: str, kernel_ms: float, peak: float):
    f = hw_flop(kind, variant)
    return None if f is None else f / (kernel_ms * 1e-3) / (peak * 1e12)


def _sclk_path(torch, dev):
    """sysfs file with the driver's current graphics clock for `dev`."""
    try:
        pr = torch.cuda.get_device_properties(dev)
        path = (f"/sys/bus/pci/devices/{pr.pci_domain_id:04x}:{pr.pci_bus_id:02x}:"
                f"{pr.pci_device_id:02x}.0/pp_dpm_sclk")
        if os.path.exists(path):
            return path
    except (AttributeError, RuntimeError):
        pass
    cands = glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk")
    return cands[0] if len(cands) == 1 else None


class SclkSampler:
    """Samples the graphics clock the driver reports (the line of
    pp_dpm_sclk marked '*') every 10 ms on a host thread while the block
    runs; ``mean_mhz`` is their mean (None where the file is unreadable)."""

    def __init__(self, torch, dev):
        self.path = _sclk_path(torch, dev)
        self.samples = []
        self._stop = threading.Event()
        self._thread = None

    def _read(self):
        try:
            with open(self.path) as f:
                for line in f:
                    if "*" in line:
                        mhz = re.search(r"(\d+)\s*Mhz", line, re.I)
                        return int(mhz.group(1)) if mhz else None
        except OSError:
            return None
        return None

    def _run(self):
        while not self._stop.is_set():
            v = self._read()
            if v is not None:
                self.samples.append(v)
            self._stop.wait(0.01)

    def __enter__(self):
        if self.path:
            self._thread = threading.Thread(target=self._run, daemon=True)
            self._thread.start()
        return self

    def __exit__(self, *exc):
        if self._thread:
            self._stop.set()
            self._thread.join()

    @property
    def mean_mhz(self):
        return sum(self.samples) / len(self.samples) if self.samples else None


def warm_up(fn, torch, seconds: float = 0.1, min_calls: int = 3) -> None:
    """Call fn() (synchronising after each call) for at least `seconds` of
    wall time and `min_calls` calls, so that the GPU clock has come back up
    after host-side work before a timed loop."""
    t0 = time.perf_counter()
    k = 0
    while k < min_calls or time.perf_counter() - t0 < seconds:
        fn()
        torch.cuda.synchronize()
        k += 1


def timed_calls(fn, reps: int, torch, nb, events_in_timed_loop: bool = False):
    """Run fn() reps times between two synchronisations.

    Returns (wall seconds of that loop, mean pair-kernel ms, mean whole-call
    kernel ms).  The kernel figures come from the library's own HIP events,
    recorded on the stream it launches on (torch's current stream) around
    its pair kernel and after its last kernel.  With events_in_timed_loop
    they are recorded inside the timed loop itself (the 2^20 forward, where
    they cost nothing measurable); otherwise a second loop of min(reps, 256)
    calls records them (the library keeps the last 256 calls' events),
    since at small n the records add several microseconds per call to the
    loop they sit in."""
    torch.cuda.synchronize()
    if events_in_timed_loop:
        nb.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    recorded = reps
    if not events_in_timed_loop:
        recorded = min(reps, 256)
        nb.profile_enable(True)
        for _ in range(recorded):
            fn()
        torch.cuda.synchronize()
    main_ms, total_ms, calls, launches = nb.profile_read(launches=True)
    nb.profile_enable(False)
    assert calls == min(recorded, 256), (calls, recorded)
    timed_calls.launches = launches
    return wall, main_ms, total_ms


def cpu_baseline(w, budget_s: float = 12.0, keep: bool = False):
    """The FP64 oracle, as it stands, on a bounded row sample of the same
    workload: chunks of seeded rows until about ``budget_s`` seconds.

    With ``keep`` the oracle's rows are returned too, as (record, rows,
    a_rows, p_rows), so that the timed GPU result can be checked on them."""
    from oracle import reference as R
    from paper_0904_3659_amd import inputs
    n = w.n
    rows = inputs.check_rows(n, 65536, (3, 3))
    done, chunk, spent = 0, 256, 0.0
    a_parts, p_parts = [], []
    while done < rows.size and spent < budget_s:
        part = rows[done:done + chunk]
        t0 = time.perf_counter()
        ar, pr = R.forces_rows(w.x, w.m, w.eps2, part)
        spent += time.perf_counter() - t0
        if keep:
            a_parts.append(ar)
            p_parts.append(pr)
        done += part.size
        chunk = min(chunk * 2, 8192)
    pairs = done * (n - 1)
    threads = R.num_threads()
    # the same oracle on one thread (the paper's cpu-only program ran on one
    # core, Sec. V-A): the first rows of the same sample for about 3 s
    R.set_num_threads(1)
    try:
        done1, spent1 = 0, 0.0
        while done1 < rows.size and spent1 < 3.0:
            part = rows[done1:done1 + 64]
            t0 = time.perf_counter()
            R.forces_rows(w.x, w.m, w.eps2, part)
            spent1 += time.perf_counter() - t0
            done1 += part.size
    finally:
        R.set_num_threads(threads)
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")),
                         None)
    except OSError:
        pass
    rec = {"value": pairs / spent, "unit": "pair-interactions/s", "cores": threads,
           "kind": "oracle", "cpu_model": model, "host_cpus": os.cpu_count(),
           "sample": f"{done} seeded rows x {n - 1} j of {w.name}, FP64, {spent:.2f} s",
           "single_thread_value": done1 * (n - 1) / spent1,
           "single_thread_sample": f"first {done1} of the same rows, 1 thread, {spent1:.2f} s"}
    if not keep:
        return rec
    return rec, rows[:done], np.concatenate(a_parts), np.concatenate(p_parts)


def rel_errors(a, p, a_ref, p_ref) -> dict:
    """Max relative errors of (a, p) against float64 reference rows:
    |.|a|-|a_ref|.|/|a_ref|, |a - a_ref|/|a_ref| and |p - p_ref|/p_ref."""
    a = np.asarray(a, np.float64)
    na = np.linalg.norm(a_ref, axis=1)
    ok = na > 0
    mag = np.abs(np.linalg.norm(a, axis=1) - na)[ok] / na[ok]
    vec = np.linalg.norm(a - a_ref, axis=1)[ok] / na[ok]
    out = {"a_mag": float(mag.max()) if mag.size else 0.0,
           "a_vec": float(vec.max()) if vec.size else 0.0}
    if p is not None:
        pos = p_ref > 0
        pe = np.abs(np.asarray(p, np.float64) - p_ref)[pos] / p_ref[pos]
        out["p"] = float(pe.max()) if pe.size else 0.0
    out["max"] = max(out.values())
    return out


def oracle_checks(held: dict) -> dict:
    """Compare the results the timed legs left behind (host copies in
    ``held``) with the FP64 oracle.  Runs inside the CPU-baseline leg, the
    only part of this script that calls the oracle."""
    from oracle import reference as R
    checks = {}
    if "sizes" in held:
        for name, (w, a, p) in held["sizes"].items():
            if w.n <= 4096:
                ar, pr = R.forces(w.x, w.m, w.eps2)
                checks[name] = rel_errors(a, p, ar, pr)
            else:
                rows = np.arange(0, w.n, max(1, w.n // 1024))
                ar, pr = R.forces_rows(w.x, w.m, w.eps2, rows)
                checks[name] = rel_errors(a[rows], p[rows], ar, pr)
                checks[name]["rows"] = int(rows.size)
    for key in ("adjoint", "adjoint_1k"):
        if key in held:
            wa, gx, gm = held[key]
            rx, rm = R.forces_vjp(wa.x, wa.m, wa.eps2, wa.extra["w"], wa.extra["v"])
            ex = float(np.abs(gx - rx).max() / np.abs(rx).max())
            em = float(np.abs(gm - rm).max() / np.abs(rm).max())
            checks[wa.name] = {"grad_x_normwise": ex, "grad_m_normwise": em, "max": max(ex, em)}
    if "batched" in held:
        ens, a, p = held["batched"]
        sizes = ens.sizes()
        g = np.random.default_rng(11)
        pick = np.unique(np.concatenate([
            g.choice(ens.num_systems, min(192, ens.num_systems), replace=False),
            [int(np.argmax(sizes)), int(np.argmin(np.where(sizes > 1, sizes, 1 << 30)))]]))
        worst = {"a_mag": 0.0, "a_vec": 0.0, "p": 0.0, "max": 0.0}
        for s in pick:
            lo, hi = int(ens.offsets[s]), int(ens.offsets[s + 1])
            if hi - lo < 2:
                continue
            ar, pr = R.forces(ens.x[lo:hi], ens.m[lo:hi], ens.eps2)
            e = rel_errors(a[lo:hi], p[lo:hi], ar, pr)
            worst = {k: max(worst[k], e[k]) for k in worst}
        worst["systems_checked"] = int(pick.size)
        checks[ens.name] = worst
    if "unroll" in held:
        xu, mu, e2, res = held["unroll"]
        rows = np.arange(0, xu.shape[0], max(1, xu.shape[0] // 512))
        ar, pr = R.forces_rows(xu, mu, e2, rows)
        for label, (a, p) in res.items():
            checks["unroll_study_n100000 " + label] = rel_errors(a[rows], p[rows], ar, pr)
    return checks


def graph_plain_ms(plain, ab, pb, torch):
    """The per-system launches captured once in a HIP graph and replayed: a
    stronger baseline than launching them from Python.  The replay must
    reproduce the eager result bitwise, else None is reported."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plain()                      # grows the library's workspace for s
    s.synchronize()
    ref_a, ref_p = ab.clone(), pb.clone()
    g = torch.cuda.CUDAGraph()
    try:
        with torch.cuda.graph(g, stream=s):
            plain()
    except RuntimeError as e:
        log(f"graph capture failed: {e}")
        return None
    torch.cuda.synchronize()
    ab.zero_()
    pb.zero_()
    g.replay()
    torch.cuda.synchronize()
    if not (torch.equal(ab, ref_a) and torch.equal(pb, ref_p)):
        log("graph replay differs from the eager launches")
        return None
    t0 = time.perf_counter()
    for _ in range(5):
        g.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / 5
    ok = torch.equal(ab, ref_a) and torch.equal(pb, ref_p)
    del g
    return ms if ok else None


SWEEP_SIZES = (1024, 2048, 4096, 7500, 10000, 16384, 18000, 32768, 65536, 100000, 262144,
               1048576)
SWEEP_PROGRAMS = (("gpu-no-unrolling", "fwd_b256_k1_u1"), ("simple-unrolling", "fwd_b256_k4_u1"),
                  ("double-unrolling", "fwd_b256_k4_u4"), ("default", None))


def size_sweep(nb, torch, dev, inputs, metrics):
    """pairs/s of the paper's three GPU programs (Sec. IV, Figs. no-u, sim-u,
    double-u as (K, U) = (1, 1), (4, 1), (4, 4) gathers) and of the default
    variant against N: Plummer spheres, masses 1/N, eps2 = 1e-4."""
    names = nb.variant_names(nb.FORWARD)
    table = {}
    for n in SWEEP_SIZES:
        x = torch.from_numpy(inputs.plummer_positions(n, (8, n))).to(dev)
        m = torch.from_numpy(inputs.equal_masses(n)).to(dev)
        reps = max(3, min(50, int(4e11 / (n * n))))
        row = {}
        for label, vname in SWEEP_PROGRAMS:
            nb.set_variant(nb.FORWARD, names.index(vname) if vname else -1)
            f = lambda: nb.forces(x, m, 1e-4)
            warm_up(f, torch, 0.05, 1)
            wall, _, _ = timed_calls(f, reps, torch, nb)
            row[label] = {"variant": vname or names[nb.selected_variant(nb.FORWARD, n)],
                          "ms": wall * 1e3 / reps,
                          "pairs_per_s": metrics.pairs(n) / (wall / reps)}
        nb.set_variant(nb.FORWARD, -1)
        table[str(n)] = row
        log(f"size sweep n={n}: " + ", ".join(f"{k} {v['pairs_per_s']:.3e}" for k, v in row.items()))
    return table


def adjoint_leg(nb, torch, dev, inputs, metrics, peak, held=None):
    """The adjoint at N = 16,384 with upstream weights on a and p: (its
    workload, the JSON record).  With ``held`` a host copy of the result is
    kept there for the oracle check."""
    log("adjoint leg")
    wa = inputs.adjoint_16k()
    xa = torch.from_numpy(wa.x).to(dev)
    ma = torch.from_numpy(wa.m).to(dev)
    ga = torch.from_numpy(wa.extra["w"]).to(dev)
    gp = torch.from_numpy(wa.extra["v"]).to(dev)
    gx = torch.empty_like(xa)
    gm = torch.empty_like(ma)
    bwd = lambda: nb.forces_backward(xa, ma, wa.eps2, ga, gp, out=(gx, gm))
    warm_up(bwd, torch)
    wall_a, ka, ca = timed_calls(bwd, 50, torch, nb)
    variant = nb.variant_names(nb.BACKWARD)[nb.selected_variant(nb.BACKWARD, wa.n)]
    pa = metrics.pairs(wa.n)
    ev = metrics.evaluated_pairs(pa, variant)
    own = metrics.ADJOINT_FLOP_PER_PAIR
    rec = {
        "workload": wa.name, "ms_per_call": wall_a * 1e3 / 50, "pairs_per_s": pa / (wall_a / 50),
        "pair_kernel_ms": ka, "kernels_ms": ca,
        "pairs_per_s_kernels": pa / (ca * 1e-3),
        "evaluated_pairs": ev,
        # fractions of the FP32 peak on the interactions the pair kernel
        # evaluates, at the adjoint's own 68 flop and at the forward's 38
        "frac_fp32_peak_own_flop": ev * own / (ka * 1e-3) / (peak * 1e12),
        "frac_fp32_peak_38flop": ev * 38 / (ka * 1e-3) / (peak * 1e12),
        "frac_hw": frac_hw("adjoint", variant, ka, peak),
        "own_flop_per_pair": own,
        "variant": variant,
    }
    if held is not None:
        torch.cuda.synchronize()
        held["adjoint"] = (wa, gx.cpu().numpy().astype(np.float64),
                           gm.cpu().numpy().astype(np.float64))
    log(f"adjoint {ka:.3f} ms pair kernel, {ca:.3f} ms with its reduction")
    return wa, rec


def latency_leg(nb, torch, dev, inputs, held=None, reps: int = 2000):
    """Forward and adjoint at N = 1,024, where a call costs launch latency:
    microseconds per call from Python over `reps` back-to-back calls with
    preallocated outputs, and the pair kernel's own duration from the
    library's events.  With ``held`` the adjoint's result is kept for the
    oracle check."""
    log("latency leg (N = 1,024)")
    w = inputs.adjoint_16k(1024)
    x = torch.from_numpy(w.x).to(dev)
    m = torch.from_numpy(w.m).to(dev)
    ga = torch.from_numpy(w.extra["w"]).to(dev)
    gp = torch.from_numpy(w.extra["v"]).to(dev)
    a, p = torch.empty_like(x), torch.empty_like(m)
    gx, gm = torch.empty_like(x), torch.empty_like(m)
    rec = {"workload": w.name}
    for kind, fn, k in (("forward", lambda: nb.forces(x, m, w.eps2, out=(a, p)), nb.FORWARD),
                        ("adjoint", lambda: nb.forces_backward(x, m, w.eps2, ga, gp, out=(gx, gm)),
                         nb.BACKWARD)):
        warm_up(fn, torch)
        wall, km, cm = timed_calls(fn, reps, torch, nb)
        rec[kind] = {"us_per_call": wall * 1e6 / reps, "pair_kernel_us": km * 1e3,
                     "kernels_us": cm * 1e3,
                     "variant": nb.variant_names(k)[nb.selected_variant(k, w.n)]}
        log(f"{kind} N = 1,024: {wall * 1e6 / reps:.2f} us per call, kernel {km * 1e3:.2f} us")
    # the same forward through a prepared call (tensors checked once)
    bound = nb.BoundForces(x, m, w.eps2, a, p)
    warm_up(bound, torch)
    wall, _, _ = timed_calls(bound, reps, torch, nb)
    rec["forward"]["us_per_call_bound"] = wall * 1e6 / reps
    log(f"forward N = 1,024 through BoundForces: {wall * 1e6 / reps:.2f} us per call")
    if held is not None:
        torch.cuda.synchronize()
        held["adjoint_1k"] = (w, gx.cpu().numpy().astype(np.float64),
                              gm.cpu().numpy().astype(np.float64))
    return rec


def batched_leg(nb, torch, dev, inputs, metrics, peak, comparisons: bool = True, held=None):
    """The 4,096-system ensemble in one persistent launch, tuned on the
    ensemble first; with ``comparisons`` also the plain per-system launches
    and their HIP-graph replay."""
    log("batched leg")
    ens = inputs.ensemble_4096()
    xb = torch.from_numpy(ens.x).to(dev)
    mb = torch.from_numpy(ens.m).to(dev)
    ab = torch.empty_like(xb)
    pb = torch.empty_like(mb)
    t0 = time.perf_counter()
    nb.forces_batched(xb, mb, ens.offsets, ens.eps2, out=(ab, pb))
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    bnames = nb.variant_names(nb.BATCHED)
    mean_n = int(ens.offsets[-1]) // ens.num_systems
    default_b = bnames[nb.selected_variant(nb.BATCHED, mean_n)]
    # the persistent launch is tuned on this ensemble: every batched
    # variant timed, the fastest kept for its mean system size
    t0 = time.perf_counter()
    tuned_b = nb.autotune_batched(xb, mb, ens.offsets, ens.eps2) if comparisons else None
    tune_s = time.perf_counter() - t0
    bat = lambda: nb.forces_batched(xb, mb, ens.offsets, ens.eps2, out=(ab, pb))
    warm_up(bat, torch)
    wall_b, kbm, kb = timed_calls(bat, 10, torch, nb)
    variant = bnames[nb.selected_variant(nb.BATCHED, mean_n)]
    pb_pairs = metrics.pairs_ensemble(ens.sizes())
    ev = metrics.evaluated_pairs(pb_pairs, variant)
    rec = {
        "workload": ens.name, "systems": ens.num_systems, "particles": int(ens.offsets[-1]),
        "pairs": pb_pairs, "evaluated_pairs": ev,
        "persistent_ms": kb, "persistent_pair_kernel_ms": kbm,
        "ms_per_call": wall_b * 1e3 / 10, "pairs_per_s": pb_pairs / (kb * 1e-3),
        "frac_fp32_peak_38flop": ev * 38 / (kbm * 1e-3) / (peak * 1e12),
        "frac_hw": frac_hw("batched", variant, kbm, peak),
        "plan_build_s": plan_s,
        "variant": variant,
        "default_variant": default_b,
    }
    if held is not None:
        torch.cuda.synchronize()
        held["batched"] = (ens, ab.cpu().numpy().astype(np.float64),
                           pb.cpu().numpy().astype(np.float64))
    if not comparisons:
        return rec
    views = [(xb[lo:hi], mb[lo:hi], ab[lo:hi], pb[lo:hi])
             for lo, hi in zip(ens.offsets[:-1], ens.offsets[1:]) if hi > lo]

    def plain():
        for xs, ms, as_, ps in views:
            nb.forces(xs, ms, ens.eps2, out=(as_, ps))

    plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain()
    torch.cuda.synchronize()
    wall_plain = time.perf_counter() - t0
    graph_ms = graph_plain_ms(plain, ab, pb, torch)
    rec.update({
        "plain_launches_ms": wall_plain * 1e3,
        "speedup_vs_plain": wall_plain * 1e3 / kb,
        "graph_plain_launches_ms": graph_ms,
        "speedup_vs_graph": (graph_ms / kb) if graph_ms else None,
        "autotuned": True, "autotune_s": tune_s, "tuned_variant": bnames[tuned_b],
    })
    log(f"batched {kb:.3f} ms vs plain {wall_plain * 1e3:.1f} ms")
    return rec


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU reference timing")
    ap.add_argument("--only-forward", action="store_true", help="skip adjoint and batched legs")
    ap.add_argument("--size-sweep", action="store_true",
                    help="instead of the legs, time the paper's three unrolling programs and "
                         "the default variant over a range of N (pairs/s vs N)")
    ap.add_argument("--only-leg", choices=("adjoint", "batched", "latency"),
                    help="run only this leg and print its record (for profiling its kernel; "
                         "the batched leg then skips the tuner and the per-system launches)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="first run one plain device-to-device copy of BYTES (the reference "
                         "kernel that scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the path runs on a single MI355X and "
              "sharding over several GPUs is not built; run with --gpus 1.", file=sys.stderr)
        return 2

    import torch
    from paper_0904_3659_amd import inputs, metrics
    from paper_0904_3659_amd import nbody as nb

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        return 2
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.size_sweep:
        print(json.dumps({"size_sweep": size_sweep(nb, torch, dev, inputs, metrics),
                          "unit": "pair-interactions/s", "data": "synthetic"}), flush=True)
        return 0

    if args.only_leg:
        peak = metrics.MI355X_FP32_VECTOR_TFLOPS
        if args.only_leg == "adjoint":
            rec = adjoint_leg(nb, torch, dev, inputs, metrics, peak)[1]
        elif args.only_leg == "latency":
            rec = latency_leg(nb, torch, dev, inputs)
        else:
            rec = batched_leg(nb, torch, dev, inputs, metrics, peak, comparisons=False)
        print(json.dumps({args.only_leg: rec}), flush=True)
        return 0

    if args.copy_calibration:
        src = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {src.numel() * 4} bytes copied")
        del src, dst

    # ---------------------------------------------------------- forward, 2^20
    log("generating plummer_n1048576 inputs")
    w = inputs.plummer_1m_lognormal()
    x = torch.from_numpy(w.x).to(dev)
    m = torch.from_numpy(w.m).to(dev)
    a = torch.empty((w.n, 3), device=dev)
    p = torch.empty((w.n,), device=dev)
    fwd = lambda: nb.forces(x, m, w.eps2, out=(a, p))
    log(f"forward warmup x{args.warmup}")
    for _ in range(args.warmup):
        fwd()
    torch.cuda.synchronize()
    log(f"forward timed x{args.steps}")
    with SclkSampler(torch, dev) as clk:
        wall, kern_ms, call_ms = timed_calls(fwd, args.steps, torch, nb, events_in_timed_loop=True)
    launches = timed_calls.launches
    # host copy of the last timed result, checked against the oracle below
    a_last = a.cpu().numpy().astype(np.float64)
    p_last = p.cpu().numpy().astype(np.float64)
    pairs = metrics.pairs(w.n)
    ms_step = wall * 1e3 / args.steps
    value = pairs / (wall / args.steps)
    peak = metrics.MI355X_FP32_VECTOR_TFLOPS
    variant = nb.variant_names(nb.FORWARD)[nb.selected_variant(nb.FORWARD, w.n)]
    evaluated = metrics.evaluated_pairs(pairs, variant)
    # algorithmic rate of the pair kernel: 38 flop per interaction it evaluates
    achieved = evaluated * metrics.FLOP_PER_PAIR / (kern_ms * 1e-3) / 1e12
    traffic = read_traffic(variant)
    log(f"forward {ms_step:.2f} ms/step, {value:.3e} pairs/s, kernel {kern_ms:.2f} ms")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "eps2": w.eps2, "pairs_per_step": pairs,
                   "variant": variant},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": variant, "kernel_ms": kern_ms, "call_kernels_ms": call_ms,
                     # the pair kernel runs as several launches (ring groups):
                     # kernel_ms is their sum per evaluation
                     "kernel_launches_per_call": launches,
                     "kernel_ms_per_launch": kern_ms / launches if launches else None,
                     "flop_per_pair": metrics.FLOP_PER_PAIR,
                     "evaluated_pairs": evaluated,
                     # FP32 operations the hardware counted for this kernel
                     # (committed rocprofv3 counters, same source and variant)
                     "frac_hw": frac_hw("forward", variant, kern_ms, peak),
                     # the rate at which ordered-pair terms are delivered, priced
                     # at 38 flop each: what an every-ordered-pair kernel would
                     # need to reach the same time; exceeds 1 for pair-once
                     "frac_effective_ordered": pairs * metrics.FLOP_PER_PAIR / (kern_ms * 1e-3)
                                               / (peak * 1e12),
                     # the peak scaled to the clock the driver reported while timing
                     "sclk_mhz_observed": clk.mean_mhz,
                     "frac_at_observed_sclk": (achieved / (peak * clk.mean_mhz / 2400.0)
                                               if clk.mean_mhz else None)},
    }
    held = {}

    # ---------------------------------------------------------- other sizes
    if not args.only_forward:
        sizes = {}
        held["sizes"] = {}
        for make in (inputs.plummer_1k, inputs.plummer_64k, inputs.cube_64k):
            ws = make()
            xs, ms_ = torch.from_numpy(ws.x).to(dev), torch.from_numpy(ws.m).to(dev)
            as_, ps = torch.empty_like(xs), torch.empty_like(ms_)
            f = lambda: nb.forces(xs, ms_, ws.eps2, out=(as_, ps))
            warm_up(f, torch)
            reps = 50 if ws.n <= 4096 else 20
            wl, km, cm = timed_calls(f, reps, torch, nb)
            pr = metrics.pairs(ws.n)
            vname = nb.variant_names(nb.FORWARD)[nb.selected_variant(nb.FORWARD, ws.n)]
            ev = metrics.evaluated_pairs(pr, vname)
            sizes[ws.name] = {"ms_per_call": wl * 1e3 / reps, "kernels_ms": cm, "pair_kernel_ms": km,
                              "pairs_per_s": pr / (wl / reps),
                              "frac_fp32_peak_38flop_kernel": ev * 38 / (km * 1e-3) / (peak * 1e12),
                              "variant": vname}
            if ws.n <= 4096:
                # latency-bound: the time per call is the figure of merit
                sizes[ws.name]["latency_us_per_call"] = wl * 1e6 / reps
            held["sizes"][ws.name] = (ws, as_.cpu().numpy().astype(np.float64),
                                      ps.cpu().numpy().astype(np.float64))
            log(f"forward {ws.name}: {wl * 1e3 / reps:.4f} ms/call")
        out["forward_other_sizes"] = sizes
        # ------------------------------------------ latency, forward + adjoint
        out["latency_n1024"] = latency_leg(nb, torch, dev, inputs, held)

    if not args.only_forward:
        # ------------------------------------------------------ adjoint, 16k
        wa, out["adjoint"] = adjoint_leg(nb, torch, dev, inputs, metrics, peak, held)

        # ------------------------------------------- leap-frog with checkpoints
        log("leap-frog leg")
        x0 = torch.from_numpy(wa.x).to(dev).requires_grad_(True)
        v0 = torch.from_numpy(wa.extra["v0"]).to(dev).requires_grad_(True)
        mm = torch.from_numpy(wa.m).to(dev).requires_grad_(True)
        u = torch.from_numpy(wa.extra["u"]).to(dev)

        def lf(graphs):
            xT, _ = nb.leapfrog(x0, v0, mm, wa.eps2, 1e-3, 64, checkpoint_every=8, graphs=graphs)
            torch.autograd.grad((xT * u).sum(), (x0, v0, mm))

        lf_times = {}
        for graphs in (False, True):
            lf(graphs)                   # the first graphs call captures them
        # both paths in alternation, best of five rounds of three calls, so
        # that a drift of the clock during the leg favours neither
        for _ in range(5):
            for graphs in (False, True):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(3):
                    lf(graphs)
                torch.cuda.synchronize()
                t = (time.perf_counter() - t0) / 3
                lf_times[graphs] = min(lf_times.get(graphs, t), t)
        from paper_0904_3659_amd import leapfrog as LF
        lf_default = wa.n <= LF.GRAPHS_MAX_N     # what graphs=None takes
        lf_s = lf_times[lf_default]
        # forward: a(x0) and one force evaluation per step; reverse: the
        # positions inside every segment but the last (whose positions the
        # forward pass kept) are recomputed from its checkpoint (x, v, a),
        # 8 - 2 evaluations each (the end is the next checkpoint, the step
        # before it needs only a kick and a drift): 7 x 6 evaluations
        f_evals = 1 + 64 + 7 * 6
        out["leapfrog_grad"] = {"workload": wa.name + "_64steps_dt1e-3_ckpt8", "seconds": lf_s,
                                "graphs_by_default": lf_default,
                                "seconds_with_graphs": lf_times[True],
                                "seconds_without_graphs": lf_times[False],
                                "force_evals": f_evals, "vjp_evals": 64,
                                "pairs_per_s": (f_evals + 64) * metrics.pairs(wa.n) / lf_s}
        log(f"leap-frog gradient {lf_s * 1e3:.1f} ms")

        # ------------------------------------------------------ batched
        out["batched"] = batched_leg(nb, torch, dev, inputs, metrics, peak, held=held)

    if not args.only_forward:
        # -------------------- the paper's unrolling programs (Sec. IV, Fig. p)
        log("unroll study")
        wu = inputs.paper_experiment_set(3)
        xu, mu = torch.from_numpy(wu[1]).to(dev), torch.from_numpy(wu[3]).to(dev)
        names = nb.variant_names(nb.FORWARD)
        study, res = {}, {}
        for label, vname in (("gpu-no-unrolling (K=1, U=1)", "fwd_b256_k1_u1"),
                             ("simple-unrolling (K=4, U=1)", "fwd_b256_k4_u1"),
                             ("double-unrolling (K=4, U=4)", "fwd_b256_k4_u4"),
                             ("default", None)):
            nb.set_variant(nb.FORWARD, names.index(vname) if vname else -1)
            au, pu = torch.empty_like(xu), torch.empty_like(mu)
            f = lambda: nb.forces(xu, mu, wu[4], out=(au, pu))
            warm_up(f, torch, 0.1, 1)
            wl, km, cm = timed_calls(f, 10, torch, nb)
            pr = metrics.pairs(xu.shape[0]) / (wl / 10)
            study[label] = {"variant": vname or names[nb.selected_variant(nb.FORWARD, xu.shape[0])],
                            "ms": wl * 100, "pairs_per_s": pr,
                            "gflops_38": pr * 38 / 1e9}
            res[label] = (au.cpu().numpy().astype(np.float64), pu.cpu().numpy().astype(np.float64))
        nb.set_variant(nb.FORWARD, -1)
        out["unroll_study_n100000"] = study
        held["unroll"] = (wu[1], wu[3], wu[4], res)

        # ---------------- Experiment 2 of the paper: 100 leap-frog steps
        log("paper experiment 2 stand-ins")
        from paper_0904_3659_amd import leapfrog as LF
        paper_s = {"three_figure_eight_galaxies": 0.68, "four_figure_eight_galaxies": 0.92,
                   "cart_wheel_galaxy": 2.43, "random_100000_body": 55.0}
        exp2 = {}
        for k in range(4):
            name, x0, v0, m0, e2, dt = inputs.paper_experiment_set(k)
            xt, vt, mt = (torch.from_numpy(t).to(dev) for t in (x0, v0, m0))
            LF.integrate(xt, vt, mt, e2, dt, 2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            LF.integrate(xt, vt, mt, e2, dt, 100)
            torch.cuda.synchronize()
            secs = time.perf_counter() - t0
            exp2[name] = {"n": int(x0.shape[0]), "dt": dt, "eps2": e2, "seconds_100_steps": secs,
                          "paper_double_unrolling_seconds": paper_s[name],
                          "speedup_vs_paper": paper_s[name] / secs}
        out["paper_experiment2_standins"] = exp2

    ok = True
    if not args.no_cpu:
        # ------------------------------------ CPU baseline and oracle checks
        log("cpu baseline (FP64 oracle, bounded sample) and oracle checks")
        rec, rows, ar, pr = cpu_baseline(w, keep=True)
        out["cpu_baseline"] = rec
        err = rel_errors(a_last[rows], p_last[rows], ar, pr)
        err["rows"] = int(rows.size)
        out["max_rel_err"] = err["max"]
        checks = {w.name + " (timed result)": err}
        checks.update(oracle_checks(held))
        out["oracle_checks"] = checks
        out["oracle_tolerance"] = TOL
        bad = {k: v["max"] for k, v in checks.items() if v["max"] > TOL}
        if bad:
            log(f"results differ from the FP64 oracle beyond {TOL}: {bad}")
            ok = False
    else:
        out["cpu_baseline"] = None
        out["max_rel_err"] = None

    print(json.dumps(out), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
