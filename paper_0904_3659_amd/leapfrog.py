"""Device-resident leap-frog integration and its checkpointed adjoint.

The integrator is the kick-drift-kick scheme of Eqs. (1)-(3) with the
seven-step algorithm of Sec. III: one force evaluation per step, reused by
the next step's first kick.  The paper's a (Eq. (gravity)) points away from
the attracting body, so the physical acceleration is g = -a and a kick is
v += (dt/2) g = v - (dt/2) a.  A run of steps is one library call
(``nbody_leapfrog``): per step the force kernel, then a reduction whose
epilogue applies the step's end kick, the next step's start kick and its
drift; the reverse sweep over a segment is one ``nbody_leapfrog_adjoint``
call in the same way.  Tensors only hold device memory.

Reverse sweep for a loss on the final state.  With adjoints (lx, lv) of the
step output (x_t, v_t), stepping back over step t-1 is
    lx += -(dt/2) VJP_a(x_t)[lv]        (end kick of step t-1)
    lv += dt lx                         (drift: lv is now the half-step adjoint)
    lx += -(dt/2) VJP_a(x_{t-1})[lv]    (start kick of step t-1)
and the start kick of step t-1 and the end kick of step t-2 meet at the
same positions with the same weight, so they are applied as one product with
factor dt.  Masses collect the same products' dL/dm parts.

Checkpointing: the forward pass keeps (x, v) every ``checkpoint_every``
steps; the reverse pass recomputes the positions inside each segment from
its checkpoint before sweeping it.  A k-step segment needs k - 2 force
evaluations for that: its end position is the next checkpoint, and the
position before the end takes only the start kick and drift of the last
step, so the forces at those two positions are never recomputed.  The
kernels are deterministic, so the recomputed positions and hence the
gradients are bitwise equal to those of a run that stores every position.

HIP graphs: a k-step segment (2k + 1 launches), the recomputation of a
segment's positions and the reverse sweep over an interior segment are each
captured once as a HIP graph on fixed device buffers and replayed once per
segment, instead of issuing every launch from the host.  The graphs run the
same kernels on the same data, so results are bitwise equal to the eager
path (``graphs=False``).  In the reverse pass the recomputation of the
next segment's positions (into the other of two position buffers) runs on
a second stream while the current segment is swept, so each fills the
other's partial-sum folds and the drain at the end of each pair kernel.
"""

from __future__ import annotations

import threading

import torch

from . import nbody as _nb


def _last_start(steps: int, k: int) -> int:
    """First step of the last checkpoint segment."""
    return ((steps - 1) // k) * k


def integrate(x0, v0, m, eps2, dt, steps, *, keep_every: int | None = None):
    """Run ``steps`` KDK steps from (x0, v0).

    Returns (x_T, v_T, saved).  With ``keep_every=k``, ``saved[t]`` is a
    copy of (x, v, a) at every step t that is a multiple of k and at
    t = steps, and ``saved["tail"]`` holds the positions of the last
    segment ([steps - last + 1, n, 3]: x at its first step .. x_T), which
    the reverse sweep then need not recompute.  Without it ``saved`` is {}.
    """
    x = x0.detach().clone().contiguous()
    v = v0.detach().clone().contiguous()
    a, _ = _nb.forces(x, m, eps2, potential=False)
    saved = {}
    if not keep_every:
        _nb.leapfrog_(x, v, a, m, eps2, dt, steps)
        return x, v, saved
    last = _last_start(steps, keep_every) if steps > 0 else None
    for s0 in range(0, steps, keep_every):
        count = min(keep_every, steps - s0)
        saved[s0] = (x.clone(), v.clone(), a.clone())
        if s0 == last:
            tail = torch.empty((count + 1,) + tuple(x.shape), dtype=x.dtype, device=x.device)
            tail[0].copy_(x)
            _nb.leapfrog_(x, v, a, m, eps2, dt, count, x_hist=tail[1:])
            saved["tail"] = tail
        else:
            _nb.leapfrog_(x, v, a, m, eps2, dt, count)
    saved[steps] = (x.clone(), v.clone(), a.clone())
    return x, v, saved


def _positions(xs, vs, a0, x_end, m, eps2, dt, count):
    """Positions [count + 1, n, 3] after 0..count steps from (xs, vs) with
    a0 = a(xs), given x_end, the positions after the last step: count - 2
    full steps, then the start kick and drift of the next one (bitwise the
    fused step, as nbody_leapfrog is bitwise its composed calls)."""
    pos = torch.empty((count + 1,) + tuple(xs.shape), dtype=xs.dtype, device=xs.device)
    pos[0].copy_(xs)
    pos[count].copy_(x_end)
    if count >= 2:
        x, v, a = xs.clone(), vs.clone(), a0.clone()
        if count > 2:
            _nb.leapfrog_(x, v, a, m, eps2, dt, count - 2, x_hist=pos[1:count - 1])
        pos[count - 1].copy_(x)
        _nb.kick_drift_(pos[count - 1], v, a, -0.5 * dt, dt)
    return pos


def _flags(s0: int, last: int, final_kick: bool) -> int:
    f = _nb.LEAPFROG_INITIAL if s0 == 0 else 0
    if s0 == last and final_kick:
        f |= _nb.LEAPFROG_FINAL
    return f


_SIDE = threading.local()


def _side_stream(dev: torch.device) -> torch.cuda.Stream:
    """The recomputation stream of this host thread on ``dev`` (default
    priority).  One per thread and device: the library keeps one workspace
    per stream, and a library call's launches must not interleave with
    another thread's on the same stream."""
    streams = getattr(_SIDE, "streams", None)
    if streams is None:
        streams = _SIDE.streams = {}
    s = streams.get(dev.index)
    if s is None:
        s = streams[dev.index] = torch.cuda.Stream(device=dev)
    return s


def reverse_sweep(saved, m, eps2, dt, steps, gx_T, gv_T, checkpoint_every):
    """Adjoints (dL/dx0, dL/dv0, dL/dm) from the output adjoints (gx_T, gv_T).

    Without gv_T the final end kick carries zero weight and is skipped.  As
    in ``reverse_sweep_graphs``, each segment's positions are recomputed on
    a second stream one segment ahead of the sweep (each into a tensor of
    its own, allocated there and recorded for the sweep stream); the result
    is bitwise that of the serial order."""
    dev = m.device
    n = m.shape[0]
    lx = gx_T.detach().clone().contiguous() if gx_T is not None else torch.zeros((n, 3), device=dev)
    lv = gv_T.detach().clone().contiguous() if gv_T is not None else torch.zeros((n, 3), device=dev)
    lm = torch.zeros((n,), device=dev)
    if steps == 0:
        return lx, lv, lm
    k = checkpoint_every
    last = _last_start(steps, k)
    order = list(reversed(range(0, steps, k)))
    rec = [s0 for s0 in order if s0 != last]
    main, side = torch.cuda.current_stream(dev), _side_stream(dev)
    side.wait_stream(main)                        # checkpoints are ready
    pending = {}

    def launch(i):
        if i >= len(rec):
            return
        s0 = rec[i]
        xs, vs, a0 = saved[s0]
        with torch.cuda.stream(side):
            pos = _positions(xs, vs, a0, saved[s0 + k][0], m, eps2, dt, k)
            ev = torch.cuda.Event()
            ev.record(side)
        pos.record_stream(main)
        pending[s0] = (pos, ev)

    launch(0)                                     # runs while the last segment is swept
    for s0 in order:
        if s0 == last:
            pos = saved["tail"]                   # kept by the forward pass
        else:
            i = rec.index(s0)
            pos, ev = pending.pop(s0)
            main.wait_event(ev)
            launch(i + 1)
        _nb.leapfrog_adjoint_(pos, m, eps2, dt, lx, lv, lm,
                              flags=_flags(s0, last, gv_T is not None))
    main.wait_stream(side)
    return lx, lv, lm


class SegmentGraphs:
    """HIP graphs over fixed buffers for one (m, eps2, dt, k):

    ``fwd``     k steps on (x, v, a), with a = a(x) on entry and exit;
    ``pos<b>``  pos[b][1..k-1] from (pos[b][0], pv[b], pa[b]): k - 2 steps,
                then the start kick and drift of the next, for position
                buffers b = 0, 1 (pos[b][k] is the next checkpoint);
    ``rev<b>``  the reverse sweep over an interior segment (global step > 0)
                with positions pos[b][0..k].

    Each graph is captured on a stream of its own after one eager run there,
    so the library workspace its kernels point at belongs to that stream and
    is never regrown while the graph lives (graphs that run at the same time
    never share workspace).  The buffers are scratch for one call at a time
    (no concurrent use from several host threads).
    """

    def __init__(self, m, eps2: float, dt: float, k: int):
        n = m.shape[0]
        dev = m.device
        z = lambda *shape: torch.zeros(shape, dtype=torch.float32, device=dev)
        self.m, self.eps2, self.dt, self.k = m, eps2, dt, k
        self.x, self.v, self.a = z(n, 3), z(n, 3), z(n, 3)
        self.pos = [z(k + 1, n, 3), z(k + 1, n, 3)]
        self.px = [z(n, 3), z(n, 3)]
        self.pv = [z(n, 3), z(n, 3)]
        self.pa = [z(n, 3), z(n, 3)]
        self.lx, self.lv, self.lm = z(n, 3), z(n, 3), z(n)
        # the stream the reverse pass recomputes positions on (default
        # priority, as every stream here)
        self.side = torch.cuda.Stream(device=dev)
        fns = {"fwd": self._fwd}
        for b in (0, 1):
            fns[f"pos{b}"] = lambda b=b: self._pos(b)
            fns[f"rev{b}"] = lambda b=b: self._rev(b)
        self._graphs = {name: self._capture(fn, dev) for name, fn in fns.items()}

    def _fwd(self):
        _nb.leapfrog_(self.x, self.v, self.a, self.m, self.eps2, self.dt, self.k)

    def _pos(self, b: int):
        k, P = self.k, self.pos[b]
        if k > 2:
            self.px[b].copy_(P[0])
            _nb.leapfrog_(self.px[b], self.pv[b], self.pa[b], self.m, self.eps2, self.dt, k - 2,
                          x_hist=P[1:k - 1])
        P[k - 1].copy_(P[k - 2])
        _nb.kick_drift_(P[k - 1], self.pv[b], self.pa[b], -0.5 * self.dt, self.dt)

    def _rev(self, b: int):
        _nb.leapfrog_adjoint_(self.pos[b], self.m, self.eps2, self.dt, self.lx, self.lv, self.lm)

    @staticmethod
    def _capture(fn, dev):
        s = torch.cuda.Stream(device=dev)
        s.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(s):
            fn()                         # sizes this stream's library workspace
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            fn()
        return g, s

    def replay(self, name: str):
        self._graphs[name][0].replay()

    def segment_positions(self, b: int, xs, vs, a0, x_end):
        """pos[b][0..k] of the k steps from (xs, vs, a0 = a(xs)) that end at
        x_end, by one replay on the current stream."""
        self.pos[b][0].copy_(xs)
        self.pos[b][self.k].copy_(x_end)
        self.pv[b].copy_(vs)
        self.pa[b].copy_(a0)
        self.replay(f"pos{b}")
        return self.pos[b]


_GRAPH_CACHE: dict = {}
_GRAPH_CACHE_SIZE = 2


def segment_graphs(m, eps2: float, dt: float, k: int) -> SegmentGraphs:
    """Cached SegmentGraphs for (m's storage and version, eps2, dt, k)."""
    key = (m.device.index, m.data_ptr(), m._version, int(m.shape[0]), float(eps2), float(dt), k)
    g = _GRAPH_CACHE.pop(key, None)
    if g is None:
        g = SegmentGraphs(m, float(eps2), float(dt), k)
        while len(_GRAPH_CACHE) >= _GRAPH_CACHE_SIZE:
            _GRAPH_CACHE.pop(next(iter(_GRAPH_CACHE)))
    _GRAPH_CACHE[key] = g
    return g


def integrate_graphs(G: SegmentGraphs, x0, v0, steps: int):
    """``integrate(..., keep_every=G.k)`` with segments replayed from G's
    graphs; the same ``saved`` contents, bitwise."""
    k = G.k
    G.x.copy_(x0)
    G.v.copy_(v0)
    _nb.forces(G.x, G.m, G.eps2, out=(G.a, None), potential=False)
    saved = {}
    last = _last_start(steps, k)
    for t in range(0, steps, k):
        saved[t] = (G.x.clone(), G.v.clone(), G.a.clone())
        if t < last:
            G.replay("fwd")
        else:                                # the last segment: keep its positions
            count = steps - t
            tail = torch.empty((count + 1,) + tuple(G.x.shape), dtype=G.x.dtype, device=G.x.device)
            tail[0].copy_(G.x)
            _nb.leapfrog_(G.x, G.v, G.a, G.m, G.eps2, G.dt, count, x_hist=tail[1:])
            saved["tail"] = tail
    saved[steps] = (G.x.clone(), G.v.clone(), G.a.clone())
    return G.x.clone(), G.v.clone(), saved


def reverse_sweep_graphs(G: SegmentGraphs, saved, steps, gx_T, gv_T):
    """``reverse_sweep`` with segments recomputed and interior segments swept
    by G's graphs; bitwise equal to the eager sweep.

    The segments that need their positions recomputed take the two position
    buffers in turn.  Each recomputation is replayed on G's side stream,
    after the sweep that last read its buffer (an event on the sweep
    stream), and is launched one segment ahead, so it runs while the
    previous segment is swept; each sweep waits for its positions (an event
    on the side stream).  Every kernel reads what it would read in the
    serial order, so the result is bitwise the same."""
    k, m, eps2, dt = G.k, G.m, G.eps2, G.dt
    lx, lv, lm = G.lx, G.lv, G.lm
    if gx_T is not None:
        lx.copy_(gx_T)
    else:
        lx.zero_()
    if gv_T is not None:
        lv.copy_(gv_T)
    else:
        lv.zero_()
    lm.zero_()
    last = _last_start(steps, k)
    order = list(reversed(range(0, steps, k)))
    rec = [s0 for s0 in order if s0 != last]      # interior segments are full
    buf = {s0: i % 2 for i, s0 in enumerate(rec)}
    main, side = torch.cuda.current_stream(m.device), G.side
    side.wait_stream(main)                        # checkpoints and G's buffers are ready
    ready, freed = {}, [None, None]

    def launch(i):
        if i >= len(rec):
            return
        s0, b = rec[i], buf[rec[i]]
        with torch.cuda.stream(side):
            if freed[b] is not None:
                side.wait_event(freed[b])         # the sweep that last read buffer b
            G.segment_positions(b, *saved[s0], saved[s0 + k][0])
            ready[s0] = torch.cuda.Event()
            ready[s0].record(side)

    launch(0)                                     # runs while the last segment is swept
    for s0 in order:
        if s0 == last:
            pos, b = saved["tail"], None
        else:
            i = rec.index(s0)
            b = buf[s0]
            main.wait_event(ready[s0])
            pos = G.pos[b]
            # the next recomputation takes the other buffer, whose last
            # reader (the previous segment's sweep) has recorded freed[]
            launch(i + 1)
        if b is not None and s0 > 0:
            G.replay(f"rev{b}")
        else:
            _nb.leapfrog_adjoint_(pos, m, eps2, dt, lx, lv, lm,
                                  flags=_flags(s0, last, gv_T is not None))
        if b is not None:
            freed[b] = torch.cuda.Event()
            freed[b].record(main)
    main.wait_stream(side)
    return lx.clone(), lv.clone(), lm.clone()


class Leapfrog(torch.autograd.Function):
    """(x_T, v_T) = leap-frog(x0, v0, m) with a checkpointed adjoint backward."""

    @staticmethod
    def forward(ctx, x0, v0, m, eps2, dt, steps, checkpoint_every, graphs):
        k = int(checkpoint_every) if checkpoint_every else 1
        if k < 1:
            raise ValueError("checkpoint_every must be >= 1")
        md = m.detach()
        if graphs is None:
            graphs = md.shape[0] <= GRAPHS_MAX_N
        G = segment_graphs(md, eps2, dt, k) if graphs and k > 1 and steps >= k else None
        if G is not None:
            x, v, saved = integrate_graphs(G, x0.detach(), v0.detach(), int(steps))
        else:
            x, v, saved = integrate(x0, v0, m, eps2, dt, steps, keep_every=k)
        ctx.saved = saved
        ctx.m = md
        ctx.graphs = G
        ctx.args = (float(eps2), float(dt), int(steps), k)
        ctx.set_materialize_grads(False)
        return x, v

    @staticmethod
    def backward(ctx, gx_T, gv_T):
        eps2, dt, steps, k = ctx.args
        if ctx.graphs is not None:
            lx, lv, lm = reverse_sweep_graphs(ctx.graphs, ctx.saved, steps, gx_T, gv_T)
        else:
            lx, lv, lm = reverse_sweep(ctx.saved, ctx.m, eps2, dt, steps, gx_T, gv_T, k)
        return lx, lv, lm, None, None, None, None, None


# Largest n for which ``leapfrog(graphs=None)`` replays HIP graphs.  The
# 64-step gradient with checkpoints every 8 steps takes 11-19% less time
# with graphs from 128 to 2,048 bodies, where a step's kernels take a few
# microseconds and the host's launches show; from 3,000 bodies on the
# eager launches are faster (5% at 3,000, 18% at 4,096, 2-8% at 16,384): a
# graph's kernel nodes start a little later than launches into a stream,
# and the eager reverse pass recomputes positions as far ahead of the sweep
# as the host gets (a tensor per segment) where the graphs have two fixed
# position buffers.
GRAPHS_MAX_N = 2048


def leapfrog(x0, v0, m, eps2: float, dt: float, steps: int, checkpoint_every: int | None = 8,
             graphs: bool | None = None):
    """Integrate ``steps`` leap-frog steps; differentiable in (x0, v0, m).

    ``checkpoint_every=k`` keeps (x, v) every k steps and recomputes the
    rest in the backward pass; ``None`` or 1 keeps every step.  With
    ``graphs`` (and k > 1) the segments replay from cached HIP graphs
    (``SegmentGraphs``); the result is bitwise that of ``graphs=False``.
    ``None`` takes graphs for n <= ``GRAPHS_MAX_N``.  The graphs read ``m``
    in place at every replay.
    """
    return Leapfrog.apply(x0, v0, m, eps2, dt, steps, checkpoint_every, graphs)
