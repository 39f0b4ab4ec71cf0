"""Device-resident leap-frog integration and its checkpointed adjoint.

The integrator is the kick-drift-kick scheme of Eqs. (1)-(3) with the
seven-step algorithm of Sec. III: one force evaluation per step, reused by
the next step's first kick.  The paper's a (Eq. (gravity)) points away from
the attracting body, so the physical acceleration is g = -a and a kick is
v += (dt/2) g = v - (dt/2) a.  Every step is a library call: the force
evaluation (``nbody_forces``), its adjoint (``nbody_forces_backward``) and
the kick/drift updates (``nbody_kick_drift``, ``nbody_axpy``); tensors only
hold device memory.

Reverse sweep for a loss on the final state.  With adjoints (lx, lv) of the
step output (x_t, v_t), stepping back over step t-1 is
    lx += -(dt/2) VJP_a(x_t)[lv]        (end kick of step t-1)
    lv += dt lx                         (drift: lv is now the half-step adjoint)
    lx += -(dt/2) VJP_a(x_{t-1})[lv]    (start kick of step t-1)
and the start kick of step t-1 and the end kick of step t-2 meet at the
same positions with the same weight, so they are applied as one product with
factor dt.  Masses collect the same products' dL/dm parts.

Checkpointing: the forward pass keeps (x, v) every ``checkpoint_every``
steps; the reverse pass recomputes each segment's positions from its
checkpoint before sweeping it.  The kernels are deterministic, so the
recomputed positions and hence the gradients are bitwise equal to those of a
run that stores every position.

HIP graphs: a k-step segment (3k launches), the recomputation of a
segment's positions and the reverse sweep over an interior segment are each
captured once as a HIP graph on fixed device buffers and replayed once per
segment, instead of issuing every launch from Python.  The graphs run the
same kernels on the same data, so results are bitwise equal to the eager
path (``graphs=False``).
"""

from __future__ import annotations

import torch

from . import nbody as _nb


def _step(x, v, a, m, eps2, dt):
    """One KDK step in place; `a` holds a(x) on entry and a(x') on exit."""
    _nb.kick_drift_(x, v, a, -0.5 * dt, dt)      # Eqs. (1)-(2)
    _nb.forces(x, m, eps2, out=(a, None), potential=False)
    _nb.axpy_(v, a, -0.5 * dt)                   # Eq. (3)


def _last_start(steps: int, k: int) -> int:
    """First step of the last checkpoint segment."""
    return ((steps - 1) // k) * k


def integrate(x0, v0, m, eps2, dt, steps, *, keep_every: int | None = None):
    """Run ``steps`` KDK steps from (x0, v0).

    Returns (x_T, v_T, saved).  With ``keep_every=k``, ``saved[t]`` is a
    copy of (x, v, a) at every step t that is a multiple of k and at
    t = steps, and ``saved["tail"]`` holds the positions of the last
    segment (x at its first step .. x_T), which the reverse sweep then need
    not recompute.  Without it ``saved`` is {}.
    """
    x = x0.detach().clone().contiguous()
    v = v0.detach().clone().contiguous()
    a, _ = _nb.forces(x, m, eps2, potential=False)
    saved = {}
    last = _last_start(steps, keep_every) if keep_every and steps > 0 else None
    tail = []
    for t in range(steps):
        if keep_every and t % keep_every == 0:
            saved[t] = (x.clone(), v.clone(), a.clone())
        if t == last:
            tail.append(x.clone())
        _step(x, v, a, m, eps2, dt)
        if last is not None and t >= last:
            tail.append(x.clone())
    if keep_every:
        saved[steps] = (x.clone(), v.clone(), a.clone())
        saved["tail"] = tail
    return x, v, saved


def _positions(xs, vs, a0, m, eps2, dt, count):
    """Positions after 0..count steps from (xs, vs) with a0 = a(xs)."""
    x = xs.clone()
    v = vs.clone()
    a = a0.clone()
    out = [x.clone()]
    for _ in range(count):
        _step(x, v, a, m, eps2, dt)
        out.append(x.clone())
    return out


def _sweep_segment(pos, s0, s1, m, eps2, dt, lx, lv, lm, gxw, gmw):
    """Reverse over steps s1-1 .. s0 with positions pos[0..s1-s0]."""
    half = 0.5 * dt
    for t in range(s1, s0, -1):
        _nb.axpy_(lv, lx, dt)                            # drift of step t-1
        c = -dt if t - 1 > 0 else -half                   # start kick of t-1 (+ end kick of t-2)
        _nb.forces_backward(pos[t - 1 - s0], m, eps2, lv, None, out=(gxw, gmw))
        _nb.axpy_(lx, gxw, c)
        _nb.axpy_(lm, gmw, c)


def _end_kick(pos_T, m, eps2, dt, lx, lv, lm, gxw, gmw):
    """The last step's end kick, weight lv_T."""
    _nb.forces_backward(pos_T, m, eps2, lv, None, out=(gxw, gmw))
    _nb.axpy_(lx, gxw, -0.5 * dt)
    _nb.axpy_(lm, gmw, -0.5 * dt)


def reverse_sweep(saved, m, eps2, dt, steps, gx_T, gv_T, checkpoint_every):
    """Adjoints (dL/dx0, dL/dv0, dL/dm) from the output adjoints (gx_T, gv_T)."""
    dev = m.device
    n = m.shape[0]
    lx = gx_T.detach().clone().contiguous() if gx_T is not None else torch.zeros((n, 3), device=dev)
    lv = gv_T.detach().clone().contiguous() if gv_T is not None else torch.zeros((n, 3), device=dev)
    lm = torch.zeros((n,), device=dev)
    gxw = torch.empty((n, 3), device=dev)
    gmw = torch.empty((n,), device=dev)
    if steps == 0:
        return lx, lv, lm
    k = checkpoint_every
    last = _last_start(steps, k)
    for s0 in reversed(range(0, steps, k)):
        s1 = min(s0 + k, steps)
        if s0 == last:
            pos = saved["tail"]                          # kept by the forward pass
            if gv_T is not None:
                _end_kick(pos[-1], m, eps2, dt, lx, lv, lm, gxw, gmw)
        else:
            xs, vs, a0 = saved[s0]
            pos = _positions(xs, vs, a0, m, eps2, dt, s1 - s0)  # x_{s0} .. x_{s1}
        _sweep_segment(pos, s0, s1, m, eps2, dt, lx, lv, lm, gxw, gmw)
    return lx, lv, lm


class SegmentGraphs:
    """Three HIP graphs over fixed buffers for one (m, eps2, dt, k):

    ``fwd``  k steps on (x, v, a), with a = a(x) on entry and exit;
    ``pos``  k steps from (pos[0], pv, pa), keeping pos[1..k];
    ``rev``  the reverse sweep over an interior segment (global step > 0):
             for local t = k..1: lv += dt lx; lx, lm -= dt VJP(pos[t-1])[lv].

    Each graph is captured on a stream of its own after one eager run there,
    so the library workspace its kernels point at belongs to that stream and
    is never regrown while the graph lives.  The buffers are scratch for one
    call at a time (no concurrent use from several host threads).
    """

    def __init__(self, m, eps2: float, dt: float, k: int):
        n = m.shape[0]
        dev = m.device
        z = lambda *shape: torch.zeros(shape, dtype=torch.float32, device=dev)
        self.m, self.eps2, self.dt, self.k = m, eps2, dt, k
        self.x, self.v, self.a = z(n, 3), z(n, 3), z(n, 3)
        self.pos = [z(n, 3) for _ in range(k + 1)]
        self.pv, self.pa = z(n, 3), z(n, 3)
        self.lx, self.lv, self.lm = z(n, 3), z(n, 3), z(n)
        self.gxw, self.gmw = z(n, 3), z(n)
        self._graphs = {name: self._capture(fn, dev)
                        for name, fn in (("fwd", self._fwd), ("pos", self._pos), ("rev", self._rev))}

    def _fwd(self):
        for _ in range(self.k):
            _step(self.x, self.v, self.a, self.m, self.eps2, self.dt)

    def _pos(self):
        for i in range(self.k):
            self.pos[i + 1].copy_(self.pos[i])
            _step(self.pos[i + 1], self.pv, self.pa, self.m, self.eps2, self.dt)

    def _rev(self):
        _sweep_segment(self.pos, 1, 1 + self.k, self.m, self.eps2, self.dt,
                       self.lx, self.lv, self.lm, self.gxw, self.gmw)

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

    def segment_positions(self, xs, vs, a0):
        """pos[0..k] from (xs, vs, a0 = a(xs)) by one replay."""
        self.pos[0].copy_(xs)
        self.pv.copy_(vs)
        self.pa.copy_(a0)
        self.replay("pos")
        return self.pos


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
        elif steps - t == k:                 # a full last segment: keep its positions
            pos = G.segment_positions(G.x, G.v, G.a)
            saved["tail"] = [p.clone() for p in pos]
            G.x.copy_(pos[k])
            G.v.copy_(G.pv)
            G.a.copy_(G.pa)
        else:
            tail = [G.x.clone()]
            for _ in range(steps - t):
                _step(G.x, G.v, G.a, G.m, G.eps2, G.dt)
                tail.append(G.x.clone())
            saved["tail"] = tail
    saved[steps] = (G.x.clone(), G.v.clone(), G.a.clone())
    return G.x.clone(), G.v.clone(), saved


def reverse_sweep_graphs(G: SegmentGraphs, saved, steps, gx_T, gv_T):
    """``reverse_sweep`` with segments recomputed and interior segments swept
    by G's graphs; bitwise equal to the eager sweep."""
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
    for s0 in reversed(range(0, steps, k)):
        s1 = min(s0 + k, steps)
        if s0 == last:
            pos = saved["tail"]
            if gv_T is not None:
                _end_kick(pos[-1], m, eps2, dt, lx, lv, lm, G.gxw, G.gmw)
        else:
            xs, vs, a0 = saved[s0]
            pos = G.segment_positions(xs, vs, a0)    # interior segments are full
            if s0 > 0:
                G.replay("rev")
                continue
        _sweep_segment(pos, s0, s1, m, eps2, dt, lx, lv, lm, G.gxw, G.gmw)
    return lx.clone(), lv.clone(), lm.clone()


class Leapfrog(torch.autograd.Function):
    """(x_T, v_T) = leap-frog(x0, v0, m) with a checkpointed adjoint backward."""

    @staticmethod
    def forward(ctx, x0, v0, m, eps2, dt, steps, checkpoint_every, graphs):
        k = int(checkpoint_every) if checkpoint_every else 1
        if k < 1:
            raise ValueError("checkpoint_every must be >= 1")
        md = m.detach()
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


def leapfrog(x0, v0, m, eps2: float, dt: float, steps: int, checkpoint_every: int | None = 8,
             graphs: bool = True):
    """Integrate ``steps`` leap-frog steps; differentiable in (x0, v0, m).

    ``checkpoint_every=k`` keeps (x, v) every k steps and recomputes the
    rest in the backward pass; ``None`` or 1 keeps every step.  With
    ``graphs`` (and k > 1) the segments replay from cached HIP graphs
    (``SegmentGraphs``); the result is bitwise that of ``graphs=False``.
    The graphs read ``m`` in place at every replay.
    """
    return Leapfrog.apply(x0, v0, m, eps2, dt, steps, checkpoint_every, graphs)
