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
"""

from __future__ import annotations

import torch

from . import nbody as _nb


def _step(x, v, a, m, eps2, dt):
    """One KDK step in place; `a` holds a(x) on entry and a(x') on exit."""
    _nb.kick_drift_(x, v, a, -0.5 * dt, dt)      # Eqs. (1)-(2)
    _nb.forces(x, m, eps2, out=(a, None), potential=False)
    _nb.axpy_(v, a, -0.5 * dt)                   # Eq. (3)


def integrate(x0, v0, m, eps2, dt, steps, *, keep_every: int | None = None):
    """Run ``steps`` KDK steps from (x0, v0).

    Returns (x_T, v_T, saved) where ``saved`` maps step index -> (x, v)
    copies taken every ``keep_every`` steps (step 0 included), or {} if
    ``keep_every`` is None.
    """
    x = x0.detach().clone().contiguous()
    v = v0.detach().clone().contiguous()
    a, _ = _nb.forces(x, m, eps2, potential=False)
    saved = {}
    for t in range(steps):
        if keep_every and t % keep_every == 0:
            saved[t] = (x.clone(), v.clone())
        _step(x, v, a, m, eps2, dt)
    if keep_every:
        saved[steps] = (x.clone(), v.clone())
    return x, v, saved


def _positions(xs, vs, m, eps2, dt, count):
    """Positions after 0..count steps from (xs, vs)."""
    x = xs.clone()
    v = vs.clone()
    a, _ = _nb.forces(x, m, eps2, potential=False)
    out = [x.clone()]
    for _ in range(count):
        _step(x, v, a, m, eps2, dt)
        out.append(x.clone())
    return out


def reverse_sweep(saved, m, eps2, dt, steps, gx_T, gv_T, checkpoint_every):
    """Adjoints (dL/dx0, dL/dv0, dL/dm) from the output adjoints (gx_T, gv_T)."""
    dev = m.device
    n = m.shape[0]
    lx = gx_T.detach().clone().contiguous() if gx_T is not None else torch.zeros((n, 3), device=dev)
    lv = gv_T.detach().clone().contiguous() if gv_T is not None else torch.zeros((n, 3), device=dev)
    lm = torch.zeros((n,), device=dev)
    half = 0.5 * dt
    gxw = torch.empty((n, 3), device=dev)
    gmw = torch.empty((n,), device=dev)
    if steps == 0:
        return lx, lv, lm
    k = checkpoint_every
    seg_starts = list(range(0, steps, k))
    first = True
    for s0 in reversed(seg_starts):
        s1 = min(s0 + k, steps)
        xs, vs = saved[s0]
        if s1 - s0 == 1:
            pos = [xs, saved[s1][0]]                     # every step was kept
        else:
            pos = _positions(xs, vs, m, eps2, dt, s1 - s0)  # x_{s0} .. x_{s1}
        if first:
            # end kick of the last step, weight lv_T
            if gv_T is not None:
                _nb.forces_backward(pos[-1], m, eps2, lv, None, out=(gxw, gmw))
                _nb.axpy_(lx, gxw, -half)
                _nb.axpy_(lm, gmw, -half)
            first = False
        for t in range(s1, s0, -1):
            _nb.axpy_(lv, lx, dt)                        # drift of step t-1
            c = -dt if t - 1 > 0 else -half               # start kick of t-1 (+ end kick of t-2)
            _nb.forces_backward(pos[t - 1 - s0], m, eps2, lv, None, out=(gxw, gmw))
            _nb.axpy_(lx, gxw, c)
            _nb.axpy_(lm, gmw, c)
    return lx, lv, lm


class Leapfrog(torch.autograd.Function):
    """(x_T, v_T) = leap-frog(x0, v0, m) with a checkpointed adjoint backward."""

    @staticmethod
    def forward(ctx, x0, v0, m, eps2, dt, steps, checkpoint_every):
        k = int(checkpoint_every) if checkpoint_every else 1
        if k < 1:
            raise ValueError("checkpoint_every must be >= 1")
        x, v, saved = integrate(x0, v0, m, eps2, dt, steps, keep_every=k)
        ctx.saved = saved
        ctx.m = m.detach()
        ctx.args = (float(eps2), float(dt), int(steps), k)
        ctx.set_materialize_grads(False)
        return x, v

    @staticmethod
    def backward(ctx, gx_T, gv_T):
        eps2, dt, steps, k = ctx.args
        lx, lv, lm = reverse_sweep(ctx.saved, ctx.m, eps2, dt, steps, gx_T, gv_T, k)
        return lx, lv, lm, None, None, None, None


def leapfrog(x0, v0, m, eps2: float, dt: float, steps: int, checkpoint_every: int | None = 8):
    """Integrate ``steps`` leap-frog steps; differentiable in (x0, v0, m).

    ``checkpoint_every=k`` keeps (x, v) every k steps and recomputes the
    rest in the backward pass; ``None`` or 1 keeps every step.
    """
    return Leapfrog.apply(x0, v0, m, eps2, dt, steps, checkpoint_every)
