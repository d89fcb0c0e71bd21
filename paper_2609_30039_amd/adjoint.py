"""Reverse sweep driver and the torch autograd bridge (Section 3: discrete
adjoint with binomial checkpoint replay).

The forward recording sweep runs the recording prefix of the binomial
schedule (advances with monitors on, checkpoint saves), then one more step to
u^N so that every monitor sample n = 1..N is taken.  The reverse phase
re-establishes u^{N-1} from the last saved slot and follows the rest of the
schedule: restores, replays (monitors off) and adjoint steps.  Every numeric
operation runs in libfdtd; this module only orders calls.
"""
from __future__ import annotations

from typing import Callable, Dict, Optional

import numpy as np

from . import revolve
from .sim import Simulation


class RevolvePlan:
    """Binomial schedule for n_steps with n_slots checkpoint slots."""

    def __init__(self, n_steps: int, n_slots: int):
        if n_slots < 1:
            raise ValueError("at least one checkpoint slot is needed")
        self.n_steps = n_steps
        self.n_slots = n_slots
        actions = revolve.schedule(n_steps, n_slots) if n_steps > 0 else []
        self.record, self.reverse = revolve.split_recording(actions)
        self.forward_evals = revolve.forward_count(n_steps, n_slots)


def forward_record(sim: Simulation, plan: RevolvePlan):
    """Recording sweep u^0 -> u^N with the schedule's checkpoints."""
    sim.reset()
    sim.save(0)
    last_slot, last_pos = 0, 0
    t = 0
    for a in plan.record:
        if a[0] == "advance":
            sim.step(a[1], record=True)
            t += a[1]
        elif a[0] == "save":
            sim.save(a[1])
            last_slot, last_pos = a[1], t
        elif a[0] == "restore":
            raise RuntimeError("recording prefix never restores")
    N = plan.n_steps
    if t < N:
        sim.step(N - t, record=True)
    return last_slot, last_pos


def reverse_sweep(sim: Simulation, plan: RevolvePlan, last_slot: int, last_pos: int, progress=None):
    """Reverse phase: ubar^N -> ubar^0, accumulating dJ/deps in the library.
    progress(m), if given, is called after every 500th adjoint step."""
    N = plan.n_steps
    sim.adjoint_begin(N)
    if N == 0:
        return
    # the schedule expects the current state u^{N-1}; the recording sweep ended at u^N
    sim.restore(last_slot)
    if N - 1 - last_pos > 0:
        sim.step(N - 1 - last_pos, record=False)
    for a in plan.reverse:
        if a[0] == "advance":
            sim.step(a[1], record=False)
        elif a[0] == "save":
            sim.save(a[1])
        elif a[0] == "restore":
            sim.restore(a[1])
        elif a[0] == "adjoint":
            sim.step_adjoint(1)
            if progress is not None and sim.steps[1] % 500 == 0:
                progress(sim.steps[1])


def gradient(sim: Simulation, n_steps: int, n_slots: int,
             cotangent_fn: Callable[[Simulation], Dict[int, np.ndarray]]):
    """Forward record, cotangents from the monitors, reverse sweep.  Returns
    the per-domain gradient arrays (dJ/deps over each gradient box)."""
    plan = RevolvePlan(n_steps, n_slots)
    last_slot, last_pos = forward_record(sim, plan)
    cots = cotangent_fn(sim)
    for (dom, mon), g in cots.items():
        sim.set_cotangent(mon, g, domain=dom)
    reverse_sweep(sim, plan, last_slot, last_pos)
    return [sim.grad(d) if s.grad_box is not None else None for d, s in enumerate(sim.specs)]


# ---------------------------------------------------------------- reversible mode
def reversible_admissible(specs) -> bool:
    """Whether the reversible mode applies (Section 3.2: it follows from the
    content of the problem): every domain with a gradient has no dispersive
    box, no tensor media and no periodic axis, and its gradient box lies
    between the absorbing slabs, one cell clear of a low slab (the curl at
    the gradient box reads H one cell back)."""
    if not isinstance(specs, (list, tuple)):
        specs = [specs]
    any_grad = False
    for s in specs:
        if s.grad_box is None:
            continue
        any_grad = True
        if s.lorentz or s.eps_kind == "tensor" or any(getattr(s, "periodic", (0, 0, 0))):
            return False
        (glo, ghi) = s.grad_box
        for a in range(3):
            lo, hi = s.pml[2 * a], s.shape[a] - s.pml[2 * a + 1]
            if glo[a] < lo + (1 if lo > 0 else 0) or ghi[a] > hi:
                return False
    return any_grad


def reversible_sweep(sim: Simulation, n_steps: int, progress=None):
    """Reverse sweep of a handle created with reversible=True whose forward
    state is u^N: each adjoint step m -> m-1 is preceded by one backward step
    of the lossless box (u^m -> u^{m-1}); no checkpoint is read."""
    sim.adjoint_begin(n_steps)
    for m in range(n_steps, 0, -1):
        sim.step_reverse(1)
        sim.step_adjoint(1)
        if progress is not None and (m - 1) % 500 == 0:
            progress(m - 1)


def reversible_gradient(sim: Simulation, n_steps: int,
                        cotangent_fn: Callable[[Simulation], Dict[int, np.ndarray]]):
    """Forward from rest with the interface recorded, cotangents from the
    monitors, reversible reverse sweep.  Returns the per-domain gradients."""
    sim.reset()
    sim.step(n_steps, record=True)
    for (dom, mon), g in cotangent_fn(sim).items():
        sim.set_cotangent(mon, g, domain=dom)
    reversible_sweep(sim, n_steps)
    return [sim.grad(d) if s.grad_box is not None else None for d, s in enumerate(sim.specs)]


def retained_gradients(sim: Simulation, n_steps: int, objectives, slot: int = 0):
    """Several objectives from one forward run (the retained backward pass of
    Section 3.2): the forward sweep runs once and its final state u^N is kept
    in checkpoint slot `slot`; each objective's cotangents (a function of the
    recorded spectra) then get their own reverse sweep from that state, in the
    reversible mode.  Returns one gradient list per objective."""
    sim.reset()
    sim.step(n_steps, record=True)
    sim.save(slot)
    cots = [fn(sim) for fn in objectives]          # every objective sees the same forward run
    out = []
    for c in cots:
        sim.restore(slot)
        for (dom, mon), g in c.items():
            sim.set_cotangent(mon, g, domain=dom)
        reversible_sweep(sim, n_steps)
        out.append([sim.grad(d) if s.grad_box is not None else None for d, s in enumerate(sim.specs)])
    return out


# ---------------------------------------------------------------- torch bridge
def _torch():
    import torch
    return torch


class FDTDFunction:
    """torch.autograd.Function: eps (over the eps box) -> monitor spectra.

    forward(eps) uploads eps, runs the recording sweep and returns one complex
    tensor per plane monitor; backward(grad spectra) sets the cotangents
    (torch's dJ/dRe + i dJ/dIm convention), runs the reverse sweep and
    returns dJ/deps (zero outside the gradient box).  The checkpoints live in
    the Simulation, so backward raises if another forward sweep ran on it in
    between."""

    @staticmethod
    def build():
        torch = _torch()

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, eps, sim, n_slots):
                spec = sim.specs[0]
                sim.set_eps(eps.detach().cpu().double().numpy())
                plan = RevolvePlan(spec.n_steps, n_slots)
                ctx.sim, ctx.plan = sim, plan
                ctx.last = forward_record(sim, plan)
                ctx.generation = sim.generation
                ctx.eps_shape = tuple(eps.shape)
                ctx.device, ctx.dtype = eps.device, eps.dtype
                outs = []
                ctx.mons = []
                for mi, m in enumerate(spec.monitors):
                    if m.kind == "probe":
                        continue
                    outs.append(torch.from_numpy(sim.spectra(mi)).to(eps.device))
                    ctx.mons.append(mi)
                return tuple(outs)

            @staticmethod
            def backward(ctx, *grads):
                sim, plan = ctx.sim, ctx.plan
                if sim.generation != ctx.generation:
                    # another forward (or a new eps) replaced the checkpoints and
                    # the permittivity this backward pass would replay
                    raise RuntimeError("the Simulation ran another forward sweep since this output was computed; "
                                       "use one Simulation per pending backward pass")
                spec = sim.specs[0]
                for mi, g in zip(ctx.mons, grads):
                    if g is None:
                        sim.set_cotangent(mi, np.zeros_like(sim.spectra(mi)))
                    else:
                        sim.set_cotangent(mi, g.detach().cpu().numpy().astype(np.complex128))
                reverse_sweep(sim, plan, *ctx.last)
                gb = sim.grad(0)
                full = np.zeros(ctx.eps_shape)
                (elo, ehi), (glo, ghi) = spec.eps_box, spec.grad_box
                sl = tuple(slice(glo[a] - elo[a], ghi[a] - elo[a]) for a in (2, 1, 0))
                full[(slice(None),) + sl] = gb if full.shape[0] == gb.shape[0] else gb.sum(axis=0, keepdims=True)
                return torch.from_numpy(full).to(ctx.device, ctx.dtype), None, None

        return _Fn


def differentiable_spectra(eps, sim: Simulation, n_slots: int):
    """Plane-monitor spectra of sim's first domain as differentiable functions of eps."""
    return FDTDFunction.build().apply(eps, sim, n_slots)
