"""Differentiable COLA run: d(loss on the final density or binned P(k)) / d(white noise).

The backward pass is the hand-written adjoint of libcola (reverse kick/drift,
transposed CIC readout and deposit, transposed Green's function, transposed
2LPT maps).  Memory: the full particle state is kept every ``segment`` steps;
inside a segment the step-start positions are recomputed forward, then the
segment is reversed (each step is recomputed at most once).  With
keep_forces the recomputed steps leave their force meshes in one slot per
step of the segment (cola_step_keep) and the adjoint reads them instead of
recomputing the forces a second time (same gradient, bit for bit; a slot is
three PM meshes).
"""
from __future__ import annotations

import numpy as np
import torch

from .sim import ColaSim


def _run_segment(sim, edges, i0, i1, slots=None):
    """Forward steps i0..i1-1 from the current state; returns step-start (disp, a_v).
    slots: one force slot per step (cola_step_keep) or None."""
    out = []
    for i in range(i0, i1):
        st = sim.get_state()
        out.append((st["disp"], st["a_v"]))
        if slots is None:
            sim.step(edges[i], edges[i + 1])
        else:
            sim.step_keep(edges[i], edges[i + 1], slots[i - i0])
    return out


def _backward(sim, noise, edges, saved_states, segment, dbar, vbar, keep_forces=False):
    p1b = torch.zeros_like(dbar)
    p2b = torch.zeros_like(dbar)
    nstep = len(edges) - 1
    starts = list(range(0, nstep, segment))
    slots = [sim.force_slot() for _ in range(min(segment, nstep))] if keep_forces else None
    for s0 in reversed(starts):
        s1 = min(s0 + segment, nstep)
        st = saved_states[s0]
        sim.set_state(st["disp"], st["vres"], st["psi1"], st["psi2"], st["a_x"], st["a_v"])
        steps = _run_segment(sim, edges, s0, s1, slots)
        for i in reversed(range(s0, s1)):
            disp0, a_v0 = steps[i - s0]
            sim.step_adjoint(edges[i], edges[i + 1], a_v0, disp0, dbar, vbar, p1b, p2b,
                             slot=None if slots is None else slots[i - s0])
    return sim.init_adjoint(noise, dbar, p1b, p2b)


def _forward(sim, noise, k, pk, edges, segment):
    sim.init_from_noise(noise, k, pk)
    saved = {}
    nstep = len(edges) - 1
    for i in range(nstep):
        if i % segment == 0:
            saved[i] = {n: (v.clone() if torch.is_tensor(v) else v) for n, v in sim.get_state().items()}
        sim.step(edges[i], edges[i + 1])
    return saved


class ColaDensity(torch.autograd.Function):
    """noise (np^3) -> final density contrast (nmesh^3) through a full COLA run."""

    @staticmethod
    def forward(ctx, noise, sim: ColaSim, k, pk, edges, segment=1, keep_forces=False):
        saved = _forward(sim, noise.detach().contiguous(), k, pk, edges, segment)
        ctx.sim, ctx.edges, ctx.saved, ctx.segment = sim, list(edges), saved, segment
        ctx.keep = keep_forces
        final = sim.get_state()
        ctx.final_disp = final["disp"]
        ctx.save_for_backward(noise)
        return sim.density()

    @staticmethod
    def backward(ctx, grad_delta):
        (noise,) = ctx.saved_tensors
        sim = ctx.sim
        dbar = torch.zeros_like(ctx.final_disp)
        sim.density_adjoint(ctx.final_disp, grad_delta.contiguous(), dbar)
        vbar = torch.zeros_like(dbar)
        wbar = _backward(sim, noise.contiguous(), ctx.edges, ctx.saved, ctx.segment, dbar, vbar, ctx.keep)
        return wbar, None, None, None, None, None, None


class ColaPowerSpectrum(torch.autograd.Function):
    """noise -> binned P(k) of the final particles (host bins returned as a CPU tensor)."""

    @staticmethod
    def forward(ctx, noise, sim: ColaSim, k, pk, edges, kedges, ngrid=None, segment=1, keep_forces=False):
        saved = _forward(sim, noise.detach().contiguous(), k, pk, edges, segment)
        ctx.sim, ctx.edges, ctx.saved, ctx.segment = sim, list(edges), saved, segment
        ctx.keep = keep_forces
        ctx.kedges, ctx.ngrid = np.asarray(kedges, np.float64), ngrid
        final = sim.get_state()
        ctx.final_disp = final["disp"]
        ctx.save_for_backward(noise)
        _, p, n = sim.pk(ctx.kedges, ngrid)
        return torch.from_numpy(np.where(n > 0, p, 0.0))

    @staticmethod
    def backward(ctx, grad_p):
        (noise,) = ctx.saved_tensors
        sim = ctx.sim
        dbar = torch.zeros_like(ctx.final_disp)
        sim.pk_adjoint(ctx.final_disp, ctx.kedges, grad_p.detach().cpu().double().numpy(), dbar, ctx.ngrid)
        vbar = torch.zeros_like(dbar)
        wbar = _backward(sim, noise.contiguous(), ctx.edges, ctx.saved, ctx.segment, dbar, vbar, ctx.keep)
        return wbar, None, None, None, None, None, None, None, None


def pk_noise_gradient(sim: ColaSim, noise, k, pk, edges, kedges, cbar, ngrid=None, every=None,
                      times=None):
    """d(sum_b cbar_b P_b) / d(noise) for P(k) of the final particles, in the
    least device memory: one position buffer, the four cotangent arrays and
    a (displacement, velocity) checkpoint every ``every`` steps (None: none;
    the initial conditions are rebuilt from the noise instead).  Each step's
    start positions are recomputed from the nearest earlier checkpoint; the
    step is deterministic, so they equal the forward's bit for bit.
    ``times``: a dict that receives the wall seconds of the forward run
    ("forward"), of the recomputed steps ("recompute") and of the adjoint
    steps ("adjoint"), the device synchronised around each phase.
    Returns (gradient, P(k) of the forward run)."""
    import time

    def mark():
        if times is not None:
            torch.cuda.synchronize(sim.device)
        return time.perf_counter()

    if times is not None:
        times.update(forward=0.0, recompute=0.0, adjoint=0.0, recomputed_steps=0)
    kedges = np.asarray(kedges, np.float64)
    nstep = len(edges) - 1
    every = nstep if every is None else max(1, int(every))
    noise = noise.detach().contiguous()
    ckpt = {}

    def restart(i0):
        """The state at the start of step i0, from the nearest earlier checkpoint."""
        base = max([j for j in ckpt if j <= i0], default=0)
        if base == 0:
            sim.init_from_noise(noise, k, pk)
        else:
            d, v, ax, av = ckpt[base]
            sim.set_state(d, v, None, None, ax, av)
        for i in range(base, i0):
            sim.step(edges[i], edges[i + 1])

    t0 = mark()
    sim.init_from_noise(noise, k, pk)
    for i in range(nstep):
        if i > 0 and i % every == 0:
            st = sim.get_state(("disp", "vres"))
            ckpt[i] = (st["disp"], st["vres"], st["a_x"], st["a_v"])
        sim.step(edges[i], edges[i + 1])
    if times is not None:
        times["forward"] = mark() - t0
    _, p, n = sim.pk(kedges, ngrid)
    pos = sim.get_state(("disp",))["disp"]
    dbar = torch.zeros_like(pos)
    sim.pk_adjoint(pos, kedges, np.where(n > 0, np.asarray(cbar, np.float64), 0.0), dbar, ngrid)
    vbar = torch.zeros_like(dbar)
    p1b = torch.zeros_like(dbar)
    p2b = torch.zeros_like(dbar)
    for i in reversed(range(nstep)):
        t0 = mark()
        restart(i)
        st = sim.get_state(("disp",), out={"disp": pos})
        t1 = mark()
        sim.step_adjoint(edges[i], edges[i + 1], st["a_v"], pos, dbar, vbar, p1b, p2b)
        if times is not None:
            t2 = mark()
            times["recompute"] += t1 - t0
            times["adjoint"] += t2 - t1
            times["recomputed_steps"] += i
    del pos, vbar
    return sim.init_adjoint(noise, dbar, p1b, p2b), np.where(n > 0, p, 0.0)

