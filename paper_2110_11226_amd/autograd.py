"""Differentiable fitness: d(fitness)/d(program constants) through
gp_fitness_backward, and gradient refinement of elite programs' constants.

The forward pass is gp_fitness and the backward pass gp_fitness_backward
(reverse mode over each prefix list, recomputing the forward values per row
tile); both run in libgp.so.  PyTorch only holds the tensors.
"""
from __future__ import annotations

import torch

from . import _binding as B


class GPFitness(torch.autograd.Function):
    """fitness = GPFitness.apply(consts, pop, data, metric).

    consts is a float32 device tensor laid out like pop.consts (constant slot
    s of program p at consts[const_off[p] + s]); the result is the float32
    fitness of every program, differentiable with respect to consts."""

    @staticmethod
    def forward(ctx, consts, pop, data, metric):
        consts = consts.contiguous()
        view = pop.make_view(consts)
        out = torch.empty(pop.n_programs, dtype=torch.float32, device=consts.device)
        B._check(B._fitness(B.ctypes.byref(view), B.ctypes.byref(data.view), B.metric_id(metric),
                            B._tptr(out), B._stream()), "gp_fitness")
        ctx.save_for_backward(consts)
        ctx.pop, ctx.data, ctx.metric = pop, data, metric
        return out

    @staticmethod
    def backward(ctx, grad_fit):
        (consts,) = ctx.saved_tensors
        g = B.fitness_backward(ctx.pop, ctx.data, ctx.metric,
                               grad_fitness=grad_fit.contiguous().to(torch.float32), consts=consts)
        full = torch.zeros_like(consts)
        full[:g.shape[0]] = g
        return full, None, None, None


def refine_constants(pop, data, metric, programs, steps=5, lr=1e-2):
    """Adam steps on the constants of `programs` (indices) to improve their
    fitness; a program keeps its refined constants only if its fitness
    improved.  Returns (new consts tensor, fitness before, fitness after)."""
    larger = B.larger_is_better(metric)
    dev = pop.consts.device
    progs = torch.as_tensor(programs, dtype=torch.int64, device=dev)
    co = pop.const_off
    mask = torch.zeros(pop.consts.shape[0], dtype=torch.bool, device=dev)
    lo, hi = co[progs], co[progs + 1]
    for a, b in zip(lo.tolist(), hi.tolist()):
        mask[a:b] = True
    c0 = pop.consts.detach().clone()
    c = c0.clone().requires_grad_(True)
    opt = torch.optim.Adam([c], lr=lr)
    sel = torch.zeros(pop.n_programs, dtype=torch.float32, device=dev)
    sel[progs] = -1.0 if larger else 1.0
    with torch.no_grad():
        f0 = GPFitness.apply(c0, pop, data, metric)
    for _ in range(steps):
        opt.zero_grad()
        fit = GPFitness.apply(c, pop, data, metric)
        loss = (torch.nan_to_num(fit, nan=0.0, posinf=0.0, neginf=0.0) * sel).sum()
        loss.backward()
        with torch.no_grad():
            c.grad = torch.nan_to_num(c.grad * mask, nan=0.0, posinf=0.0, neginf=0.0)
        opt.step()
    with torch.no_grad():
        c1 = c.detach()
        f1 = GPFitness.apply(c1, pop, data, metric)
        better = (f1 > f0) if larger else (f1 < f0)
        keep_prog = torch.zeros(pop.n_programs, dtype=torch.bool, device=dev)
        keep_prog[progs] = better[progs]
        # constant k belongs to the program p with const_off[p] <= k < const_off[p+1]
        owner = torch.repeat_interleave(torch.arange(pop.n_programs, device=dev), co[1:] - co[:-1])
        keep = keep_prog[owner] if owner.numel() else torch.zeros(0, dtype=torch.bool, device=dev)
        out = torch.where(keep, c1[:owner.numel()], c0[:owner.numel()])
        f_final = torch.where(keep_prog, f1, f0)
    return out, f0, f_final
