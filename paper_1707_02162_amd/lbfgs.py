"""Batched L-BFGS ascent for REDO-GRAPE (an optimiser beside the gradient steps of
Sec. III; not the paper's method).

Every instance of the batch runs its own L-BFGS iteration on its fidelity F_U:
the direction comes from the two-loop recursion over its own history of at most
`m` pairs, the step from a backtracking line search (Armijo sufficient increase,
halving the step), and an instance whose search finds no acceptable step within
`halvings` trials keeps its point and starts its history again.  With the REDO
codes the objective is piecewise constant in the amplitudes (steps of the code
quantum eps) and the gradient is the adjoint's straight-through one: a step too
small to change any code leaves F exactly where it was, so the search never
halves below the step that moves the largest entry of the direction by eps/2,
and a trial counts only when it raises F strictly; at that smallest step any
strict increase is accepted.

The fidelities and gradients come from redo_grape_fidelity_grad, the directions,
trial points and history updates from the library's L-BFGS kernels; this module
only sequences the calls and keeps the per-instance bookkeeping.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import redo as R


def grape_lbfgs(table: R.RedoTable, u0: torch.Tensor, U_target: torch.Tensor, iters: int, m: int = 8,
                gamma0: float = 1e3, c1: float = 1e-4, halvings: int = 8, n_steps=None,
                precision: int = R.PREC_F32, goal: Optional[float] = None):
    """gamma0: the largest amplitude change of a step without curvature information (the
    first step, and after a reset).  Returns (u, F float64 [B], history: list of F per
    iteration, including the start)."""
    lib = R.lib()
    P_ = R._ptr
    x = u0.clone().contiguous()
    B = x.shape[0]
    P = x[0].numel()
    dev = x.device
    F, _, g = table.grape(x, U_target, n_steps=n_steps, precision=precision)
    S = torch.zeros((m, B, P), dtype=torch.float32, device=dev)
    Y = torch.zeros_like(S)
    rho = torch.zeros((m, B), dtype=torch.float64, device=dev)
    count = torch.zeros(B, dtype=torch.int32, device=dev)
    head = torch.zeros(B, dtype=torch.int32, device=dev)
    d = torch.empty_like(x)
    gd = torch.empty(B, dtype=torch.float64, device=dev)
    xt = torch.empty_like(x)
    shape = (B,) + (1,) * (x.dim() - 1)
    hist = [F.clone()]
    st = R._stream()
    for _ in range(iters):
        if goal is not None and bool(((1.0 - F) <= goal).all()):
            break
        R._check(lib.redo_lbfgs_direction(B, P, m, P_(g), P_(S), P_(Y), P_(rho), P_(count), P_(head), gamma0,
                                          P_(d), P_(gd), st))
        alpha = torch.ones(B, dtype=torch.float64, device=dev)
        # the smallest step: the largest entry of the direction moves by half a code quantum
        dmax = d.abs().reshape(B, -1).amax(dim=1).double()
        alpha_min = torch.clamp(0.5 * table.eps / torch.clamp(dmax, min=1e-300), max=1.0)
        done = torch.zeros(B, dtype=torch.bool, device=dev)
        xn, Fn, gn = x.clone(), F.clone(), g.clone()
        for _h in range(halvings):
            R._check(lib.redo_lbfgs_trial(B, P, P_(x), P_(d), P_(alpha), P_(xt), st))
            Ft, _, gt = table.grape(xt, U_target, n_steps=n_steps, precision=precision)
            last = alpha <= alpha_min
            ok = ~done & (Ft > F) & ((Ft >= F + c1 * alpha * gd) | last)
            xn = torch.where(ok.view(shape), xt, xn)
            gn = torch.where(ok.view(shape), gt, gn)
            Fn = torch.where(ok, Ft, Fn)
            done |= ok | last
            if bool(done.all()):
                break
            alpha = torch.where(done, alpha, torch.maximum(0.5 * alpha, alpha_min))
        done = Fn > F
        acc = done.to(torch.int32)
        R._check(lib.redo_lbfgs_push(B, P, m, P_(x), P_(xn), P_(g), P_(gn), P_(acc), P_(S), P_(Y), P_(rho),
                                     P_(count), P_(head), st))
        x, F, g = xn, Fn, gn
        hist.append(F.clone())
    return x, F, hist
