"""torch.autograd.Function around one step of the scheme, with the
hand-written adjoint of librelsim as its backward (FP64 contexts only).

One step maps (offsets, momenta, E^n, B^n) to the next state.  The forward
runs the library's deposit, field solve and push with re-sort, and records
the permutation of the re-sort; autograd keeps the step's inputs alive, which
are exactly the per-step checkpoints (particle state, E^n, B^n) plus E_theta.
The backward reloads the checkpoint, re-deposits M (needed by the transposed
solve), and calls relsim_push_adjoint, relsim_field_solve_adjoint and
relsim_deposit_adjoint.  Offsets are in cell units; their gradients are the
library's physical-position cotangents times the cell size.
"""
from __future__ import annotations

import math
from typing import Optional

import torch

from . import relsim


class Stepper:
    """Work buffers for differentiable steps on one FP64 context."""

    def __init__(self, ctx: relsim.Context):
        if ctx.precision != "fp64":
            raise ValueError("the adjoint needs an FP64 context")
        self.ctx = ctx
        self.parts = relsim.Particles(ctx)
        self.J = ctx.grid()
        self.M = ctx.mass_matrix()
        self.h = [ctx.params.dx, ctx.params.dy, ctx.params.dz][: ctx.dim]
        self.solve_iters = []

    def load(self, off, u, w, cell, bin_start):
        """Copy a state (device tensors) into the front buffers."""
        p = self.parts
        n = w.numel()
        if n > p.capacity:
            raise ValueError("state larger than the context's max_particles")
        f = p.sets[p.front]
        p.n = n
        for d in range(self.ctx.dim):
            f["xy"][:n, d].copy_(off[d])
        for k in range(3):
            f["uw"][:n, k].copy_(u[k])
        f["uw"][:n, 3].copy_(w)
        f["cell"][:n].copy_(cell)
        f["bin_start"].copy_(bin_start)
        p._bind()


class StepFn(torch.autograd.Function):
    """(off [dim][n], u [3][n], E [3][N], B [3][N]; cell, bin_start, w)
    -> (off', u', E', B', cell', bin_start', w')"""

    @staticmethod
    def forward(fctx, stepper: Stepper, off, u, E, B, cell, bin_start, w):
        ctx, p = stepper.ctx, stepper.parts
        stepper.load(off, u, w, cell, bin_start)
        relsim.deposit_moments(ctx, p, B, stepper.J, stepper.M)
        Eth, E1, B1, it, rr = relsim.field_solve(ctx, stepper.M, stepper.J, E.contiguous(), B.contiguous())
        stepper.solve_iters.append(it)
        perm = torch.empty(w.numel(), dtype=torch.int32, device=ctx.device)
        relsim.push(ctx, p, Eth, B.contiguous(), resort=True, new_index=perm)
        off1 = torch.stack([t.clone() for t in p.off])
        u1 = torch.stack([t.clone() for t in p.u])
        cell1 = p.cell.clone()
        bin1 = p.bin_start.clone()
        w1 = p.w.clone()
        fctx.stepper = stepper
        fctx.save_for_backward(off, u, E, B, cell, bin_start, w, Eth, perm)
        fctx.mark_non_differentiable(cell1, bin1, w1)
        return off1, u1, E1, B1, cell1, bin1, w1

    @staticmethod
    def backward(fctx, g_off1, g_u1, g_E1, g_B1, _gc, _gb, _gw):
        stepper = fctx.stepper
        ctx, p = stepper.ctx, stepper.parts
        off, u, E, B, cell, bin_start, w, Eth, perm = fctx.saved_tensors
        n = w.numel()
        dim = ctx.dim
        dev = ctx.device
        f64 = dict(dtype=torch.float64, device=dev)
        stepper.load(off, u, w, cell, bin_start)
        B = B.contiguous()
        relsim.deposit_moments(ctx, p, B, stepper.J, stepper.M)
        h = torch.tensor(stepper.h, **f64)[:, None]
        lx_in = (g_off1 / h).contiguous() if g_off1 is not None else torch.zeros((dim, n), **f64)
        lu_in = g_u1.contiguous() if g_u1 is not None else torch.zeros((3, n), **f64)
        lE1 = g_E1.contiguous() if g_E1 is not None else ctx.grid()
        lB1 = g_B1.contiguous() if g_B1 is not None else ctx.grid()
        lx = torch.empty((dim, n), **f64)
        lu = torch.empty((3, n), **f64)
        lEth, lB, lE, mu = ctx.grid(), ctx.grid(), ctx.grid(), ctx.grid()
        relsim.push_adjoint(ctx, p, Eth, B, perm, lx_in, lu_in, lx, lu, lEth, lB)
        relsim.field_solve_adjoint(ctx, stepper.M, lEth, lE1, lB1, mu, lE, lB)
        relsim.deposit_adjoint(ctx, p, B, Eth, mu, lx, lu, lB)
        return None, lx * h, lu, lE, lB, None, None, None


class FieldEnergyFn(torch.autograd.Function):
    """F = V/(8 pi) (sum |E|^2 + sum |B|^2) by relsim_energy; dF/dE = V E/(4 pi)."""

    @staticmethod
    def forward(fctx, stepper: Stepper, E, B):
        ctx = stepper.ctx
        W = relsim.energy(ctx, stepper.parts, E.contiguous(), B.contiguous())
        fctx.save_for_backward(E, B)
        fctx.V = float(ctx.params.dx * ctx.params.dy * (ctx.params.dz if ctx.dim == 3 else 1.0))
        return torch.tensor(W[1] + W[2], dtype=torch.float64, device=E.device)

    @staticmethod
    def backward(fctx, g):
        E, B = fctx.saved_tensors
        s = g * fctx.V / (4.0 * math.pi)
        return None, s * E, s * B


def field_energy_after(stepper: Stepper, off, u, E, B, cell, bin_start, w, steps: int):
    """Differentiable field energy after `steps` steps from the given state."""
    for _ in range(steps):
        off, u, E, B, cell, bin_start, w = StepFn.apply(stepper, off, u, E, B, cell, bin_start, w)
    return FieldEnergyFn.apply(stepper, E, B)
