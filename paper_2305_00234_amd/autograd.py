"""Differentiable objective: rho -> F as a torch.autograd.Function.

The forward solve is the library's forward run (Eqs. Maxwells2 a-c, objective
Eq. Objective_analyitically_enhancement); the hand-written backward is the
adjoint run plus the time-exact gradient of Eq. Gradient_FDTD, read straight
into a device tensor.  Nothing here computes: it binds the density tensor,
launches the library's calls on torch's current stream and returns its
results.  Long time-domain runs use the solver's segment checkpoint /
recompute (set it with Solver.set_checkpointing, or let the solver pick the
segment count that fits its workspace).

Use a float64 density where the objective is in SI units: the gradient of the
time-domain objective is of order 1e-47 and underflows float32.  The solve
itself always runs in FP32 (the density is handed to it as float32).
"""
from __future__ import annotations

import torch

from .lib import Solver, filter_project, filter_project_edges, filter_project_grad, filter_project_grad_edges


class CCPRObjective(torch.autograd.Function):
    """F = CCPRObjective.apply(rho, solver, nsteps, design_lo, gamma).

    rho: CUDA tensor (dz, dy, dx) with values in [0, 1]; solver: a configured
    Solver with a bound workspace (materials, source and objective set);
    nsteps: leapfrog steps of the forward run.  Returns F as a 0-d float64
    tensor on rho's device.  backward() runs the adjoint and returns dF/drho
    in rho's dtype.
    """

    @staticmethod
    def forward(ctx, rho, solver: Solver, nsteps: int, design_lo, gamma: float):
        if not rho.is_cuda:
            raise ValueError("rho must be a CUDA tensor")
        r32 = rho.detach().to(torch.float32).contiguous()
        solver.set_design(design_lo, r32, gamma)
        F = solver.forward(int(nsteps))  # synchronises on the objective
        ctx.solver = solver
        ctx.rho_dtype = rho.dtype
        ctx.shape = rho.shape
        ctx.args = (int(nsteps), tuple(design_lo), float(gamma))
        ctx.serial = solver.forward_serial
        ctx.save_for_backward(r32)
        return torch.tensor(F, dtype=torch.float64, device=rho.device)

    @staticmethod
    def backward(ctx, grad_out):
        s: Solver = ctx.solver
        if s.forward_serial != ctx.serial:
            # the solver's forward state is no longer this node's: another
            # objective ran on the same solver since, or an earlier backward's
            # segment recompute overwrote the history (retain_graph): run this
            # node's forward again
            (r32,) = ctx.saved_tensors
            nsteps, lo, gamma = ctx.args
            s.set_design(lo, r32, gamma)
            s.forward(nsteps)
            ctx.serial = s.forward_serial
        s.adjoint()
        g = torch.empty(ctx.shape, dtype=torch.float64, device=grad_out.device)
        s.gradient(out=g)
        return (grad_out.to(torch.float64) * g).to(ctx.rho_dtype), None, None, None, None


def objective(rho, solver: Solver, nsteps: int, design_lo, gamma: float = 0.0):
    """Functional form of CCPRObjective.apply."""
    return CCPRObjective.apply(rho, solver, nsteps, design_lo, gamma)


class FilterProject(torch.autograd.Function):
    """rho_projected = FilterProject.apply(rho, radius, beta, eta): the cone
    filter (Eq. FilterFunction) and the smoothed Heaviside projection (Eq.
    Projection) of a CUDA density tensor (dz, dy, dx), computed by the
    library's kernels in FP32; the backward is the chain rule of Eq.
    GradientsFiltered, in FP64, returned in rho's dtype."""

    @staticmethod
    def forward(ctx, rho, radius: float, beta: float, eta: float):
        if not rho.is_cuda:
            raise ValueError("rho must be a CUDA tensor")
        r32 = rho.detach().to(torch.float32).contiguous()
        rt, rb, ws = filter_project(r32, radius, beta, eta)
        ctx.save_for_backward(rt, ws)
        ctx.params = (radius, beta, eta)
        ctx.rho_dtype = rho.dtype
        return rb.to(rho.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        rt, ws = ctx.saved_tensors
        radius, beta, eta = ctx.params
        g = filter_project_grad(grad_out.detach().to(torch.float64).contiguous(), rt, ws, radius, beta, eta)
        return g.to(ctx.rho_dtype), None, None, None


def filtered_objective(rho, solver: Solver, nsteps: int, design_lo, gamma: float, radius: float,
                       beta: float, eta: float = 0.5):
    """F(project(filter(rho))): the density the solver sees is the filtered and
    projected one; autograd chains Eq. GradientsFiltered after the adjoint
    gradient."""
    return CCPRObjective.apply(FilterProject.apply(rho, radius, beta, eta), solver, nsteps, design_lo, gamma)


# ---- per-edge design variables (one density per E edge, flat x, y, z edges
# of a dims-cell design; Sec. "FDTD implementation and design export")

class CCPREdgeObjective(torch.autograd.Function):
    """F = CCPREdgeObjective.apply(rho, solver, nsteps, design_lo, dims, gamma)
    for a flat CUDA tensor of per-edge densities (ccpr_set_design_edges
    layout); backward returns dF/drho per edge in rho's dtype."""

    @staticmethod
    def forward(ctx, rho, solver: Solver, nsteps: int, design_lo, dims, gamma: float):
        if not rho.is_cuda:
            raise ValueError("rho must be a CUDA tensor")
        r32 = rho.detach().to(torch.float32).contiguous()
        solver.set_design_edges(design_lo, dims, r32, gamma)
        F = solver.forward(int(nsteps))
        ctx.solver = solver
        ctx.rho_dtype = rho.dtype
        ctx.n = rho.numel()
        return torch.tensor(F, dtype=torch.float64, device=rho.device)

    @staticmethod
    def backward(ctx, grad_out):
        s: Solver = ctx.solver
        s.adjoint()
        g = torch.empty(ctx.n, dtype=torch.float64, device=grad_out.device)
        s.gradient(out=g)
        return (grad_out.to(torch.float64) * g).to(ctx.rho_dtype), None, None, None, None, None


class FilterProjectEdges(torch.autograd.Function):
    """FilterProject for per-edge densities: the cone filter over the
    staggered edge positions (all three components in the sphere) and the
    projection; backward is Eq. GradientsFiltered over the same sphere."""

    @staticmethod
    def forward(ctx, rho, dims, radius: float, beta: float, eta: float):
        if not rho.is_cuda:
            raise ValueError("rho must be a CUDA tensor")
        r32 = rho.detach().to(torch.float32).contiguous()
        rt, rb, ws = filter_project_edges(r32, dims, radius, beta, eta)
        ctx.save_for_backward(rt, ws)
        ctx.params = (tuple(dims), radius, beta, eta)
        ctx.rho_dtype = rho.dtype
        return rb.to(rho.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        rt, ws = ctx.saved_tensors
        dims, radius, beta, eta = ctx.params
        g = filter_project_grad_edges(grad_out.detach().to(torch.float64).contiguous(), rt, ws, dims, radius,
                                      beta, eta)
        return g.to(ctx.rho_dtype), None, None, None, None


def filtered_edge_objective(rho, solver: Solver, nsteps: int, design_lo, dims, gamma: float, radius: float,
                            beta: float, eta: float = 0.5):
    """F(project(filter(rho))) for per-edge densities (flat CUDA tensor)."""
    return CCPREdgeObjective.apply(FilterProjectEdges.apply(rho, dims, radius, beta, eta), solver, nsteps,
                                   design_lo, dims, gamma)
