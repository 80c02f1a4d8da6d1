"""A small density-based topology-optimisation loop around the library (Sec.
"Topology Optimization Setup" and Sec. "Filtering and projection"): each
iteration filters and projects the design variables (Eqs. FilterFunction,
Projection), runs the forward and adjoint solves, chains the gradient back
through the projection and the filter (Eq. GradientsFiltered), reports the
measure of non-discreteness (Eq. MeasureOfNon-discretness), and raises the
projection sharpness beta on a schedule (beta continuation).  All of that
runs in the library's kernels; the design update itself is a plain host-side
normalised gradient-ascent step with a move limit -- the paper's MMA
optimiser is not part of this package.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

from .inputs import Workload, voxel_edge_densities
from .lib import (edge_count, filter_project, filter_project_edges, filter_project_grad,
                  filter_project_grad_edges, nondiscreteness)
from .solver import configure


@dataclasses.dataclass
class Iteration:
    index: int
    objective: float
    beta: float
    nondiscreteness: float
    max_step: float


def optimize(w: Workload, iterations: int, radius: float, beta0: float = 2.0, beta_max: float = 32.0,
             beta_every: int = 5, move: float = 0.1, eta: float = 0.5, per_edge: bool = False):
    """Maximise the workload's objective over its design densities (w.rho is
    the start; with per_edge, one density per E edge as in Sec. "FDTD
    implementation and design export", started from w.rho_edges, or from
    w.rho copied to the edges each voxel owns and 0.5 on the far faces).
    Returns (rho, history): the final design variables (numpy float64 in
    [0, 1]: voxel array, or the flat per-edge vector) and one Iteration
    record per step."""
    import torch
    if per_edge and w.rho_edges is None:
        # the solver's workspace is sized for the per-edge layout from the start
        w = dataclasses.replace(w, rho_edges=voxel_edge_densities(w.rho, fill=0.5))
    s = configure(w)
    s.bind_torch(w.steps)
    dims = w.design_dims
    if per_edge:
        rho = np.clip(np.concatenate([np.asarray(r, np.float64).ravel() for r in w.rho_edges]), 0.0, 1.0)
        assert rho.size == edge_count(dims)
    else:
        rho = np.clip(np.asarray(w.rho, dtype=np.float64), 0.0, 1.0)
    beta = beta0
    hist: List[Iteration] = []
    try:
        for it in range(iterations):
            r32 = torch.tensor(rho, dtype=torch.float32, device="cuda")
            if per_edge:
                rt, rb, ws = filter_project_edges(r32, dims, radius, beta, eta)
                s.set_design_edges(w.design_lo, dims, rb, w.gamma)
            else:
                rt, rb, ws = filter_project(r32, radius, beta, eta)
                s.set_design(w.design_lo, rb, w.gamma)
            F = s.forward(w.steps)
            s.adjoint()
            g_b = torch.empty(rb.shape, dtype=torch.float64, device="cuda")
            s.gradient(out=g_b)
            if per_edge:
                g = filter_project_grad_edges(g_b, rt, ws, dims, radius, beta, eta).cpu().numpy()
            else:
                g = filter_project_grad(g_b, rt, ws, radius, beta, eta).cpu().numpy()
            mnd = nondiscreteness(rb)
            gmax = float(np.max(np.abs(g)))
            step = move / gmax if gmax > 0 else 0.0
            new = np.clip(rho + step * g, 0.0, 1.0)
            hist.append(Iteration(it, F, beta, mnd, float(np.max(np.abs(new - rho)))))
            rho = new
            if (it + 1) % beta_every == 0:
                beta = min(2.0 * beta, beta_max)
    finally:
        s.close()
    return rho, hist
