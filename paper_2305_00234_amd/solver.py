"""Configure a library solver from a seeded workload description."""
from __future__ import annotations

from .inputs import Workload
from .lib import OBJ_DFT_E2, OBJ_TIME_E2, Solver


def configure(w: Workload, s: Solver | None = None) -> Solver:
    """Create (or reconfigure) a solver for workload w: grid, CPML, materials,
    design densities (host), source and objective.  No device work."""
    nx, ny, nz = w.shape
    if s is None:
        s = Solver(nx, ny, nz, w.dx, w.courant, w.npml, w.pml_m, w.pml_kappa_max,
                   w.pml_alpha_max, w.pml_sigma_scale)
    for ax in range(3):
        for slot, m in ((1, w.mat1[ax]), (2, w.mat2[ax])):
            s.set_material(slot, ax, m.eps_inf, m.sigma, m.a, m.c)
    if w.rho_edges is not None:
        s.set_design_edges(w.design_lo, w.design_dims, w.rho_edges, w.gamma)
    else:
        s.set_design(w.design_lo, w.rho, w.gamma)
    if w.source == "dipole":
        s.set_source_dipole(w.dipole_cell, w.dipole_axis, w.wave)
    else:
        s.set_source_planewave(w.pw_prop_axis, w.pw_sign, w.pw_pol_axis, w.tfsf_lo, w.tfsf_hi,
                               w.wave)
    kind = OBJ_DFT_E2 if w.objective == "dft" else OBJ_TIME_E2
    s.set_objective(kind, w.gap_lo, w.gap_dims, w.omega, w.window[0],
                    -1 if w.window[1] < 0 else w.window[1])
    if w.checkpoint_every:
        s.set_checkpointing(w.checkpoint_every)
    s.set_gradient_mode(w.gradient)
    return s


def solver_for(w: Workload, nsteps: int | None = None, device=None, extra_bytes: int = 0) -> Solver:
    """configure() plus a torch-allocated workspace sized for nsteps (default
    w.steps) bound with torch's current stream."""
    s = configure(w)
    s.bind_torch(w.steps if nsteps is None else nsteps, device=device, extra=extra_bytes)
    return s
