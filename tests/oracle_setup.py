"""Build FP64 oracle simulations from the seeded workloads (test helper)."""
from __future__ import annotations

import numpy as np

from oracle.oracle import OBJ_DFT, OBJ_TIME, OracleSim
from paper_2305_00234_amd.inputs import Workload


def oracle_from_workload(w: Workload, with_source: bool = True) -> OracleSim:
    nx, ny, nz = w.shape
    s = OracleSim(nx, ny, nz, w.dx, w.courant, w.npml, w.pml_m, w.pml_kappa_max,
                  w.pml_alpha_max, w.pml_sigma_scale)
    for ax in range(3):
        for slot, m in ((1, w.mat1[ax]), (2, w.mat2[ax])):
            s.set_material(slot, ax, m.eps_inf, m.sigma, m.a, m.c)
    if w.rho_edges is not None:
        s.set_design_edges(w.design_lo, w.design_dims, [r.astype(np.float64) for r in w.rho_edges],
                           w.gamma)
    else:
        s.set_design(w.design_lo, w.rho.astype(np.float64), w.gamma)
    if with_source:
        if w.source == "dipole":
            s.set_dipole(w.dipole_cell, w.dipole_axis, w.wave)
        else:
            s.set_planewave(w.pw_prop_axis, w.pw_sign, w.pw_pol_axis, w.tfsf_lo, w.tfsf_hi,
                            w.wave)
    return s


def oracle_gradient(w: Workload, want_hist: bool = False):
    s = oracle_from_workload(w)
    kind = OBJ_DFT if w.objective == "dft" else OBJ_TIME
    out = s.gradient(w.steps, kind, w.gap_lo, w.gap_dims, w.omega, w.window[0], w.window_end,
                     want_hist=want_hist)
    return (s,) + tuple(out)


def oracle_objective(w: Workload) -> float:
    s = oracle_from_workload(w)
    kind = OBJ_DFT if w.objective == "dft" else OBJ_TIME
    return s.objective(w.steps, kind, w.gap_lo, w.gap_dims, w.omega, w.window[0], w.window_end)
