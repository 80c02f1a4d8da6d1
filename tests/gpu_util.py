"""Helpers for the GPU parity tests: run the same seeded workload through the
library (FP32, gfx950) and through the FP64 oracle, and compare."""
from __future__ import annotations

import os
import sys

import numpy as np

from oracle.oracle import OBJ_DFT, OBJ_TIME
from paper_2305_00234_amd.inputs import Workload
from tests.oracle_setup import oracle_from_workload


# Every measurement a GPU test prints, with the test that printed it; the
# session's terminal summary lists them (tests/conftest.py), so the errors
# behind a pass are visible in a quiet run too.
MEASURED: list[tuple[str, str]] = []


def say(*a):
    msg = " ".join(str(x) for x in a)
    test = os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0]
    MEASURED.append((test, msg))
    print(msg, flush=True)
    sys.stdout.flush()


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2305_00234_amd import lib
    lib.load()  # raises if the HIP library was not built: no fallback exists
    return torch


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


ETA0 = 376.730313668


def field_errors(gpu_fields, or_fields):
    """Relative L2 errors of the field state: (E, eta0 H) together in the
    energy norm (the parity bar), E alone and H alone (diagnostics)."""
    g = np.stack([np.asarray(f, np.float64) for f in gpu_fields])
    o = np.stack([np.asarray(f, np.float64) for f in or_fields])
    w = np.array([1, 1, 1, ETA0, ETA0, ETA0]).reshape(6, 1, 1, 1)
    state = rel_l2(g * w, o * w)
    return state, rel_l2(g[:3], o[:3]), rel_l2(g[3:], o[3:])


def gpu_fields_after_steps(w: Workload, steps: int, tile_planes=None, tile_rows=None):
    from paper_2305_00234_amd.solver import configure
    torch = require_gpu()
    s = configure(w)
    if tile_planes:
        s.set_tile_planes(tile_planes)
    if tile_rows:
        s.set_tile_rows(tile_rows)
    s.bind_torch(0)
    s.reset()
    s.step(steps)
    out = [s.field(c) for c in range(6)]
    torch.cuda.synchronize()
    s.close()
    return out


def oracle_fields_after_steps(w: Workload, steps: int):
    o = oracle_from_workload(w)
    o.reset()
    o.run(steps)
    return o.fields()


def gpu_gradient(w: Workload, tile_planes=None, checkpoint_every=None, want_adjoint_fields=False, resident=None):
    from paper_2305_00234_amd.solver import configure
    torch = require_gpu()
    s = configure(w)
    if tile_planes:
        s.set_tile_planes(tile_planes)
    if checkpoint_every is not None:
        s.set_checkpointing(checkpoint_every)
    if resident is not None:
        s.set_resident_segments(resident)
    s.bind_torch(w.steps)
    F = s.forward(w.steps)
    fwd = [s.field(c) for c in range(6)]
    s.adjoint()
    g = s.gradient()
    adj = [s.field(c) for c in range(6)] if want_adjoint_fields else None
    info = s.info()
    torch.cuda.synchronize()
    s.close()
    return F, g, fwd, adj, info


def oracle_gradient(w: Workload):
    o = oracle_from_workload(w)
    kind = OBJ_DFT if w.objective == "dft" else OBJ_TIME
    if w.gradient == "dft":
        F, g = o.gradient_dft(w.steps, w.gap_lo, w.gap_dims, w.omega)
    else:
        F, g = o.gradient(w.steps, kind, w.gap_lo, w.gap_dims, w.omega, w.window[0], w.window_end)
    fwd = o.forward_end_fields()    # the state at the end of the forward run
    adj = o.fields()                # the gradient call leaves the adjoint fields
    return F, g, fwd, adj


def fp32_storage_fields(w: Workload, marks):
    """The oracle's forward fields at the given steps (ascending) with every
    stored state word rounded to FP32 after each update (FP64 arithmetic):
    the floor that FP32 storage alone puts under any FP32 implementation of
    the same recurrence."""
    o = oracle_from_workload(w)
    o.set_fp32_storage(True)
    o.reset()
    out, n = [], 0
    for m in marks:
        o.run(m - n)
        n = m
        out.append(o.fields())
    return out


def _state(fields):
    """(6, nz, ny, nx) float64 state with H scaled by eta0 (energy norm)."""
    f = np.stack([np.asarray(x, np.float64) for x in fields])
    f[3:] *= ETA0
    return f


def region_masks(w: Workload):
    """Cell masks (nz, ny, nx) of the regions where local errors would be
    diluted in a whole-grid norm: the design box, the gap, the CPML slabs,
    the TF/SF shell (cells within one cell of the total-field box's faces),
    the far faces (the last two cell layers along each axis, where the
    kernels' tiles end ragged) and the rest of the grid."""
    nx, ny, nz = w.shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = {}
    lo, d = w.design_lo, w.design_dims
    e = 1 if w.rho_edges is not None else 0
    out["design"] = ((i >= lo[0]) & (i < lo[0] + d[0] + e) & (j >= lo[1]) & (j < lo[1] + d[1] + e) &
                     (k >= lo[2]) & (k < lo[2] + d[2] + e))
    g, gd = w.gap_lo, w.gap_dims
    out["gap"] = ((i >= g[0]) & (i < g[0] + gd[0]) & (j >= g[1]) & (j < g[1] + gd[1]) &
                  (k >= g[2]) & (k < g[2] + gd[2]))
    p = w.npml
    if p > 0:
        out["cpml"] = ((i < p) | (i >= nx - p) | (j < p) | (j >= ny - p) | (k < p) | (k >= nz - p))
    if w.source == "planewave":
        a, b = w.tfsf_lo, w.tfsf_hi
        near = np.zeros_like(out["gap"])
        inside = np.ones_like(out["gap"])
        for ax, q in ((0, i), (1, j), (2, k)):
            near |= (np.abs(q - a[ax]) <= 1) | (np.abs(q - b[ax]) <= 1)
            inside &= (q >= a[ax] - 1) & (q <= b[ax] + 1)
        out["tfsf_shell"] = near & inside
    out["far_faces"] = (i >= nx - 2) | (j >= ny - 2) | (k >= nz - 2)
    rest = np.ones_like(out["gap"])
    for m in out.values():
        rest &= ~m
    out["rest"] = rest
    return out


def region_errors(gpu_fields, or_fields, w: Workload):
    """Relative L2 error of the (E, eta0 H) state inside each region of
    region_masks, and the largest error of any field word over the state's
    peak ("max_abs/peak"), with each region's share of the state's norm."""
    g, o = _state(gpu_fields), _state(or_fields)
    d = g - o
    tot = np.linalg.norm(o)
    res = {"max_abs/peak": float(np.max(np.abs(d)) / np.max(np.abs(o)))}
    for name, m in region_masks(w).items():
        if not m.any():
            continue
        on = np.linalg.norm(o[:, m])
        res[name] = (float(np.linalg.norm(d[:, m]) / on) if on > 0 else float(np.linalg.norm(d[:, m])),
                     float(on / tot))
    return res


def fmt_regions(r):
    return ", ".join(f"{k} {v:.2e}" if not isinstance(v, tuple) else f"{k} {v[0]:.2e} (norm share {v[1]:.1e})"
                     for k, v in r.items())
