"""Seeded random small problems against the oracle: odd grid extents (ragged
wave lanes, y strips and z chunks), bare PEC or a CPML, per-voxel or per-edge
designs, random material pairs (vacuum, Drude, Lorentz, Table-1 sets,
diagonal anisotropy), a dipole of random axis and place, a gap inside or
outside the design, DFT or time-domain objective, conductivity damping on or
off.  Objective and time-exact gradient against the FP64 oracle."""
import math

import numpy as np
import pytest

from paper_2305_00234_amd import inputs as I
from tests.gpu_util import gpu_gradient, oracle_gradient, rel_l2, require_gpu, say

pytestmark = pytest.mark.gpu

C0 = 299792458.0


def _materials(rng):
    diel = I.lorentz(2.0 + rng.random(), 0.5 + rng.random(), 2 * math.pi * C0 / (200e-9 + 200e-9 * rng.random()),
                     1e14 * (0.5 + rng.random()))
    drude = I.drude(1.0, 1.37e16 * (0.8 + 0.4 * rng.random()), 1e14 * (0.5 + rng.random()))
    pool = [I.VACUUM, diel, drude, I.GOLD_TABLE1, I.ALUMINIUM_TABLE1, I.SILICON_TABLE1]
    m1 = pool[int(rng.integers(0, 3))]
    if rng.random() < 0.5:
        m2 = (pool[int(rng.integers(2, 6))],) * 3
    else:  # diagonal anisotropy: a different set per axis
        m2 = tuple(pool[int(k)] for k in rng.choice(np.arange(2, 6), size=3, replace=False))
    return (m1,) * 3, m2


def random_case(seed):
    rng = np.random.default_rng(1000 + seed)
    n = tuple(int(x) for x in rng.integers(18, 44, size=3))
    npml = int(rng.choice([0, 3, 5]))
    per_edge = bool(rng.random() < 0.5)
    steps = int(rng.integers(120, 260))
    w = I.drude_dipole_32(steps=steps, n=32, npml=npml, gamma=float(rng.choice([0.0, 5e4])), seed=seed)
    w.shape = n
    w.name = f"random_{seed}"
    w.mat1, w.mat2 = _materials(rng)
    m = max(npml, 1) + 2
    dims = tuple(int(rng.integers(3, max(4, (n[a] - 2 * m) // 2))) for a in range(3))
    lo = tuple(int(rng.integers(m, max(m + 1, n[a] - m - dims[a] - 1))) for a in range(3))
    w.design_lo = lo
    w.rho = rng.random((dims[2], dims[1], dims[0])).astype(np.float32)
    w.rho_edges = I.random_edge_densities(dims, seed=2000 + seed) if per_edge else None
    # gap: 1-2 cells, inside the design or beside it
    gd = tuple(int(rng.integers(1, 3)) for _ in range(3))
    if rng.random() < 0.6:
        w.gap_lo = tuple(int(lo[a] + rng.integers(0, max(1, dims[a] - gd[a]))) for a in range(3))
    else:
        w.gap_lo = tuple(int(max(m, lo[a] - gd[a] - 1)) for a in range(3))
    w.gap_dims = gd
    # dipole: random axis, outside the CPML, off the walls
    w.dipole_axis = int(rng.integers(0, 3))
    w.dipole_cell = tuple(int(rng.integers(m, n[a] - m)) for a in range(3))
    t = (np.arange(steps) + 0.5) * w.dt
    lam = 300e-9 + 400e-9 * rng.random()
    w.wave = I.gaussian_sine(t, lam, 1.0e-15, 1.5e-15, amp=1e9)
    w.omega = 2 * math.pi * C0 / lam
    if rng.random() < 0.5:
        w.objective = "time"
        w.window = (int(rng.integers(0, steps // 3)), -1)
    else:
        w.objective = "dft"
    return w


@pytest.mark.parametrize("seed", range(24))
def test_random_config_matches_oracle(seed):
    require_gpu()
    w = random_case(seed)
    F, g, _, _, _ = gpu_gradient(w)
    Fo, go, _, _ = oracle_gradient(w)
    flat = (lambda x: np.concatenate([np.ravel(a) for a in x])) if w.rho_edges is not None else np.ravel
    err = rel_l2(flat(g), flat(go))
    say("random", seed, w.shape, "npml", w.npml, "edges" if w.rho_edges is not None else "voxels",
        w.objective, "dipole", w.dipole_axis, w.dipole_cell, "F", F, Fo, "grad", err)
    assert Fo > 0 and abs(F - Fo) <= 1e-5 * abs(Fo)
    assert err <= 1e-3


def random_planewave_case(seed):
    """A TF/SF plane wave of random axis, direction and polarisation around a
    random design (inside the total-field box, which lies in the
    background); DFT objective, time-exact or DFT-mode gradient."""
    rng = np.random.default_rng(5000 + seed)
    w = random_case(seed + 100)
    n = w.shape
    npml = w.npml
    d = w.design_dims
    box = 1 if w.rho_edges is not None else 0
    # TF/SF box [tl, th] strictly inside the grid and outside the CPML, with
    # the design (and the gap) at least one cell inside it
    tl, th = [], []
    for a in range(3):
        lo_min, hi_max = npml + 1, n[a] - npml - 2
        dl, dh = w.design_lo[a], w.design_lo[a] + d[a] + box
        gl, gh = w.gap_lo[a], w.gap_lo[a] + w.gap_dims[a]
        inner_lo, inner_hi = min(dl, gl) - 1, max(dh, gh) + 1
        tl.append(int(rng.integers(lo_min, max(lo_min + 1, inner_lo + 1))) if inner_lo >= lo_min else lo_min)
        th.append(int(rng.integers(min(inner_hi, hi_max), hi_max + 1)))
    w.source = "planewave"
    w.tfsf_lo, w.tfsf_hi = tuple(tl), tuple(th)
    w.pw_prop_axis = int(rng.integers(0, 3))
    w.pw_sign = int(rng.choice([-1, 1]))
    w.pw_pol_axis = int(rng.choice([a for a in range(3) if a != w.pw_prop_axis]))
    t = np.arange(w.steps + 1) * w.dt
    lam = 2 * math.pi * C0 / w.omega
    w.wave = I.gaussian_sine(t, lam, 1.0e-15, 1.5e-15, amp=1.0)
    w.objective = "dft"
    w.gradient = "dft" if rng.random() < 0.4 else "time"
    if w.gradient == "dft":
        w.steps = max(w.steps, 400)
        t = np.arange(w.steps + 1) * w.dt
        w.wave = I.gaussian_sine(t, lam, 1.0e-15, 1.5e-15, amp=1.0)
    return w


def _tfsf_ok(w):
    """Whether the TF/SF box keeps the design and gap strictly inside and
    stays strictly inside the grid outside the CPML."""
    d, box = w.design_dims, 1 if w.rho_edges is not None else 0
    for a in range(3):
        if not (w.npml + 1 <= w.tfsf_lo[a] < w.tfsf_hi[a] <= w.shape[a] - w.npml - 2):
            return False
        lo = min(w.design_lo[a], w.gap_lo[a])
        hi = max(w.design_lo[a] + d[a] + box, w.gap_lo[a] + w.gap_dims[a])
        if not (w.tfsf_lo[a] < lo and hi < w.tfsf_hi[a]):
            return False
    return True


PW_SEEDS = [s for s in range(40) if _tfsf_ok(random_planewave_case(s))][:12]


@pytest.mark.parametrize("seed", PW_SEEDS)
def test_random_planewave_config_matches_oracle(seed):
    require_gpu()
    w = random_planewave_case(seed)
    F, g, _, _, _ = gpu_gradient(w)
    Fo, go, _, _ = oracle_gradient(w)
    flat = (lambda x: np.concatenate([np.ravel(a) for a in x])) if w.rho_edges is not None else np.ravel
    err = rel_l2(flat(g), flat(go))
    say("random plane wave", seed, w.shape, "npml", w.npml, "prop", w.pw_prop_axis, w.pw_sign, "pol",
        w.pw_pol_axis, "tfsf", w.tfsf_lo, w.tfsf_hi, "gradient", w.gradient, "F", F, Fo, "grad", err)
    assert Fo > 0 and abs(F - Fo) <= 1e-5 * abs(Fo)
    assert err <= 1e-3


@pytest.mark.parametrize("seed", range(6))
def test_random_segmentation_bitwise(seed):
    """Random problems with the time-domain objective, run with a random
    segment length and number of resident segments: objective and gradient
    bit for bit those of the whole history (the recompute is deterministic)."""
    require_gpu()
    rng = np.random.default_rng(7000 + seed)
    w = random_case(seed + 200)
    w.objective = "time"
    w.window = (int(rng.integers(0, w.steps // 3)), -1)
    every = int(rng.integers(7, max(8, w.steps // 2)))
    resident = int(rng.integers(1, 4))
    F1, g1, _, _, _ = gpu_gradient(w)
    F2, g2, _, _, info = gpu_gradient(w, checkpoint_every=every, resident=resident)
    flat = (lambda x: np.concatenate([np.ravel(a) for a in x])) if w.rho_edges is not None else np.ravel
    say("segmentation", seed, w.shape, "every", every, "resident", resident, info)
    assert info["segment_steps"] == every and info["resident_segments"] == min(resident, info["segments"])
    assert F1 == F2
    assert np.array_equal(flat(g1), flat(g2))


@pytest.mark.parametrize("seed", range(4))
def test_random_launch_shape_bitwise(seed):
    """Random problems: the fields after the run do not depend on the launch
    shape (z-chunk height, rows per thread), bit for bit."""
    require_gpu()
    from tests.gpu_util import gpu_fields_after_steps
    rng = np.random.default_rng(8000 + seed)
    w = random_case(seed + 300)
    steps = min(w.steps, 120)
    ref = gpu_fields_after_steps(w, steps)
    for planes, rows in ((int(rng.integers(2, 9)), 2), (int(rng.integers(2, 9)), 4)):
        got = gpu_fields_after_steps(w, steps, tile_planes=planes, tile_rows=rows)
        say("launch shape", seed, w.shape, "planes", planes, "rows", rows)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("seed", range(6))
def test_random_filter_matches_oracle(seed):
    """Random design sizes, radii (1-8 voxels), sharpness and thresholds, per
    voxel and per edge: filtered densities, projection and the chain rule
    against the FP64 oracle (relative 1e-5)."""
    torch = require_gpu()
    from oracle import filters as OF
    from paper_2305_00234_amd.lib import (filter_project, filter_project_edges, filter_project_grad,
                                          filter_project_grad_edges)
    rng = np.random.default_rng(9000 + seed)
    dims = tuple(int(x) for x in rng.integers(3, 24, size=3))
    R = float(1.0 + 7.0 * rng.random())
    beta, eta = float(1.0 + 15.0 * rng.random()), float(0.2 + 0.6 * rng.random())
    if seed % 2 == 0:
        rho = rng.random((dims[2], dims[1], dims[0])).astype(np.float32)
        gb = rng.standard_normal(rho.shape)
        rt, rb, ws = filter_project(torch.tensor(rho, device="cuda"), R, beta, eta)
        g = filter_project_grad(torch.tensor(gb, device="cuda"), rt, ws, R, beta, eta)
        ot = OF.cone_filter(rho.astype(np.float64), R)
        og = OF.filter_project_grad(gb, rho.astype(np.float64), R, beta, eta)
        ot_flat, og_flat = ot.ravel(), og.ravel()
    else:
        parts = [rng.random(OF.edge_shape(dims, c)) for c in range(3)]
        rho = np.concatenate([p.ravel() for p in parts]).astype(np.float32)
        gparts = [rng.standard_normal(OF.edge_shape(dims, c)) for c in range(3)]
        gb = np.concatenate([p.ravel() for p in gparts])
        rt, rb, ws = filter_project_edges(torch.tensor(rho, device="cuda"), dims, R, beta, eta)
        g = filter_project_grad_edges(torch.tensor(gb, device="cuda"), rt, ws, dims, R, beta, eta)
        split, o = [], 0
        for c in range(3):
            n = int(np.prod(OF.edge_shape(dims, c)))
            split.append(rho[o:o + n].astype(np.float64).reshape(OF.edge_shape(dims, c)))
            o += n
        ot_flat = np.concatenate([x.ravel() for x in OF.cone_filter_edges(split, dims, R)])
        og_flat = np.concatenate([x.ravel() for x in OF.filter_project_grad_edges(gparts, split, dims, R, beta, eta)])
    torch.cuda.synchronize()
    rt_h = rt.cpu().numpy().ravel()
    e_t = rel_l2(rt_h, ot_flat)
    e_b = rel_l2(rb.cpu().numpy().ravel(), OF.project(rt_h.astype(np.float64), beta, eta))
    e_g = rel_l2(g.cpu().numpy().ravel(), og_flat)
    say("random filter", seed, dims, "R", round(R, 2), "beta", round(beta, 2), "eta", round(eta, 2),
        "edges" if seed % 2 else "voxels", "rho_t", e_t, "rho_b", e_b, "chain", e_g)
    assert e_t <= 1e-5 and e_b <= 1e-5 and e_g <= 1e-5
