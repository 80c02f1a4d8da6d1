"""Per-edge design variables on the GPU (one density per E edge, N_l + 1 -
delta_kl edges of component k along axis l; Sec. "FDTD implementation and
design export") against the FP64 oracle, through the C-ABI: fields, the
time-exact and DFT-mode gradients (one value per edge, far-face edges
included), device-resident densities, the reduction to a per-voxel design
and the x <-> y mirror symmetry of the gradient."""
import math

import numpy as np
import pytest

from paper_2305_00234_amd import inputs as I
from tests.gpu_util import (field_errors, gpu_fields_after_steps, gpu_gradient, oracle_fields_after_steps,
                            oracle_gradient, rel_l2, require_gpu, say)

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-5
GRAD_TOL = 1e-3
C0 = 299792458.0


def _flat(g):
    return np.concatenate([np.asarray(x, np.float64).ravel() for x in g])


def _aniso_dipole_case(steps=300, gradient="time", seed=41):
    """CPML grid with ragged extents, a 13 x 11 x 9 per-edge design of a
    Lorentz dielectric (rho = 0) and a diagonal-anisotropic metal (rho = 1:
    x gold, y aluminium set, z gold with Im a x 1.1), gamma = 5e4, an x dipole
    beside the design and a 2^3 air gap inside it."""
    w = I.drude_dipole_32(steps=steps, n=40, npml=6, gamma=5e4)
    w.shape = (40, 37, 34)
    diel = I.lorentz(2.1, 1.0, 2 * math.pi * C0 / 150e-9, 1e14)
    w.mat1 = (diel, diel, diel)
    w.mat2 = (I.GOLD_TABLE1, I.ALUMINIUM_TABLE1, I.GOLD_TABLE1.scaled_imag_a(1.1))
    w.design_lo = (12, 11, 10)
    dims = (13, 11, 9)
    w.rho_edges = I.random_edge_densities(dims, seed)
    w.gap_lo, w.gap_dims = (17, 15, 13), (2, 2, 2)
    g0 = [w.gap_lo[a] - w.design_lo[a] for a in range(3)]
    for r in w.rho_edges:  # edges of the gap cells stay air
        r[g0[2]:g0[2] + 2, g0[1]:g0[1] + 2, g0[0]:g0[0] + 2] = 0.0
    w.rho = np.zeros((dims[2], dims[1], dims[0]), np.float32)  # unused: the design is per edge
    w.dipole_cell, w.dipole_axis = (9, 16, 14), 0
    w.gradient = gradient
    return w


def test_edge_design_fields_match_oracle():
    require_gpu()
    w = _aniso_dipole_case()
    g = gpu_fields_after_steps(w, 80)
    o = oracle_fields_after_steps(w, 80)
    st, eE, eH = field_errors(g, o)
    say("per-edge design fields: state", st, "E", eE, "H", eH)
    assert st <= FIELD_TOL


@pytest.mark.parametrize("gradient", ["time", "dft"])
def test_edge_gradient_matches_oracle(gradient):
    require_gpu()
    w = _aniso_dipole_case(steps=300 if gradient == "time" else 600, gradient=gradient)
    F, g, _, _, info = gpu_gradient(w)
    Fo, go, _, _ = oracle_gradient(w)
    assert isinstance(g, tuple) and len(g) == 3
    for c in range(3):
        assert g[c].shape == I.edge_shape(w.design_dims, c) == go[c].shape
    err = rel_l2(_flat(g), _flat(go))
    # far-face edges (the ones a per-voxel layout lacks) on their own
    nx, ny, nz = w.design_dims
    far = np.concatenate([g[0][nz, :, :].ravel(), g[0][:, ny, :].ravel(), g[1][:, :, nx].ravel(),
                          g[2][:, :, nx].ravel()])
    far_o = np.concatenate([go[0][nz, :, :].ravel(), go[0][:, ny, :].ravel(), go[1][:, :, nx].ravel(),
                            go[2][:, :, nx].ravel()])
    say(gradient, "F", F, Fo, "grad rel L2", err, "far-face rel L2", rel_l2(far, far_o), info)
    assert abs(F - Fo) <= 1e-5 * abs(Fo)
    assert err <= GRAD_TOL
    assert rel_l2(far, far_o) <= GRAD_TOL
    assert np.max(np.abs(far_o)) > 1e-3 * np.max(np.abs(_flat(go)))  # far faces do carry gradient


def test_edge_gradient_planewave_time_objective():
    """TF/SF plane wave, time-domain objective over a window, CPML on all
    sides, gold per-edge design; time-exact gradient."""
    require_gpu()
    w = I.gold_gap(n=(48, 44, 40), design=(16, 14, 10), npml=8, steps=500, seed=3, objective="time",
                   name="gold_gap_edges_48")
    w.window = (50, 450)
    dims = w.design_dims
    w.rho_edges = I.random_edge_densities(dims, seed=43)
    F, g, _, _, info = gpu_gradient(w)
    Fo, go, _, _ = oracle_gradient(w)
    err = rel_l2(_flat(g), _flat(go))
    say("plane wave per-edge: F", F, Fo, "grad rel L2", err)
    assert abs(F - Fo) <= 1e-5 * abs(Fo)
    assert err <= GRAD_TOL


def test_edge_design_from_device_memory_is_identical():
    """Densities handed over as one flat device tensor give the same solve as
    host arrays, bit for bit."""
    torch = require_gpu()
    from paper_2305_00234_amd.solver import configure
    w = _aniso_dipole_case(steps=120)
    F_h, g_h, _, _, _ = gpu_gradient(w)
    s = configure(w)
    s.bind_torch(w.steps)
    flat = torch.tensor(np.concatenate([r.ravel() for r in w.rho_edges]), device="cuda")
    s.set_design_edges(w.design_lo, w.design_dims, flat, w.gamma)
    F_d = s.forward(w.steps)
    s.adjoint()
    out = torch.empty(s.gradient_size, dtype=torch.float64, device="cuda")
    s.gradient(out=out)
    g_d = out.cpu().numpy()
    s.close()
    assert F_d == F_h
    assert np.array_equal(g_d, _flat(g_h))


def test_edge_design_reduces_to_voxel_design():
    """Edge densities copied from a per-voxel design (zero on the far faces,
    vacuum rho = 0 material): same objective, and each voxel's gradient is
    the sum of its three edges' gradients."""
    require_gpu()
    w = I.drude_dipole_32(steps=300)
    F_v, g_v, _, _, _ = gpu_gradient(w)
    w.rho_edges = I.voxel_edge_densities(w.rho, fill=0.0)
    F_e, g_e, _, _, _ = gpu_gradient(w)
    nz, ny, nx = w.rho.shape
    summed = sum(np.asarray(x)[:nz, :ny, :nx] for x in g_e)
    say("voxel vs edge: F", F_v, F_e, "grad rel L2", rel_l2(summed, g_v))
    assert abs(F_e - F_v) <= 1e-6 * abs(F_v)
    assert rel_l2(summed, g_v) <= 1e-5


def test_edge_gradient_mirror_symmetry_and_oracle():
    """A problem invariant under x <-> y (square grid and CPML, diagonal
    design and gap, z dipole on the diagonal, identical x and y materials):
    the GPU gradient has g_x(k,j,i) = g_y(k,i,j) and a symmetric g_z to FP32
    accuracy, and matches the oracle."""
    require_gpu()
    w = I.drude_dipole_32(steps=400, n=56, npml=8, gamma=5e4)
    w.shape = (56, 56, 44)
    diel = I.lorentz(2.0, 1.2, 2 * math.pi * C0 / 250e-9, 2e14)
    w.mat1 = (diel, diel, diel)
    w.mat2 = (I.GOLD_TABLE1, I.GOLD_TABLE1, I.ALUMINIUM_TABLE1)
    w.design_lo = (20, 20, 14)
    dims = (15, 15, 12)
    ex, _, ez = I.random_edge_densities(dims, seed=44)
    ey = np.ascontiguousarray(ex.transpose(0, 2, 1))
    ez = (0.5 * (ez.astype(np.float64) + ez.transpose(0, 2, 1))).astype(np.float32)
    w.rho_edges = (ex, ey, ez)
    w.rho = np.zeros((dims[2], dims[1], dims[0]), np.float32)
    w.gap_lo, w.gap_dims = (26, 26, 19), (3, 3, 2)
    w.dipole_cell, w.dipole_axis = (14, 14, 20), 2
    F, g, _, _, _ = gpu_gradient(w)
    Fo, go, _, _ = oracle_gradient(w)
    scale = np.max(np.abs(_flat(g)))
    asym_x = np.max(np.abs(g[0] - g[1].transpose(0, 2, 1))) / scale
    asym_z = np.max(np.abs(g[2] - g[2].transpose(0, 2, 1))) / scale
    err = rel_l2(_flat(g), _flat(go))
    say("mirror: F", F, Fo, "asym x/y", asym_x, "asym z", asym_z, "grad rel L2", err)
    assert abs(F - Fo) <= 1e-5 * abs(Fo)
    assert err <= GRAD_TOL
    assert asym_x <= 1e-4 and asym_z <= 1e-4


@pytest.mark.parametrize("axis", [0, 1])
def test_edge_design_dipole_on_far_face(axis):
    """A dipole on the far x face of the per-edge box (cell lo_x + N_x): along
    x that edge is not a design edge (vacuum, driven through the FP64 source
    shadow), along y it is a dispersive design edge carrying the source."""
    require_gpu()
    w = _aniso_dipole_case(steps=250)
    lo, d = w.design_lo, w.design_dims
    w.dipole_cell, w.dipole_axis = (lo[0] + d[0], lo[1] + 3, lo[2] + 4), axis
    g = gpu_fields_after_steps(w, 120)
    o = oracle_fields_after_steps(w, 120)
    st, _, _ = field_errors(g, o)
    F, gg, _, _, _ = gpu_gradient(w)
    Fo, go, _, _ = oracle_gradient(w)
    err = rel_l2(_flat(gg), _flat(go))
    say("far-face dipole axis", axis, "fields", st, "F", F, Fo, "grad rel L2", err)
    assert st <= FIELD_TOL
    assert abs(F - Fo) <= 1e-5 * abs(Fo)
    assert err <= GRAD_TOL


def test_edge_gradient_checkpointed_bitwise():
    """Per-edge design, time objective: segments recomputed from checkpoints
    (one resident segment), some resident, or the whole history give the
    same gradient bit for bit."""
    require_gpu()
    w = _aniso_dipole_case(steps=210)
    w.objective = "time"
    w.window = (20, 200)
    F1, g1, _, _, i1 = gpu_gradient(w)
    for resident in (1, 2):
        F2, g2, _, _, i2 = gpu_gradient(w, checkpoint_every=50, resident=resident)
        say("per-edge checkpointing", i1, i2)
        assert i2["segments"] == 5 and i2["resident_segments"] == resident
        assert F1 == F2
        assert np.array_equal(_flat(g1), _flat(g2))
