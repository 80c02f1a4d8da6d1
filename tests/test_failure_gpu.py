"""Failure detection forced from the host, with every kernel exiting
normally: a non-passive material (negative static susceptibility) makes the
fields grow; the divergence watchdog (a check of the gap box every 64
steps) stops the run long before its end and ccpr_forward reports
CCPR_EDIVERGED, the adjoint refuses to run on that solve, and the solver
runs again once the material is passive."""
import math

import numpy as np
import pytest

from paper_2305_00234_amd import inputs as I
from tests.gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu

C0 = 299792458.0


def test_active_medium_reports_divergence_and_recovers():
    require_gpu()
    from paper_2305_00234_amd import lib as L
    from paper_2305_00234_amd.solver import configure
    w = I.drude_dipole_32(steps=2000, n=24, npml=0, gamma=0.0)
    w.design_lo = (8, 8, 8)
    w.rho = np.ones((8, 8, 8), np.float32)
    w.gap_lo, w.gap_dims = (11, 11, 11), (2, 2, 2)
    w.dipole_cell = (6, 12, 12)
    active = I.lorentz(1.0, -3.0, 2 * math.pi * C0 / 500e-9, 1e13)  # static eps 1 - 3 < 0
    w.mat2 = (active,) * 3
    s = configure(w)
    s.bind_torch(w.steps)
    s.set_watchdog(64)
    with pytest.raises(L.CcprError) as e:
        s.forward(w.steps)
    say("active medium:", e.value, "steps done when it tripped:", s.step_count)
    assert e.value.status == L.EDIVERGED
    # the watchdog stopped the run well before its end (the steps after it
    # are skipped on the device)
    assert 0 < s.step_count < w.steps and s.step_count % 64 == 0
    with pytest.raises(L.CcprError) as e:
        s.adjoint()
    assert e.value.status == L.ESTATE
    # a passive material on the same solver and workspace runs normally
    for ax in range(3):
        m = I.GOLD_TABLE1
        s.set_material(2, ax, m.eps_inf, m.sigma, m.a, m.c)
    F = s.forward(w.steps)
    s.adjoint()
    g = s.gradient()
    s.close()
    say("passive again: F", F)
    assert np.isfinite(F) and F > 0 and np.all(np.isfinite(g))


def test_invalid_device_densities_reported_at_the_next_run():
    """Densities handed over in device memory are checked on the device (the
    host cannot see them without a copy): a NaN or a value above 1 is
    reported by the next forward run as CCPR_EINVAL, for per-voxel and
    per-edge designs alike, and valid densities then run normally."""
    torch = require_gpu()
    from paper_2305_00234_amd import lib as L
    from paper_2305_00234_amd.solver import configure
    w = I.drude_dipole_32(steps=120)
    s = configure(w)
    s.bind_torch(w.steps)
    bad = torch.tensor(w.rho, device="cuda")
    bad[1, 2, 3] = float("nan")
    s.set_design(w.design_lo, bad, w.gamma)
    with pytest.raises(L.CcprError) as e:
        s.forward(w.steps)
    assert e.value.status == L.EINVAL
    dims = w.design_dims
    n = L.edge_count(dims)
    bad_e = torch.rand(n, device="cuda")
    bad_e[n // 2] = 1.5
    s.set_design_edges(w.design_lo, dims, bad_e, w.gamma)
    with pytest.raises(L.CcprError) as e:
        s.forward(w.steps)
    assert e.value.status == L.EINVAL
    s.set_design(w.design_lo, torch.tensor(w.rho, device="cuda"), w.gamma)
    F = s.forward(w.steps)
    s.close()
    assert np.isfinite(F) and F > 0


def test_empty_and_out_of_order_calls():
    """No steps, no forward before the adjoint, no gradient before the
    adjoint: rejected with the documented codes, nothing launched."""
    require_gpu()
    from paper_2305_00234_amd import lib as L
    from paper_2305_00234_amd.solver import configure
    w = I.drude_dipole_32(steps=50)
    s = configure(w)
    s.bind_torch(w.steps)
    with pytest.raises(L.CcprError) as e:
        s.forward(0)
    assert e.value.status == L.EINVAL
    with pytest.raises(L.CcprError) as e:
        s.adjoint()
    assert e.value.status == L.ESTATE
    with pytest.raises(L.CcprError) as e:
        s.gradient()
    assert e.value.status == L.ESTATE
    s.step(0)                       # zero steps: a no-op
    assert s.step_count == 0
    F = s.forward(w.steps)
    with pytest.raises(L.CcprError) as e:
        s.gradient()
    assert e.value.status == L.ESTATE
    s.adjoint()
    g = s.gradient()
    s.close()
    assert np.isfinite(F) and np.all(np.isfinite(g))


def test_sampled_grid_pass_timing():
    """ccpr_set_timing(k): the loops are timed whole and every k-th grid pass
    is timed with events; the pass count is the sampled one and the average
    pass duration stays positive and finite."""
    require_gpu()
    from paper_2305_00234_amd.solver import configure
    w = I.drude_dipole_32(steps=100)
    s = configure(w)
    s.bind_torch(w.steps)
    s.set_timing(True, every=10)
    s.forward(w.steps)
    s.adjoint()
    ms, loops = s.timing()
    gms, passes = s.grid_timing()
    s.set_timing(True, every=1)
    s.forward(w.steps)
    gms1, passes1 = s.grid_timing()
    s.close()
    say("timing: loop ms", ms, "steps", loops, "sampled passes", passes, "all passes", passes1)
    assert loops == 2 * w.steps and passes == 2 * w.steps // 10 and passes1 == w.steps
    assert 0 < gms / passes < float("inf") and 0 < gms1 / passes1 < float("inf")


def test_timed_split_passes_give_the_same_results():
    """With timing on, a timed split grid pass uses its timing events as the
    fork and join events of its two concurrent launches: every pass timed
    gives bitwise the objective and gradient of an untimed solve (the launch
    order constraints are the same)."""
    require_gpu()
    from paper_2305_00234_amd.solver import configure
    w = I.gold_gap(n=(256, 192, 200), design=(96, 64, 48), steps=1200, seed=3, name="timed_split")

    def solve(every):
        s = configure(w)
        s.bind_torch(w.steps)
        if every:
            s.set_timing(True, every=every)
        F = s.forward(w.steps)
        s.adjoint()
        g = s.gradient()
        passes = s.grid_timing()[1] if every else 0
        s.close()
        return F, g, passes

    F0, g0, _ = solve(0)
    F1, g1, p1 = solve(1)
    say("timed split passes", p1, "F", F0, F1)
    assert p1 == 2 * w.steps
    assert F0 > 0 and F0 == F1 and np.array_equal(g0, g1)
