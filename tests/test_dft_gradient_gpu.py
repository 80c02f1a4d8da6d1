"""DFT-mode gradient (on-the-fly DFT correlation for the single-frequency
objective) on the GPU, through the C-ABI: same-estimator parity with the FP64
oracle (objective 1e-5, gradient 1e-3 relative L2), convergence to the
time-exact gradient on the GPU path itself, the autograd backward in DFT mode,
the smaller workspace, and the rejection of a time-domain objective."""
import math

import numpy as np
import pytest

from paper_2305_00234_amd import inputs as I
from tests.gpu_util import gpu_gradient, oracle_gradient, rel_l2, require_gpu, say

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-5
GRAD_TOL = 1e-3


def _short_pulse_dipole(M, n=24, npml=5, lam=500e-9):
    w = I.drude_dipole_32(steps=M, n=n, npml=npml)
    t = (np.arange(M) + 0.5) * w.dt
    w.wave = I.gaussian_sine(t, lam, 2e-15, 4e-15)
    w.omega = 2 * math.pi * I.C0 / lam
    w.gradient = "dft"
    return w


def test_dft_mode_matches_oracle_estimator_dipole():
    """Drude design, 2 fs dipole pulse, 3000 steps: the run is long enough
    for a meaningful estimate but not for convergence, so the estimator
    itself (forward transform, fit window, combination) is what is compared."""
    w = _short_pulse_dipole(3000)
    Fg, gg, _, _, info = gpu_gradient(w)
    Fo, go, _, _ = oracle_gradient(w)
    say("DFT mode dipole: F", Fg, Fo, "grad rel L2", rel_l2(gg, go), "info", info)
    assert info["segments"] == 1
    assert abs(Fg - Fo) <= FIELD_TOL * abs(Fo)
    assert rel_l2(gg, go) <= GRAD_TOL


def test_dft_mode_matches_oracle_estimator_planewave_gold():
    """TF/SF plane wave on a Table-1 gold design with the conductivity
    damping, ragged tiles, 6-cell CPML."""
    w = I.gold_gap(n=(64, 44, 48), design=(24, 20, 12), gap=2, npml=6, steps=900, seed=5,
                   name="pw_dft")
    t = np.arange(w.steps + 1) * w.dt
    w.wave = I.gaussian_sine(t, 300e-9, 0.6e-15, 1.0e-15)
    w.omega = 2 * math.pi * I.C0 / 300e-9
    w.gradient = "dft"
    Fg, gg, _, _, _ = gpu_gradient(w)
    Fo, go, _, _ = oracle_gradient(w)
    say("DFT mode plane wave: F", Fg, Fo, "grad rel L2", rel_l2(gg, go))
    assert abs(Fg - Fo) <= FIELD_TOL * abs(Fo)
    assert rel_l2(gg, go) <= GRAD_TOL


def test_dft_mode_tends_to_time_exact_on_gpu():
    """On the GPU path alone: with the pulse gone, the DFT-mode gradient of a
    long run agrees with the time-exact one."""
    w = _short_pulse_dipole(8000)
    Fd, gd, _, _, _ = gpu_gradient(w)
    w.gradient = "time"
    Ft, gt, _, _, _ = gpu_gradient(w)
    say("GPU DFT mode vs time-exact, 8000 steps: rel L2", rel_l2(gd, gt))
    assert Fd == Ft
    assert rel_l2(gd, gt) <= GRAD_TOL


def test_dft_mode_autograd_backward():
    """torch.autograd.Function rho -> F with the DFT-mode backward against the
    oracle's estimator."""
    torch = require_gpu()
    from paper_2305_00234_amd.autograd import objective
    from paper_2305_00234_amd.solver import configure
    w = _short_pulse_dipole(3000)
    s = configure(w)
    s.bind_torch(w.steps)
    rho = torch.tensor(w.rho, dtype=torch.float64, device="cuda", requires_grad=True)
    F = objective(rho, s, w.steps, w.design_lo, w.gamma)
    F.backward()
    g = rho.grad.detach().cpu().numpy()
    Fv = float(F.detach())
    s.close()
    Fo, go, _, _ = oracle_gradient(w)
    say("autograd DFT mode: F", Fv, Fo, "grad rel L2", rel_l2(g, go))
    assert abs(Fv - Fo) <= FIELD_TOL * abs(Fo)
    assert rel_l2(g, go) <= GRAD_TOL


def test_dft_mode_workspace_and_time_objective_rejected():
    require_gpu()
    from paper_2305_00234_amd.lib import CcprError, EINVAL
    from paper_2305_00234_amd.solver import configure
    w = _short_pulse_dipole(2000)
    s = configure(w)
    b_dft = s.workspace_size(w.steps)
    s.set_gradient_mode("time")
    b_time = s.workspace_size(w.steps)
    say("workspace bytes DFT / time-exact", b_dft, b_time)
    assert b_dft < b_time
    s.close()
    w.objective = "time"
    s = configure(w)
    s.bind_torch(w.steps)
    with pytest.raises(CcprError) as ei:
        s.forward(w.steps)
    assert ei.value.status == EINVAL
    s.close()
