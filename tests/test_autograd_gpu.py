"""The differentiable objective (torch.autograd.Function rho -> F) on the GPU:
its backward (adjoint run + time-exact gradient) against the FP64 oracle's
adjoint gradient and against FP64 central finite differences of the oracle's
objective, and, at the full 512x512x256 / 8000-step time-domain size, the
invariance of F and dF/drho under the checkpoint segment length."""
import numpy as np
import pytest

from paper_2305_00234_amd import inputs as I
from tests.gpu_util import oracle_gradient, rel_l2, require_gpu, say
from tests.oracle_setup import oracle_objective

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-3
FD_H = 1e-4


def _small(objective):
    w = I.drude_dipole_32(steps=300, n=32, npml=6)
    w.shape = (30, 27, 33)
    w.mat2 = (I.GOLD_TABLE1,) * 3
    w.design_lo = (10, 9, 11)
    w.rho = np.random.default_rng(11).random((9, 8, 10)).astype(np.float32)
    w.dipole_cell = (7, 13, 15)
    w.gap_lo, w.gap_dims = (14, 12, 15), (2, 2, 2)
    w.objective = objective
    if objective == "time":
        w.window = (60, 280)
    return w


def _autograd_grad(w, rho_dtype, scale=1.0):
    torch = require_gpu()
    from paper_2305_00234_amd.autograd import objective
    from paper_2305_00234_amd.solver import configure
    s = configure(w)
    s.bind_torch(w.steps)
    rho = torch.tensor(w.rho, dtype=rho_dtype, device="cuda", requires_grad=True)
    F = objective(rho, s, w.steps, w.design_lo, w.gamma)
    (scale * F).backward()
    g = rho.grad.detach().double().cpu().numpy()
    Fv = float(F.detach())
    s.close()
    return Fv, g


@pytest.mark.parametrize("objective", ["time", "dft"])
def test_autograd_backward_matches_oracle_adjoint_and_fd(objective):
    w = _small(objective)
    say("autograd", objective, w.shape)
    Fg, gg = _autograd_grad(w, rho_dtype=__import__("torch").float64)
    Fo, go, _, _ = oracle_gradient(w)
    say("F", Fg, Fo, "grad rel L2 vs oracle adjoint", rel_l2(gg, go))
    assert abs(Fg - Fo) <= 1e-5 * abs(Fo)
    assert rel_l2(gg, go) <= GRAD_TOL
    # FP64 central finite differences of the oracle objective on 16 voxels
    rng = np.random.default_rng(100)
    flat = rng.choice(w.rho.size, size=16, replace=False)
    fd = []
    for f in flat:
        vals = []
        for sgn in (1, -1):
            wp = _small(objective)
            r = wp.rho.astype(np.float64).ravel()
            r[f] += sgn * FD_H
            wp.rho = r.reshape(w.rho.shape)
            vals.append(oracle_objective(wp))
        fd.append((vals[0] - vals[1]) / (2 * FD_H))
    fd = np.array(fd)
    sel = gg.ravel()[flat]
    say("FD vs autograd (16 voxels) rel L2", rel_l2(sel, fd))
    assert rel_l2(sel, fd) <= GRAD_TOL


def test_autograd_chain_rule_and_float32_density():
    torch = require_gpu()
    w = _small("dft")
    _, g1 = _autograd_grad(w, torch.float64)
    _, g3 = _autograd_grad(w, torch.float64, scale=3.0)
    assert np.allclose(g3, 3.0 * g1, rtol=1e-12, atol=0)
    # float32 density: the DFT gradient of this workload is representable
    _, g32 = _autograd_grad(w, torch.float32)
    assert rel_l2(g32, g1) <= 1e-6


def test_full_size_time_domain_checkpoint_invariance():
    """512x512x256 cells, 256x256x64 design, 8000 steps, time-domain objective
    over the whole run: F and dF/drho are bitwise identical with segments of
    1000 and of 2000 steps, and the gradient is finite and not zero."""
    torch = require_gpu()
    from paper_2305_00234_amd.autograd import objective
    from paper_2305_00234_amd.solver import configure
    out = []
    for every in (1000, 2000):
        w = I.gold_gap_timedomain_512(checkpoint_every=every)
        s = configure(w)
        s.bind_torch(w.steps)
        rho = torch.tensor(w.rho, dtype=torch.float64, device="cuda", requires_grad=True)
        F = objective(rho, s, w.steps, w.design_lo, w.gamma)
        F.backward()
        info = s.info()
        say("segments", info, "F", float(F.detach()))
        out.append((float(F.detach()), rho.grad.detach().cpu().numpy(), info["segments"]))
        s.close()
        del s, rho, F
        torch.cuda.empty_cache()
    (F1, g1, s1), (F2, g2, s2) = out
    assert (s1, s2) == (8, 4)
    assert F1 == F2 and F1 > 0
    assert np.array_equal(g1, g2)
    assert np.isfinite(g1).all() and np.abs(g1).max() > 0


def _recompute_case():
    """400-step Drude dipole run in 100-step segments, two resident: the
    adjoint recomputes two segments over the first resident one's history."""
    w = _small("time")
    w.steps = 400
    w.wave = I.drude_dipole_32(steps=400).wave
    w.window = (60, 380)
    return w


def test_second_adjoint_needs_a_new_forward_run():
    """After an adjoint that recomputed segments the history of the first
    resident segment is gone: a second adjoint is refused (CCPR_ESTATE) and
    the forward serial reads -1; a new forward run restores it, and the
    gradient is then bitwise the first one."""
    require_gpu()
    from paper_2305_00234_amd import lib as L
    from paper_2305_00234_amd.solver import configure
    w = _recompute_case()
    s = configure(w)
    s.set_checkpointing(100)
    s.set_resident_segments(2)
    s.bind_torch(w.steps)
    s.forward(w.steps)
    serial = s.forward_serial
    assert serial >= 1 and s.info()["segments"] == 4 and s.info()["resident_segments"] == 2
    s.adjoint()
    g1 = s.gradient()
    assert s.forward_serial == -1
    with pytest.raises(L.CcprError) as e:
        s.adjoint()
    assert e.value.status == L.ESTATE
    s.forward(w.steps)
    assert s.forward_serial == serial + 1
    s.adjoint()
    g2 = s.gradient()
    s.close()
    assert np.array_equal(g1, g2)


def test_autograd_retain_graph_and_shared_solver():
    """backward(retain_graph=True) twice on a recomputing layout gives the
    same gradient bitwise (the second backward runs its forward again), and
    two objectives evaluated on one solver before a joint backward each get
    their own gradient (the earlier node re-runs its forward)."""
    torch = require_gpu()
    from paper_2305_00234_amd.autograd import objective
    from paper_2305_00234_amd.solver import configure
    w = _recompute_case()
    s = configure(w)
    s.set_checkpointing(100)
    s.set_resident_segments(2)
    s.bind_torch(w.steps)
    rho = torch.tensor(w.rho, dtype=torch.float64, device="cuda", requires_grad=True)
    F = objective(rho, s, w.steps, w.design_lo, w.gamma)
    F.backward(retain_graph=True)
    g1 = rho.grad.detach().clone()
    rho.grad = None
    F.backward()
    g2 = rho.grad.detach().clone()
    assert torch.equal(g1, g2)
    # two densities through one solver, one backward
    rho_b = (0.5 * rho.detach()).clone().requires_grad_(True)
    ra = rho.detach().clone().requires_grad_(True)
    Fa = objective(ra, s, w.steps, w.design_lo, w.gamma)
    Fb = objective(rho_b, s, w.steps, w.design_lo, w.gamma)
    (Fa + Fb).backward()
    Fb_alone = objective(rho_b.detach().clone().requires_grad_(True), s, w.steps, w.design_lo, w.gamma)
    s.close()
    assert torch.equal(ra.grad, g1)
    assert float(Fb_alone.detach()) == float(Fb.detach())
    assert float(Fa.detach()) == float(F.detach())
    say("shared solver: grad a == single backward; F_b", float(Fb.detach()))


def test_objective_on_another_torch_stream():
    """The workspace is bound with torch's default stream; the density is
    produced and the objective differentiated under another torch stream.
    The binding orders the library's stream after the caller's and the
    caller's after the library's: F and the gradient equal those of the
    default-stream run bitwise."""
    torch = require_gpu()
    from paper_2305_00234_amd.autograd import objective
    from paper_2305_00234_amd.solver import configure
    w = _small("dft")
    s = configure(w)
    s.bind_torch(w.steps)
    base = torch.tensor(w.rho, dtype=torch.float64, device="cuda")
    r0 = base.clone().requires_grad_(True)
    F0 = objective(r0, s, w.steps, w.design_lo, w.gamma)
    F0.backward()
    g0 = r0.grad.detach().clone()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        # a density computed on the side stream just before the call
        r1 = (base * 2.0 - base).requires_grad_(True)
        F1 = objective(r1, s, w.steps, w.design_lo, w.gamma)
        F1.backward()
        g1 = (r1.grad * 1.0)      # consumed on the side stream
    torch.cuda.synchronize()
    s.close()
    assert float(F1.detach()) == float(F0.detach())
    assert torch.equal(g1, g0)
